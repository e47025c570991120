// Batched PDHCG: many independent linear Fisher markets in one persistent
// launch.  Each workgroup takes work from a queue (largest markets first)
// and runs the whole restarted PDHCG solve of a market: price step (eq.
// update:py), row prox (Sec. 2.2), running averages (Alg. 2), column sums,
// the adaptive step rule, the relative KKT check, restarts and primal
// weight (Sec. 5).  Each market converges (and retires) on its own: the
// per-market convergence mask is the work queue.  A single market's solve
// synchronises with workgroup barriers only; the largest markets are split
// over gangs of workgroups that also meet at a counter of their own (see
// the gang notes below), so that no market outlasts the mean load of a
// workgroup by much.
//
// The control logic follows the same readings as the single-market host
// loop (pdhcg_api.hip), executed by thread 0 between barriers.
#include "../../include/pdhcg.h"
#include "pdhcg_device.h"
#include "pdhcg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

namespace pdhcg {

constexpr int kBatchBlock = 512;
constexpr int kBatchWaves = kBatchBlock / kWave;
constexpr int kBatchMaxGoods = 2048;
constexpr int kEvalUnroll = 4;  // entries per lane loaded together in the KKT passes

struct BatchParamsDev {
  double tol;
  int64_t max_iter;
  int32_t eval_every, max_rounds, step_mode, restart;
  double rtol, beta_suff, beta_nec, beta_art, theta, omega_bound, eta0, omega0;
  int32_t omega_check_every, output;
};

struct BatchInfoDev {
  double kkt[3];
  double rel_kkt, eta, omega;
  int64_t iters, accepted;
  int32_t restarts, status, evals, pad;
  int64_t ticks;  // the market's solve time in device wall-clock ticks
};

// Per-solve arguments, read by the kernel from device memory (so that one
// graph of the solve serves every call): parameters and the caller's
// outputs (null outputs are not written, as in the tuning runs).
struct BatchArgs {
  BatchParamsDev prm;
  float *p_out, *x_out;
};

struct BatchDev {
  int32_t count;
  const int32_t *order, *n, *m, *shape;
  const int64_t *rp_off, *row_off, *good_off, *edge_off;
  const double *sumw;
  const int32_t *row_ptr, *col, *deg;
  const float *uh, *w, *rowmax;
  float *X0, *X1, *X2, *XA;
  double *P0, *P1, *P2, *PA, *C0, *C1, *C2;
  BatchInfoDev *info;
  uint32_t *queue;
  // Work tickets of the solve, in queue order: {market, member, gang size,
  // gang index}.  A market of gang size G > 1 has G consecutive tickets;
  // gang g exchanges partial sums through gang_buf + gang_off[g] and meets
  // at the barrier counter gang_cnt[g].
  const int4 *tickets;
  int32_t ntickets, ngangs;
  uint32_t *gang_cnt;
  const int64_t *gang_off;
  double *gang_buf;
};

// Pointers of one market.  Role buffers are selected with pick3 (no
// dynamically indexed arrays, which would live in scratch memory).
struct MView {
  int n, m;
  int r0, r1;  // rows of this workgroup: all of them, or a gang member's share
  const int32_t *rp, *col, *deg;
  const float *uh, *w, *rowmax;
  float *X0, *X1, *X2, *XA;
  double *P0, *P1, *P2, *PA, *C0, *C1, *C2;
  __device__ float *X(int i) const { return pick3<float *>(X0, X1, X2, i); }
  __device__ double *P(int i) const { return pick3<double *>(P0, P1, P2, i); }
  __device__ double *C(int i) const { return pick3<double *>(C0, C1, C2, i); }
};

struct WGState {
  int gG, gr, gi, r0, r1, nbar, nx, dead;  // gang size, member, index; rows; barriers, exchanges
  int ix[3], ip[3], ic[3];
  int fold, done, status, restarts, evals, cand_avg, do_restart, market;
  int64_t total, since, k_in, accepted, t0;
  double eta, omega, eta0, omega0, tau, sigma, kkt0, kkt_prev, kbest;
  double kout[3];
  double kc[3], ka[3];
};

// Values every lane holds alike (read from LDS after a barrier): move them
// to scalar registers so that pointers derived from them stay scalar.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ double uni(double x) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  v = wave_sum_d(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < kBatchWaves; ++q) t += red[q];
  __syncthreads();
  return t;
}

__device__ __forceinline__ double block_max(double v, double *red) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  v = wave_max_d(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = red[0];
  for (int q = 1; q < kBatchWaves; ++q) t = fmax(t, red[q]);
  __syncthreads();
  return t;
}

// One trial step's row pass over the market for shape (G, E): x_try,
// lagged fold of x_cur into x_avg, |x_try - x_cur|^2 (returned, this
// thread's share) and float64 column sums into lc.
template <int G, int E>
__device__ __attribute__((noinline)) double wg_rows_step(const MView &v, const double *lp, double *lc, const float *xin,
                               float *xout, float *xavg, double tau, float wfold, int max_rounds,
                               double rtol) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane & (G - 1), seg = lane / G;
  constexpr int kSeg = kWave / G;
  constexpr int kStride = kBatchWaves * kSeg;  // rows per workgroup pass
  const bool fold_read = wfold != 0.0f && wfold != 1.0f;
  double dx2 = 0.0;
  auto pget = [&](int c) { return lp[c]; };
  // rows beyond the register capacity (only G = 64): whole-wave path
  auto long_row = [&](int beg, int d, double tw) {
    int rounds = 0;
    const double sfin =
        prox_row_long(beg, d, tau, tw, v.uh, v.col, xin, pget, max_rounds, rtol, rounds);
    const double tf = tw * fast_rcp(sfin);
    // final sweep in chunks, every load of a chunk issued first
    for (int base2 = 0; base2 < d; base2 += kWave * kLongUnroll) {
      float uu[kLongUnroll], xk[kLongUnroll], y[kLongUnroll];
      int c[kLongUnroll];
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int q = beg + min(base2 + lane + kWave * e, d - 1);
        uu[e] = v.uh[q];
        c[e] = v.col[q];
        xk[e] = xin[q];
        y[e] = fold_read ? xavg[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int k = base2 + lane + kWave * e;
        if (k < d) {
          const int q = beg + k;
          const double a = fma(-tau, lp[c[e]], (double)xk[e]);
          const float xn = (float)fmax(fma((double)uu[e], tf, a), 0.0);
          xout[q] = xn;
          if (wfold != 0.0f) xavg[q] = fold_read ? fmaf(xk[e] - y[e], wfold, y[e]) : xk[e];
          dx2 += (double)(xn - xk[e]) * (double)(xn - xk[e]);
          atomicAdd(&lc[c[e]], (double)xn);
        }
      }
    }
  };
  // Register path, NP workgroup passes per trip (two when the registers
  // allow it): the entries and averaged allocations of the passes are loaded
  // before any is solved, so each wave keeps NP passes of reads in flight.
  // Loads use indices clamped into the row (every slot loads; slots past the
  // row end are masked).
  constexpr int NP = E <= 4 ? 2 : 1;
  for (int base = v.r0 + wave * kSeg; base < v.r1; base += NP * kStride) {
    int beg[NP], d[NP];
    double tw[NP];
    bool rv[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      const int i = base + h * kStride + seg;
      rv[h] = i < v.r1;
      beg[h] = rv[h] ? v.rp[i] : 0;
      d[h] = rv[h] ? v.rp[i + 1] - beg[h] : 0;
      tw[h] = rv[h] ? tau * (double)v.w[i] : 0.0;
    }
    float uh[NP][E], xk[NP][E], y[NP][E];
    int cj[NP][E];
    bool ok[NP][E];
#pragma unroll
    for (int h = 0; h < NP; ++h)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = r + G * e;
        ok[h][e] = idx < d[h];
        const int q = beg[h] + (ok[h][e] ? idx : 0);  // row start: in bounds (nnz >= 1)
        uh[h][e] = v.uh[q];
        xk[h][e] = xin[q];
        cj[h][e] = v.col[q];
        y[h][e] = fold_read ? xavg[q] : 0.0f;
      }
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      if (G == kWave && E * G < d[h]) {
        long_row(beg[h], d[h], tw[h]);
        continue;
      }
      double a[E];
      float u[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        u[e] = ok[h][e] ? uh[h][e] : 0.0f;
        a[e] = fma(-tau, lp[cj[h][e]], (double)xk[h][e]);  // x^k - tau p
      }
      int rounds = 0;
      const double sfin =
          prox_solve<G, E, 0>(rv[h], tw[h], max_rounds, rtol, 0, ok[h], a, u, xk[h], rounds);
      const double tf = tw[h] * fast_rcp(sfin);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (ok[h][e]) {
          const int q = beg[h] + r + G * e;
          const float xn = (float)fmax(fma((double)u[e], tf, a[e]), 0.0);
          xout[q] = xn;
          if (wfold != 0.0f)
            xavg[q] = fold_read ? fmaf(xk[h][e] - y[h][e], wfold, y[h][e]) : xk[h][e];
          const double df = (double)xn - (double)xk[h][e];
          dx2 = fma(df, df, dx2);
          atomicAdd(&lc[cj[h][e]], (double)xn);
        }
      }
    }
  }
  return dx2;
}

// KKT row pass (Sec. 5 Criteria) over the current point and, if xa is not
// NULL, the averaged point (folded in place with weight wf).  G lanes per
// row, entries visited with stride G.  Row statistics go to st[0..9]
// (same layout as the single-market KKT pass); column maxima of u y - p go
// to lMc/lMa (ord_key keys), column sums of the averaged point (or of the
// current point when sum_cur) to lcs.
template <int G>
__device__ __attribute__((noinline)) void wg_rows_eval(const MView &v, const float *xc, const double *pc, float *xa,
                             const double *pa_folded, float wf, const float *xanc, bool sum_cur,
                             unsigned int *lMc, unsigned int *lMa, double *lcs, double *st,
                             float *tc_out, float *ta_out) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane & (G - 1), seg = lane / G;
  constexpr int kSeg = kWave / G;
  const bool has_avg = xa != nullptr;
  for (int base = v.r0 + wave * kSeg; base < v.r1; base += kBatchWaves * kSeg) {
    const int i = base + seg;
    const bool rv = i < v.r1;
    const int beg = rv ? v.rp[i] : 0;
    const int d = rv ? v.rp[i + 1] - beg : 0;
    // entries in chunks of G * kEvalUnroll per segment, every load of a
    // chunk issued before any is used (indices past the row end clamped to
    // its last entry and skipped)
    constexpr int U = kEvalUnroll;
    double tc = 0.0, ta = 0.0;
    for (int k0 = r; k0 < d; k0 += G * U) {
      float x[U], uu[U], y[U], z[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int q = beg + min(k0 + G * e, d - 1);
        x[e] = xc[q];
        uu[e] = v.uh[q];
        y[e] = has_avg ? xa[q] : 0.0f;
        z[e] = xanc ? xanc[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int k = k0 + G * e;
        if (k < d) {
          tc = fma((double)uu[e], (double)x[e], tc);
          if (has_avg) {
            float yy = y[e];
            if (wf != 0.0f) {
              yy = (wf == 1.0f) ? x[e] : fmaf(x[e] - yy, wf, yy);
              xa[beg + k] = yy;
            }
            ta = fma((double)uu[e], (double)yy, ta);
            if (xanc) st[9] += ((double)yy - (double)z[e]) * ((double)yy - (double)z[e]);
          }
          if (xanc) st[8] += ((double)x[e] - (double)z[e]) * ((double)x[e] - (double)z[e]);
        }
      }
    }
    tc = seg_sum_d<G>(tc);
    ta = seg_sum_d<G>(ta);
    if (!rv) continue;
    const double wi = v.w[i];
    const double yc = wi / tc, ya = has_avg ? wi / ta : 0.0;
    if (r == 0) {
      st[0] = fmax(st[0], yc);
      if (has_avg) st[4] = fmax(st[4], ya);
      if (tc_out) tc_out[i] = (float)(tc * (double)v.rowmax[i]);
      if (ta_out && has_avg) ta_out[i] = (float)(ta * (double)v.rowmax[i]);
    }
    for (int k0 = r; k0 < d; k0 += G * U) {
      int c[U];
      float uu[U], x[U], y[U];
      double pcj[U], paj[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int q = beg + min(k0 + G * e, d - 1);
        c[e] = v.col[q];
        uu[e] = v.uh[q];
        x[e] = xc[q];
        y[e] = has_avg ? xa[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        pcj[e] = pc[c[e]];
        paj[e] = has_avg ? pa_folded[c[e]] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < U; ++e) {
        if (k0 + G * e < d) {
          const double u = uu[e];
          const double vc = u * yc, rc = pcj[e] - vc;
          if (rc > 0.0) {
            st[2] = fmax(st[2], rc);
            st[1] = fmax(st[1], (double)x[e] * rc);
          }
          st[3] = fmax(st[3], (double)x[e]);
          atomicMax(&lMc[c[e]], ord_key((float)(vc - pcj[e])));
          if (has_avg) {
            const double va = u * ya, ra = paj[e] - va;
            if (ra > 0.0) {
              st[6] = fmax(st[6], ra);
              st[5] = fmax(st[5], (double)y[e] * ra);
            }
            st[7] = fmax(st[7], (double)y[e]);
            atomicMax(&lMa[c[e]], ord_key((float)(va - paj[e])));
            if (!sum_cur) atomicAdd(&lcs[c[e]], (double)y[e]);
          }
          if (sum_cur) atomicAdd(&lcs[c[e]], (double)x[e]);
        }
      }
    }
  }
}

template <int G>
__device__ void wg_colsum_x(const MView &v, const float *x, double *lc) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane & (G - 1), seg = lane / G;
  constexpr int kSeg = kWave / G;
  for (int base = v.r0 + wave * kSeg; base < v.r1; base += kBatchWaves * kSeg) {
    const int i = base + seg;
    if (i >= v.r1) continue;
    for (int k = v.rp[i] + r; k < v.rp[i + 1]; k += G) atomicAdd(&lc[v.col[k]], (double)x[k]);
  }
}

struct EvalOut {
  double kc[3], ka[3], dxa2[2], dpa2[2];
};

// ---------------------------------------------------------------- gangs --
//
// A large market may be split over a gang of G workgroups (consecutive
// tickets of the queue, taken before any single market).  Member r owns the
// rows [r0, r1) holding about nnz r / G .. nnz (r + 1) / G entries and
// their allocations; every member keeps all prices and column sums of the
// market in LDS and makes the same control decisions from the same reduced
// numbers.  Per iteration the members meet once: each writes its column
// partials and its share of |dx|^2 to a slot of the gang's exchange area and
// arrives at the gang's counter; after the last arrival every member sums
// the slots in member order, so all hold bitwise the same column sums.  A
// KKT check adds a second meeting (row statistics, column maxima and sums of
// the averaged point) and a restart a third (so that no member overwrites
// the anchors while another still reads them).
//
// Arrays of the goods are written as follows: values every member computes
// alike (trial prices, column sums, anchors) are written by every member
// for all goods (the same bits, so the order does not matter); the running
// average of the prices, updated in place, is written only by the member
// that owns the good's range [m r / G, m (r + 1) / G).  Iteration slots
// alternate between two buffers, so a member that starts the next iteration
// early never overwrites slots another member still reads.
//
// The gangs' members are resident together (the grid never exceeds the
// resident workgroups and the gangs' tickets come first, at most one per
// workgroup), so every wait ends.  A wait longer than kGangSpinTicks marks
// the market PDHCG_ERR_HIP and its members stop meeting.

constexpr uint64_t kGangSpinTicks = 2000000000ull;  // 20 s at the 100 MHz wall clock

// Exchange area of a gang of G members for a market of m goods (doubles).
__host__ __device__ inline int64_t gang_area(int G, int m) { return 4 * (int64_t)G * m + 12 * (int64_t)G; }

struct GangView {
  int G, r, m;
  uint32_t *cnt;
  double *base;
  __device__ double *cslot(int par) const { return base + (int64_t)par * G * m; }   // [2][G][m]
  __device__ double *dxslot(int par) const { return base + 2 * (int64_t)G * m + par * G; }  // [2][G]
  __device__ double *stslot() const { return base + 2 * (int64_t)G * m + 2 * G; }  // [G][10]
  __device__ double *csslot() const { return stslot() + 10 * G; }                    // [G][m]
  __device__ unsigned int *mcslot() const {
    return reinterpret_cast<unsigned int *>(csslot() + (int64_t)G * m);  // [G][m]
  }
  __device__ unsigned int *maslot() const { return mcslot() + (int64_t)G * m; }  // [G][m]
};

// Every member of the gang arrives here before any leaves.  Stores made
// before the meeting by any member are visible to loads after it.
__device__ void gang_sync(const GangView &g, WGState &S) {
  __syncthreads();
  if (threadIdx.x == 0 && !S.dead) {
    __threadfence();  // release this workgroup's stores to the whole device
    S.nbar += 1;
    const uint32_t target = (uint32_t)S.nbar * (uint32_t)g.G;
    __hip_atomic_fetch_add(g.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(g.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > kGangSpinTicks) {
        S.dead = 1;
        break;
      }
    }
    __threadfence();  // acquire the other members' stores
  }
  __syncthreads();
}

// Column sums of the whole market in lc from every member's partials, and
// the total of the members' shares `part` (same bits in every member).
__device__ double gang_colsum(const GangView &g, WGState &S, double *lc, double part) {
  if (g.G == 1) return part;
  const int par = uni(S.nx) & 1;
  double *cs = g.cslot(par);
  double *dxs = g.dxslot(par);
  for (int j = threadIdx.x; j < g.m; j += blockDim.x) cs[(int64_t)g.r * g.m + j] = lc[j];
  if (threadIdx.x == 0) dxs[g.r] = part;
  gang_sync(g, S);  // every thread has read S.nx above
  if (S.dead) return part;
  for (int j = threadIdx.x; j < g.m; j += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < g.G; ++q) t += cs[(int64_t)q * g.m + j];
    lc[j] = t;
  }
  double t = 0.0;
  for (int q = 0; q < g.G; ++q) t += dxs[q];
  if (threadIdx.x == 0) S.nx += 1;
  __syncthreads();
  return t;
}

// Take the next ticket of the queue into S (market -1 when none is left);
// every thread returns the market.
__device__ int take_ticket(const BatchDev &bd, WGState &S) {
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(bd.queue, 1u);
    if (t < (uint32_t)bd.ntickets) {
      const int4 tk = bd.tickets[t];
      S.market = tk.x;
      S.gr = tk.y;
      S.gG = tk.z;
      S.gi = tk.w;
    } else {
      S.market = -1;
    }
  }
  __syncthreads();
  return uni(S.market);
}

// The gang of the ticket in S, and this member's rows: the first row at or
// after nnz r / G up to the first at or after nnz (r + 1) / G (a lower
// bound on the row pointer).  Resets the gang's meeting counts.
__device__ GangView member_rows(const BatchDev &bd, MView &v, WGState &S) {
  GangView g;
  g.G = uni(S.gG);
  g.r = uni(S.gr);
  g.m = v.m;
  g.cnt = g.G > 1 ? bd.gang_cnt + uni(S.gi) : nullptr;
  g.base = g.G > 1 ? bd.gang_buf + bd.gang_off[uni(S.gi)] : nullptr;
  if (threadIdx.x == 0) {
    const int nnz = v.rp[v.n];
    auto first_row = [&](int r) {
      if (r >= g.G) return v.n;
      const int64_t target = (int64_t)nnz * r / g.G;
      int lo = 0, hi = v.n;
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if ((int64_t)v.rp[mid] < target) lo = mid + 1;
        else hi = mid;
      }
      return lo;
    };
    S.r0 = first_row(g.r);
    S.r1 = first_row(g.r + 1);
    S.nbar = 0;
    S.nx = 0;
    S.dead = 0;
  }
  __syncthreads();
  v.r0 = uni(S.r0);
  v.r1 = uni(S.r1);
  return g;
}

// Full KKT check of the current point (and the average when has_avg) of
// one market; returns the residuals in `out` (valid in thread 0).  In a
// gang the rows are this member's and the row statistics, column maxima and
// column sums are combined over the members before the column pass.
__device__ void wg_eval(const MView &v, const GangView &g, int shape, WGState &S, bool has_avg,
                        float wf, double *lp, double *lc, unsigned int *lMc, unsigned int *lMa,
                        double *red10, double *tot10, EvalOut &out) {
  const float *xc = v.X(uni(S.ix[0]));
  const double *pc = v.P(uni(S.ip[0]));
  float *xa = has_avg ? v.X(uni(S.ix[2])) : nullptr;
  double *pa = v.P(uni(S.ip[2]));
  for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
    lMc[j] = 0u;
    lMa[j] = 0u;
    lc[j] = 0.0;
    if (has_avg) {
      double q = pa[j];
      if (wf != 0.0f) q = (wf == 1.0f) ? pc[j] : q + (pc[j] - q) * (double)wf;
      lp[j] = q;
      if (g.G == 1) pa[j] = q;
    }
  }
  __syncthreads();
  double st[10];
  for (int q = 0; q < 10; ++q) st[q] = 0.0;
  switch (shape) {
    case 0: wg_rows_eval<8>(v, xc, pc, xa, lp, wf, v.XA, false, lMc, lMa, lc, st, nullptr, nullptr); break;
    case 1: wg_rows_eval<16>(v, xc, pc, xa, lp, wf, v.XA, false, lMc, lMa, lc, st, nullptr, nullptr); break;
    case 2: wg_rows_eval<32>(v, xc, pc, xa, lp, wf, v.XA, false, lMc, lMa, lc, st, nullptr, nullptr); break;
    default: wg_rows_eval<64>(v, xc, pc, xa, lp, wf, v.XA, false, lMc, lMa, lc, st, nullptr, nullptr); break;
  }
  // wave-level reduction of the row statistics, combined by one thread
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const double x = (q >= 8) ? wave_sum_d(st[q]) : wave_max_d(st[q]);
    if (lane == 0) red10[wave * 10 + q] = x;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int q = threadIdx.x;
    double x = red10[q];
    for (int w = 1; w < kBatchWaves; ++w) x = (q >= 8) ? x + red10[w * 10 + q] : fmax(x, red10[w * 10 + q]);
    tot10[q] = x;
  }
  __syncthreads();
  if (g.G > 1) {
    double *sts = g.stslot(), *css = g.csslot();
    unsigned int *mcs = g.mcslot(), *mas = g.maslot();
    const int64_t o = (int64_t)g.r * v.m;
    for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
      css[o + j] = lc[j];
      mcs[o + j] = lMc[j];
      mas[o + j] = lMa[j];
    }
    if (threadIdx.x < 10) sts[g.r * 10 + threadIdx.x] = tot10[threadIdx.x];
    gang_sync(g, S);
    if (S.dead) return;
    for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
      double c = 0.0;
      unsigned int a = 0u, z = 0u;
      for (int q = 0; q < g.G; ++q) {
        const int64_t oq = (int64_t)q * v.m + j;
        c += css[oq];
        a = max(a, mcs[oq]);
        z = max(z, mas[oq]);
      }
      lc[j] = c;
      lMc[j] = a;
      lMa[j] = z;
      if (has_avg) pa[j] = lp[j];  // every member reads pa before the meeting
    }
    if (threadIdx.x < 10) {
      const int q = threadIdx.x;
      double x = sts[q];
      for (int w = 1; w < g.G; ++w) x = (q >= 8) ? x + sts[w * 10 + q] : fmax(x, sts[w * 10 + q]);
      tot10[q] = x;
    }
    __syncthreads();
  }
  double cs[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) cs[q] = (q == 3 || q == 7 || q == 2 || q == 6) ? -INFINITY : 0.0;
  const double *cc = v.C(uni(S.ic[1]));
  double *cavg = v.C(uni(S.ic[2]));
  for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
    const double Dc = ord_dec(lMc[j]);  // column max of u y - p
    const double p = pc[j];
    cs[0] = fmax(cs[0], fabs(cc[j] - 1.0));
    cs[1] = fmax(cs[1], fabs(cc[j]));
    cs[2] = fmax(cs[2], Dc);
    cs[3] = fmax(cs[3], -Dc);
    cs[8] += (p - v.PA[j]) * (p - v.PA[j]);
    if (has_avg) {
      const double Da = ord_dec(lMa[j]);
      const double ca = lc[j];
      const double q = lp[j];
      cavg[j] = ca;
      cs[4] = fmax(cs[4], fabs(ca - 1.0));
      cs[5] = fmax(cs[5], fabs(ca));
      cs[6] = fmax(cs[6], Da);
      cs[7] = fmax(cs[7], -Da);
      cs[9] += (q - v.PA[j]) * (q - v.PA[j]);
    }
  }
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const double x = (q >= 8) ? wave_sum_d(cs[q]) : wave_max_d(cs[q]);
    if (lane == 0) red10[wave * 10 + q] = x;
  }
  __syncthreads();
  if (threadIdx.x < 10) {
    const int q = threadIdx.x;
    double x = red10[q];
    for (int w = 1; w < kBatchWaves; ++w) x = (q >= 8) ? x + red10[w * 10 + q] : fmax(x, red10[w * 10 + q]);
    tot10[10 + q] = x;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double *rw = tot10, *c = tot10 + 10;
  // relative KKT error (Sec. 5 Criteria) with t = Ux, y = w/t
  for (int z = 0; z < 2; ++z) {
    const int o = 4 * z;
    double *k = z == 0 ? out.kc : out.ka;
    k[0] = c[o + 0] / (1.0 + fmax(c[o + 1], 1.0));
    k[1] = fmax(0.0, c[o + 2]) / (1.0 + fmax(rw[o + 0], c[o + 3]));
    k[2] = rw[o + 1] / (1.0 + fmax(rw[o + 3], rw[o + 2]));
  }
  out.dxa2[0] = rw[8];
  out.dxa2[1] = rw[9];
  out.dpa2[0] = c[8];
  out.dpa2[1] = c[9];
}

// Clears the work queue and the gangs' barrier counters (a kernel, not a
// memset, so that the solve graph holds kernel nodes only).
__global__ void k_batch_reset(uint32_t *queue, uint32_t *gang_cnt, int ngangs) {
  if (threadIdx.x == 0) *queue = 0u;
  for (int g = threadIdx.x; g < ngangs; g += blockDim.x) gang_cnt[g] = 0u;
}

__global__ __launch_bounds__(kBatchBlock) void k_batch_solve(BatchDev bd, const BatchArgs *args) {
  const BatchParamsDev prm = args->prm;
  float *const p_out = args->p_out;
  float *const x_out = args->x_out;
  __shared__ double lp[kBatchMaxGoods];
  __shared__ double lc[kBatchMaxGoods];
  // price changes of the trial step; during a KKT check the column maxima
  // of the current and the averaged point (two key arrays)
  __shared__ double lx[kBatchMaxGoods];
  unsigned int *const lMc = reinterpret_cast<unsigned int *>(lx);
  unsigned int *const lMa = lMc + kBatchMaxGoods;
  __shared__ double red[kBatchWaves];
  __shared__ double red10[kBatchWaves * 10];
  __shared__ double tot10[20];
  __shared__ WGState S;
  __shared__ EvalOut E;

  while (true) {
    const int b = take_ticket(bd, S);
    if (b < 0) return;
    MView v;
    v.n = bd.n[b];
    v.m = bd.m[b];
    const int64_t ro = bd.row_off[b], go = bd.good_off[b], eo = bd.edge_off[b];
    v.rp = bd.row_ptr + bd.rp_off[b];
    v.col = bd.col + eo;
    v.deg = bd.deg + go;
    v.uh = bd.uh + eo;
    v.w = bd.w + ro;
    v.rowmax = bd.rowmax + ro;
    v.X0 = bd.X0 + eo; v.X1 = bd.X1 + eo; v.X2 = bd.X2 + eo; v.XA = bd.XA + eo;
    v.P0 = bd.P0 + go; v.P1 = bd.P1 + go; v.P2 = bd.P2 + go; v.PA = bd.PA + go;
    v.C0 = bd.C0 + go; v.C1 = bd.C1 + go; v.C2 = bd.C2 + go;
    const int shape = uni(bd.shape[b]);
    const GangView g = member_rows(bd, v, S);
    const int e0 = v.rp[v.r0], e1 = v.rp[v.r1];
    // goods whose running price average this member updates
    const int g0 = (int)((int64_t)v.m * g.r / g.G), g1 = (int)((int64_t)v.m * (g.r + 1) / g.G);

    // Initial point (x0 = 1/deg_j, p0 = sum(w)/m), its column sums and KKT.
    const double p0 = bd.sumw[b] / (double)v.m;
    for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x) {
      const float x0 = 1.0f / (float)v.deg[v.col[k]];
      v.X(0)[k] = x0;
      v.XA[k] = x0;
    }
    for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
      v.P(0)[j] = p0;
      v.PA[j] = p0;
      lc[j] = 0.0;
    }
    if (threadIdx.x == 0) {
      S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
      S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
      S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
      S.fold = 0; S.done = 0; S.status = PDHCG_MAX_ITER; S.restarts = 0; S.evals = 0;
      S.cand_avg = 0; S.do_restart = 0;
      S.t0 = (int64_t)wall_clock64();
      S.total = 0; S.since = 0; S.k_in = 0; S.accepted = 0;
      const bool adaptive = prm.step_mode == 1;
      double kmax = 0.0;
      for (int j = 0; j < v.m; ++j) kmax = fmax(kmax, (double)v.deg[j]);
      S.eta0 = prm.eta0 > 0.0 ? prm.eta0 : (adaptive ? 1.0 : 0.9 / sqrt(kmax));
      S.omega0 = prm.omega0 > 0.0 ? prm.omega0 : 0.05 * bd.sumw[b] / (double)v.m;
      S.eta = S.eta0;
      S.omega = S.omega0;
      S.tau = S.eta / S.omega;
      S.sigma = S.eta * S.omega;
      S.kkt_prev = INFINITY;
      S.kbest = INFINITY;
    }
    __syncthreads();
    switch (shape) {
      case 0: wg_colsum_x<8>(v, v.X(0), lc); break;
      case 1: wg_colsum_x<16>(v, v.X(0), lc); break;
      case 2: wg_colsum_x<32>(v, v.X(0), lc); break;
      default: wg_colsum_x<64>(v, v.X(0), lc); break;
    }
    __syncthreads();
    (void)gang_colsum(g, S, lc, 0.0);
    for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
      v.C(0)[j] = lc[j];
      v.C(1)[j] = lc[j];
    }
    __syncthreads();
    if (!S.dead) wg_eval(v, g, shape, S, false, 0.0f, lp, lc, lMc, lMa, red10, tot10, E);
    __syncthreads();
    if (threadIdx.x == 0) {
      S.kkt0 = fmax(E.kc[0], fmax(E.kc[1], E.kc[2]));
      if (S.dead) {
        S.status = PDHCG_ERR_HIP;
        S.done = 1;
      }
    }
    __syncthreads();

    while (!S.done) {
      // ---- price step (eq. update:py) and lagged fold of p into p_avg
      {
        const double *pc = v.P(uni(S.ip[0]));
        double *pt = v.P(uni(S.ip[1]));
        double *pa = v.P(uni(S.ip[2]));
        const double *cp = v.C(uni(S.ic[0])), *cc = v.C(uni(S.ic[1]));
        const double sigma = uni(S.sigma);
        const bool fold = uni(S.fold) != 0;
        const double kin = (double)uni((int)S.k_in);
        for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
          const double p = pc[j];
          const double q = p + sigma * (2.0 * cc[j] - cp[j] - 1.0);
          pt[j] = q;
          lp[j] = q;
          lx[j] = q - p;
          lc[j] = 0.0;
          if (fold && j >= g0 && j < g1) pa[j] = (kin == 1.0) ? p : pa[j] + (p - pa[j]) / kin;
        }
      }
      __syncthreads();
      // ---- row prox (Sec. 2.2), lagged fold of x, column sums
      const float wfold = uni(S.fold) ? (float)(1.0 / (double)uni((int)S.k_in)) : 0.0f;
      const double tau = uni(S.tau);
      const float *xin = v.X(uni(S.ix[0]));
      float *xout = v.X(uni(S.ix[1]));
      float *xavg = v.X(uni(S.ix[2]));
      double dx2 = 0.0;
      switch (shape) {
        case 0: dx2 = wg_rows_step<8, 4>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
        case 1: dx2 = wg_rows_step<16, 4>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
        case 2: dx2 = wg_rows_step<32, 4>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
        case 3: dx2 = wg_rows_step<64, 4>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
        case 4: dx2 = wg_rows_step<64, 8>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
        default: dx2 = wg_rows_step<64, 16>(v, lp, lc, xin, xout, xavg, tau, wfold, prm.max_rounds, prm.rtol); break;
      }
      dx2 = block_sum(dx2, red);  // contains the barrier after the row pass
      dx2 = gang_colsum(g, S, lc, dx2);
      if (S.dead) break;
      // ---- column sums, dp^T K dx and |dp|^2
      double inter = 0.0, dp2 = 0.0;
      {
        const double *cc = v.C(uni(S.ic[1]));
        double *ct = v.C(uni(S.ic[2]));
        for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
          const double c = lc[j];
          ct[j] = c;
          const double dp = lx[j];
          inter = fma(dp, c - cc[j], inter);
          dp2 = fma(dp, dp, dp2);
        }
      }
      inter = block_sum(inter, red);
      dp2 = block_sum(dp2, red);
      // ---- step-size rule (Sec. 5) and role rotation
      if (threadIdx.x == 0) {
        S.total += 1;
        S.since += 1;
        bool accept = true;
        if (prm.step_mode == 1) {
          const double om = S.omega, eta = S.eta;
          const double emax =
              fabs(inter) > 0.0 ? (om * dx2 + dp2 / om) / (2.0 * fabs(inter)) : INFINITY;
          const double kk = (double)(S.total + 1);
          double enew = fmin((1.0 - pow(kk, -0.3)) * emax, (1.0 + pow(kk, -0.6)) * eta);
          enew = fmin(fmax(enew, 0.01 * S.eta0), 3.0 * S.eta0);
          accept = (eta <= emax) || (eta <= 0.01 * S.eta0);
          S.eta = enew;
          S.tau = enew / om;
          S.sigma = enew * om;
        }
        if (accept) {
          int t = S.ix[0]; S.ix[0] = S.ix[1]; S.ix[1] = t;
          t = S.ip[0]; S.ip[0] = S.ip[1]; S.ip[1] = t;
          const int cp = S.ic[0], cc = S.ic[1], ct = S.ic[2];
          S.ic[0] = cc; S.ic[1] = ct; S.ic[2] = cp;
          S.k_in += 1;
          S.accepted += 1;
          S.fold = 1;
        } else {
          S.fold = 0;
        }
      }
      __syncthreads();
      const bool eval = (S.total % prm.eval_every == 0) || S.total >= prm.max_iter;
      if (!eval) continue;
      // ---- KKT check, restart, primal weight (Sec. 5)
      const bool has_avg = S.k_in > 0;
      const float wf = (has_avg && S.fold) ? (float)(1.0 / (double)S.k_in) : 0.0f;
      wg_eval(v, g, shape, S, has_avg, wf, lp, lc, lMc, lMa, red10, tot10, E);
      __syncthreads();
      if (S.dead) break;
      if (threadIdx.x == 0) {
        S.fold = 0;
        S.evals += 1;
        const double kc = fmax(E.kc[0], fmax(E.kc[1], E.kc[2]));
        const double ka = has_avg ? fmax(E.ka[0], fmax(E.ka[1], E.ka[2])) : INFINITY;
        S.cand_avg = ka < kc;
        const double kcand = S.cand_avg ? ka : kc;
        for (int q = 0; q < 3; ++q) S.kout[q] = S.cand_avg ? E.ka[q] : E.kc[q];
        S.kbest = kcand;
        S.do_restart = 0;
        if (!(kcand == kcand)) {
          S.status = PDHCG_ERR_NUMERIC;
          S.done = 1;
        } else if (kcand <= prm.tol) {
          S.status = PDHCG_OK;
          S.done = 1;
        } else if (S.total >= prm.max_iter) {
          S.status = PDHCG_MAX_ITER;
          S.done = 1;
        } else if (prm.restart) {
          const bool rs = (kcand <= prm.beta_suff * S.kkt0) ||
                          (kcand <= prm.beta_nec * S.kkt0 && kcand > S.kkt_prev) ||
                          ((double)S.since >= prm.beta_art * (double)S.total);
          if (rs) {
            S.do_restart = 1;
            if (S.cand_avg) {
              int t = S.ix[0]; S.ix[0] = S.ix[2]; S.ix[2] = t;
              t = S.ip[0]; S.ip[0] = S.ip[2]; S.ip[2] = t;
              t = S.ic[1]; S.ic[1] = S.ic[2]; S.ic[2] = t;
            }
            const double dx = sqrt(E.dxa2[S.cand_avg ? 1 : 0]);
            const double dp = sqrt(E.dpa2[S.cand_avg ? 1 : 0]);
            if (dx > 1e-10 && dp > 1e-10)
              S.omega = exp(prm.theta * log(dp / dx) + (1.0 - prm.theta) * log(S.omega));
            S.restarts += 1;
            if (prm.omega_check_every > 0 && S.restarts % prm.omega_check_every == 0 &&
                (S.omega < S.omega0 / prm.omega_bound || S.omega > S.omega0 * prm.omega_bound))
              S.omega = S.omega0;
            S.kkt0 = kcand;
            S.kkt_prev = INFINITY;
            S.k_in = 0;
            S.since = 0;
            S.cand_avg = 0;
          } else {
            S.kkt_prev = kcand;
          }
        }
        S.tau = S.eta / S.omega;
        S.sigma = S.eta * S.omega;
      }
      __syncthreads();
      if (S.do_restart) {
        if (g.G > 1) {
          gang_sync(g, S);  // every member is done reading the anchors
          if (S.dead) break;
        }
        const float *xs = v.X(uni(S.ix[0]));
        for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x) v.XA[k] = xs[k];
        const double *ps = v.P(uni(S.ip[0]));
        const double *cs = v.C(uni(S.ic[1]));
        double *cp = v.C(uni(S.ic[0]));
        for (int j = threadIdx.x; j < v.m; j += blockDim.x) {
          v.PA[j] = ps[j];
          cp[j] = cs[j];
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0 && S.dead) {
      S.status = PDHCG_ERR_HIP;
      S.done = 1;
    }
    __syncthreads();

    // ---- outputs: the candidate (Sec. 5) or the requested point
    bool out_avg = S.cand_avg;
    if (prm.output == PDHCG_OUTPUT_CURRENT) out_avg = false;
    if (prm.output == PDHCG_OUTPUT_AVERAGE) out_avg = S.k_in > 0;
    const float *xs = v.X(uni(out_avg ? S.ix[2] : S.ix[0]));
    const double *ps = v.P(uni(out_avg ? S.ip[2] : S.ip[0]));
    if (x_out)
      for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x) x_out[eo + k] = xs[k];
    if (p_out && g.r == 0)
      for (int j = threadIdx.x; j < v.m; j += blockDim.x) p_out[go + j] = (float)ps[j];
    if (threadIdx.x == 0 && g.r == 0) {
      BatchInfoDev &I = bd.info[b];
      for (int q = 0; q < 3; ++q) I.kkt[q] = S.kout[q];
      I.rel_kkt = S.kbest;
      I.eta = S.eta;
      I.omega = S.omega;
      I.iters = S.total;
      I.accepted = S.accepted;
      I.restarts = S.restarts;
      I.status = S.status;
      I.evals = S.evals;
      I.ticks = (int64_t)wall_clock64() - S.t0;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ reverse mode --

// Arguments of the batched reverse mode.  Workspace per call: checkpoints
// of x every L steps (nck slices of the concatenated edge arrays), one
// segment of recomputed allocations (L slices), two adjoint slices R, and
// float64 checkpoints of p, c, c_prev (3 nck slices of the goods).
struct BatchAdjArgs {
  const float *x_in, *p_in, *dL_dp;
  float *dL_du, *dL_dw;
  const double *omega;
  float *ck_x, *seg_x, *R0, *R1;
  double *ck_pcc;
  int64_t nnz_total, m_total;
  int32_t K, L, nck, max_rounds;
  double rtol;
  int32_t *err;  // set when a gang meeting timed out
};

// Reverse of the row prox of one step for every row of a market (the
// single-market k_adj_row): with g = r_in + B[col] on the active set A of
// x^{k+1} (its positive entries), s = u^T x^{k+1}, Q = sum_A u^2,
// Gu = sum_A u g: h = (tau w / s^2) Gu / (1 + (tau w / s^2) Q),
// r = g - h u on A (0 elsewhere), dL/du += r tau w / s - h x^{k+1} on A,
// dL/dw += (tau / s) sum r u; column sums of r into lc.  Rows of any
// length: G lanes per row, two sweeps (sums, then outputs).
template <int G>
__device__ __attribute__((noinline)) void wg_adj_rows(const MView &v, const float *xn,
                                                       const float *r_in, const double *lB,
                                                       float *r_out, float *duh, float *dw,
                                                       double *lc, double tau) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = lane & (G - 1), seg = lane / G;
  constexpr int kSeg = kWave / G;
  for (int base = v.r0 + wave * kSeg; base < v.r1; base += kBatchWaves * kSeg) {
    const int i = base + seg;
    const bool rv = i < v.r1;
    const int beg = rv ? v.rp[i] : 0, end = rv ? v.rp[i + 1] : 0;
    const double tw = rv ? tau * (double)v.w[i] : 0.0;
    double s = 0.0, Q = 0.0, Gu = 0.0;
    for (int k = beg + r; k < end; k += G) {
      const float x = xn[k];
      if (x > 0.0f) {
        const double u = (double)v.uh[k];
        s = fma(u, (double)x, s);
        Q = fma(u, u, Q);
        Gu = fma(u, (double)r_in[k] + lB[v.col[k]], Gu);
      }
    }
    s = seg_sum_d<G>(s);
    Q = seg_sum_d<G>(Q);
    Gu = seg_sum_d<G>(Gu);
    const bool live = rv && s > 0.0;
    const double is = live ? fast_rcp(s) : 0.0;
    const double tws2 = tw * is * is;
    const double hh = live ? tws2 * Gu / (1.0 + tws2 * Q) : 0.0;
    double ru = 0.0;
    for (int k = beg + r; k < end; k += G) {
      const float x = xn[k];
      const int c = v.col[k];
      const double u = (double)v.uh[k];
      const bool act = live && x > 0.0f;
      const double rr = act ? (double)r_in[k] + lB[c] - hh * u : 0.0;
      r_out[k] = (float)rr;
      if (act) duh[k] += (float)(rr * tw * is - hh * (double)x);
      ru = fma(rr, u, ru);
      atomicAdd(&lc[c], rr);
    }
    ru = seg_sum_d<G>(ru);
    if (live && r == 0) dw[i] += (float)(tau * is * ru);
  }
}

// Reverse mode for every market of the batch in one persistent launch:
// each workgroup takes markets from the queue (largest first) and runs the
// whole reverse pass of a market (as pdhcg_backward): K fixed steps
// (eta = 0.9 / ||K|| on the support of x, tau = eta / omega_b,
// sigma = eta omega_b) forward
// from (x, p) with a checkpoint every L steps, then segment by segment
// backwards: the segment's forward steps recomputed from its checkpoint,
// then the reverse of each step (row prox, price step).  Prices, column
// sums and the price-step adjoint live in LDS (m <= 2048).  dL/du and
// dL/dw accumulate in the caller's outputs, which are finished in place
// through the row normalisation.
__global__ __launch_bounds__(kBatchBlock) void k_batch_backward(BatchDev bd, BatchAdjArgs a) {
  extern __shared__ double lds_b[];
  double *lp = lds_b;                        // p
  double *lc = lp + kBatchMaxGoods;          // column partials
  double *lcc = lc + kBatchMaxGoods;         // c (column sums of the current x)
  double *lcp = lcc + kBatchMaxGoods;        // c_prev
  double *lP = lcp + kBatchMaxGoods;         // adjoint of p
  double *lB = lP + kBatchMaxGoods;          // adjoint of x through the next price step
  double *lCn = lB + kBatchMaxGoods;         // carried part of it
  __shared__ double red[kBatchWaves];
  __shared__ WGState S;
  __shared__ double s_eta;
  while (true) {
    const int b = take_ticket(bd, S);
    if (b < 0) return;
    MView v;
    v.n = bd.n[b];
    v.m = bd.m[b];
    const int64_t ro = bd.row_off[b], go = bd.good_off[b], eo = bd.edge_off[b];
    v.rp = bd.row_ptr + bd.rp_off[b];
    v.col = bd.col + eo;
    v.deg = bd.deg + go;
    v.uh = bd.uh + eo;
    v.w = bd.w + ro;
    v.rowmax = bd.rowmax + ro;
    const int shape = uni(bd.shape[b]);
    const int m = v.m;
    const GangView g = member_rows(bd, v, S);
    const int e0 = v.rp[v.r0], e1 = v.rp[v.r1];  // this member's entries
    const float *x0 = a.x_in + eo;
    // step: eta = 0.9 / ||K|| for the column-sum operator on the support of
    // the start point (the entries that move near it), ||K|| = sqrt(largest
    // number of buyers with x_ij > 0 of a good); counted in the B area of
    // LDS, which the reverse sweep clears before use
    {
      int *lcnt = reinterpret_cast<int *>(lB);
      for (int j = threadIdx.x; j < m; j += blockDim.x) lcnt[j] = 0;
      __syncthreads();
      for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x)
        if (x0[k] > 0.0f) atomicAdd(&lcnt[v.col[k]], 1);
      __syncthreads();
      for (int j = threadIdx.x; j < m; j += blockDim.x) lc[j] = (double)lcnt[j];
      __syncthreads();
      (void)gang_colsum(g, S, lc, 0.0);  // counts of the whole market
      double cm = 0.0;
      for (int j = threadIdx.x; j < m; j += blockDim.x) cm = fmax(cm, lc[j]);
      cm = block_max(cm, red);
      if (threadIdx.x == 0) s_eta = 0.9 / sqrt(fmax(cm, 1.0));
      __syncthreads();
    }
    const double eta = uni(s_eta);
    const double om = a.omega[b];
    const double tau = eta / om, sigma = eta * om;
    float *R0 = a.R0 + eo, *R1 = a.R1 + eo;
    float *duh = a.dL_du + eo, *dw = a.dL_dw + ro;
    auto ckx = [&](int q) { return a.ck_x + (size_t)q * a.nnz_total + eo; };
    auto segx = [&](int q) { return a.seg_x + (size_t)q * a.nnz_total + eo; };
    auto ckp = [&](int q, int which) {
      return a.ck_pcc + ((size_t)q * 3 + which) * a.m_total + go;
    };

    // One forward step from xin: p += sigma (2 c - c_prev - 1), c_prev = c;
    // x_out = prox(xin - tau p); c = colsum(x_out).
    auto forward = [&](const float *xin, float *xout) {
      for (int j = threadIdx.x; j < m; j += blockDim.x) {
        lp[j] = lp[j] + sigma * (2.0 * lcc[j] - lcp[j] - 1.0);
        lcp[j] = lcc[j];
        lc[j] = 0.0;
      }
      __syncthreads();
      double dx2 = 0.0;
      switch (shape) {
        case 0: dx2 = wg_rows_step<8, 4>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
        case 1: dx2 = wg_rows_step<16, 4>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
        case 2: dx2 = wg_rows_step<32, 4>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
        case 3: dx2 = wg_rows_step<64, 4>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
        case 4: dx2 = wg_rows_step<64, 8>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
        default: dx2 = wg_rows_step<64, 16>(v, lp, lc, xin, xout, nullptr, tau, 0.0f, a.max_rounds, a.rtol); break;
      }
      (void)dx2;
      __syncthreads();
      (void)gang_colsum(g, S, lc, 0.0);
      for (int j = threadIdx.x; j < m; j += blockDim.x) lcc[j] = lc[j];
      __syncthreads();
    };

    // start point: p, c = colsum(x), c_prev = c
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      lp[j] = (double)a.p_in[go + j];
      lc[j] = 0.0;
    }
    __syncthreads();
    switch (shape) {
      case 0: wg_colsum_x<8>(v, x0, lc); break;
      case 1: wg_colsum_x<16>(v, x0, lc); break;
      case 2: wg_colsum_x<32>(v, x0, lc); break;
      default: wg_colsum_x<64>(v, x0, lc); break;
    }
    __syncthreads();
    (void)gang_colsum(g, S, lc, 0.0);
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      lcc[j] = lc[j];
      lcp[j] = lc[j];
    }
    __syncthreads();
    // forward sweep, one checkpoint every L steps, up to the last one (x
    // ping-pongs between R0 and R1, which the reverse sweep takes over
    // afterwards)
    const float *xc = x0;
    const int jlast = (a.nck - 1) * a.L;
    for (int j = 0; j <= jlast; ++j) {
      if (j % a.L == 0) {
        const int q = j / a.L;
        float *dst = ckx(q);
        for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x) dst[k] = xc[k];
        double *cp0 = ckp(q, 0), *cp1 = ckp(q, 1), *cp2 = ckp(q, 2);
        for (int jj = threadIdx.x; jj < m; jj += blockDim.x) {
          cp0[jj] = lp[jj];
          cp1[jj] = lcc[jj];
          cp2[jj] = lcp[jj];
        }
        __syncthreads();
      }
      if (j == jlast) break;
      float *xo = (j % 2 == 0) ? R0 : R1;
      forward(xc, xo);
      xc = xo;
    }
    // reverse sweep
    for (int k = e0 + threadIdx.x; k < e1; k += blockDim.x) {
      R0[k] = 0.0f;
      duh[k] = 0.0f;
    }
    for (int i = v.r0 + threadIdx.x; i < v.r1; i += blockDim.x) dw[i] = 0.0f;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
      lP[j] = (double)a.dL_dp[go + j];
      lB[j] = 0.0;
      lCn[j] = 0.0;
    }
    __syncthreads();
    float *rin = R0, *rout = R1;
    for (int q = a.nck - 1; q >= 0; --q) {
      const int j0 = q * a.L, j1 = min(a.K, j0 + a.L);
      {
        const double *cp0 = ckp(q, 0), *cp1 = ckp(q, 1), *cp2 = ckp(q, 2);
        for (int jj = threadIdx.x; jj < m; jj += blockDim.x) {
          lp[jj] = cp0[jj];
          lcc[jj] = cp1[jj];
          lcp[jj] = cp2[jj];
        }
        __syncthreads();
      }
      const float *xin = ckx(q);
      for (int j = j0; j < j1; ++j) {
        float *xo = segx(j - j0);  // x^{j+1}
        forward(xin, xo);
        xin = xo;
      }
      for (int j = j1 - 1; j >= j0; --j) {
        for (int jj = threadIdx.x; jj < m; jj += blockDim.x) lc[jj] = 0.0;
        __syncthreads();
        switch (shape) {
          case 0: wg_adj_rows<8>(v, segx(j - j0), rin, lB, rout, duh, dw, lc, tau); break;
          case 1: wg_adj_rows<16>(v, segx(j - j0), rin, lB, rout, duh, dw, lc, tau); break;
          case 2: wg_adj_rows<32>(v, segx(j - j0), rin, lB, rout, duh, dw, lc, tau); break;
          default: wg_adj_rows<64>(v, segx(j - j0), rin, lB, rout, duh, dw, lc, tau); break;
        }
        __syncthreads();
        (void)gang_colsum(g, S, lc, 0.0);
        // reverse of the price step: Pt = P - tau colsum(r), B = 2 sigma Pt
        // + Cn, Cn = -sigma Pt, P = Pt
        for (int jj = threadIdx.x; jj < m; jj += blockDim.x) {
          const double pt = lP[jj] - tau * lc[jj];
          lB[jj] = 2.0 * sigma * pt + lCn[jj];
          lCn[jj] = -sigma * pt;
          lP[jj] = pt;
        }
        __syncthreads();
        float *t = rin;
        rin = rout;
        rout = t;
      }
    }
    // through the row normalisation u_hat = u / max_j u_ij: dL/du_ij =
    // dL/du_hat_ij / r_i - [j = first maximum] sum_k u_hat_ik dL/du_hat_ik / r_i
    {
      const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
      for (int i = v.r0 + wave; i < v.r1; i += kBatchWaves) {
        const int beg = v.rp[i], end = v.rp[i + 1];
        double gs = 0.0;
        int first = end;
        for (int k = beg + lane; k < end; k += kWave) {
          gs = fma((double)v.uh[k], (double)duh[k], gs);
          if (v.uh[k] == 1.0f) first = min(first, k);
        }
        gs = wave_sum_d(gs);
        for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o));
        const double inv = 1.0 / (double)v.rowmax[i];
        for (int k = beg + lane; k < end; k += kWave) {
          double val = (double)duh[k] * inv;
          if (k == first) val -= gs * inv;
          duh[k] = (float)val;
        }
      }
    }
    if (threadIdx.x == 0 && S.dead) *a.err = 1;  // a gang meeting timed out
    __syncthreads();
  }
}

}  // namespace pdhcg

// ---------------------------------------------------------------- host API --

using namespace pdhcg;

struct pdhcg_batch_s {
  int32_t count = 0;
  hipStream_t stream = nullptr;
  std::vector<int32_t> h_n, h_m;
  std::vector<int64_t> h_rp_off, h_row_off, h_good_off, h_edge_off;
  int64_t total_rows = 0, total_goods = 0, total_edges = 0;
  // device
  int32_t *order = nullptr, *n = nullptr, *m = nullptr, *shape = nullptr;
  int64_t *rp_off = nullptr, *row_off = nullptr, *good_off = nullptr, *edge_off = nullptr;
  double *sumw = nullptr;
  int32_t *row_ptr = nullptr, *col = nullptr, *deg = nullptr;
  float *uh = nullptr, *w = nullptr, *rowmax = nullptr;
  float *u = nullptr;  // the caller's utilities (for the reverse mode)
  float *X[3] = {nullptr, nullptr, nullptr}, *XA = nullptr;
  double *P[3] = {nullptr, nullptr, nullptr}, *PA = nullptr;
  double *C[3] = {nullptr, nullptr, nullptr};
  BatchInfoDev *info = nullptr;
  uint32_t *queue = nullptr;
  BatchArgs *args = nullptr;  // device copy of the per-solve arguments
  // schedule: resident workgroups per CU (0: as many as fit) and the row
  // shape policy (0: fewest lanes per row, 1: one size wider); set by
  // pdhcg_batch_autotune
  int32_t wg_per_cu = 0, shape_policy = 0;
  std::vector<int32_t> h_dmax;  // largest row degree of each market
  // the solve as a graph (queue reset, persistent kernel), rebuilt when the
  // grid changes
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int32_t graph_grid = 0, graph_plan = -1;
  // gangs: PDHCG_BATCH_GANG at creation (-1: automatic, 0 or 1: none,
  // k >= 2: every market with at least k rows split over k workgroups),
  // and the plan for plan_P resident workgroups
  int32_t gang_mode = -1, plan_P = 0, plan_version = 0;
  int32_t ntickets = 0, ngangs = 0, max_gang = 1;
  std::vector<int32_t> h_order;
  int32_t *tickets = nullptr;  // [ntickets][4]
  uint32_t *gang_cnt = nullptr;
  int64_t *gang_off = nullptr;
  double *gang_buf = nullptr;
  int64_t cap_tickets = 0, cap_gangs = 0, cap_gang_buf = 0;
};

namespace {

template <typename T>
hipError_t balloc(T **p, size_t count) {
  *p = nullptr;
  return hipMalloc((void **)p, (count ? count : 1) * sizeof(T));
}

}  // namespace

// Error text of the batch calls is shared with the single-market calls.
void pdhcg_internal_set_error(const char *msg);

namespace {
int32_t bfail(int32_t st, const std::string &msg) {
  pdhcg_internal_set_error(msg.c_str());
  return st;
}
}  // namespace

#define BHIPC(call)                                                                  \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return bfail(e_ == hipErrorOutOfMemory ? PDHCG_ERR_OOM : PDHCG_ERR_HIP,        \
                   std::string(#call) + ": " + hipGetErrorString(e_));               \
  } while (0)

namespace {

// Row shape of a market from its largest row degree: 8x4, 16x4, 32x4,
// 64x4, 64x8, 64x16 lanes x entries (rows beyond 1024 entries take the
// whole-wave path of the 64x16 shape); policy 1 takes the next wider shape.
int32_t batch_shape(int dmax, int policy) {
  const int s = dmax <= 32 ? 0 : dmax <= 64 ? 1 : dmax <= 128 ? 2 : dmax <= 256 ? 3
              : dmax <= 512 ? 4 : 5;
  return policy == 1 ? std::min(s + 1, 5) : s;
}

}  // namespace

extern "C" void pdhcg_batch_destroy(pdhcg_batch bt) {
  if (!bt) return;
  auto f = [](void *p) {
    if (p) (void)hipFree(p);
  };
  f(bt->order); f(bt->n); f(bt->m); f(bt->shape); f(bt->rp_off); f(bt->row_off);
  f(bt->good_off); f(bt->edge_off); f(bt->sumw); f(bt->row_ptr); f(bt->col); f(bt->deg);
  f(bt->uh); f(bt->u); f(bt->w); f(bt->rowmax); f(bt->XA); f(bt->PA); f(bt->info);
  f(bt->queue); f(bt->args);
  f(bt->tickets); f(bt->gang_cnt); f(bt->gang_off); f(bt->gang_buf);
  for (int q = 0; q < 3; ++q) { f(bt->X[q]); f(bt->P[q]); f(bt->C[q]); }
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  delete bt;
}

extern "C" int32_t pdhcg_batch_create(int32_t count, const int32_t *n, const int32_t *m,
                                      const int32_t *row_ptr_cat, const int32_t *col_cat,
                                      const float *u_cat, const float *w_cat, void *stream,
                                      pdhcg_batch *out) {
  if (!out) return bfail(PDHCG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (count <= 0 || !n || !m || !row_ptr_cat || !col_cat || !u_cat || !w_cat)
    return bfail(PDHCG_ERR_ARG, "count > 0 and non-null arrays required");
  hipStream_t st = (hipStream_t)stream;
  std::vector<int64_t> rp_off(count + 1), row_off(count + 1), good_off(count + 1);
  rp_off[0] = row_off[0] = good_off[0] = 0;
  for (int b = 0; b < count; ++b) {
    if (n[b] <= 0 || m[b] <= 0) return bfail(PDHCG_ERR_ARG, "market sizes must be positive");
    if (m[b] > kBatchMaxGoods)
      return bfail(PDHCG_ERR_UNSUPPORTED, "market " + std::to_string(b) + " has more than " +
                                              std::to_string(kBatchMaxGoods) + " goods");
    rp_off[b + 1] = rp_off[b] + n[b] + 1;
    row_off[b + 1] = row_off[b] + n[b];
    good_off[b + 1] = good_off[b] + m[b];
  }
  std::vector<int32_t> h_rp(rp_off[count]);
  BHIPC(hipMemcpyAsync(h_rp.data(), row_ptr_cat, h_rp.size() * 4, hipMemcpyDeviceToHost, st));
  BHIPC(hipStreamSynchronize(st));
  std::vector<int64_t> edge_off(count + 1);
  edge_off[0] = 0;
  for (int b = 0; b < count; ++b) edge_off[b + 1] = edge_off[b] + h_rp[rp_off[b] + n[b]];
  const int64_t E = edge_off[count];
  if (E <= 0 || E > INT32_MAX) return bfail(PDHCG_ERR_ARG, "total edges must be in (0, 2^31)");
  std::vector<int32_t> h_col(E);
  std::vector<float> h_u(E), h_w(row_off[count]);
  BHIPC(hipMemcpyAsync(h_col.data(), col_cat, E * 4, hipMemcpyDeviceToHost, st));
  BHIPC(hipMemcpyAsync(h_u.data(), u_cat, E * 4, hipMemcpyDeviceToHost, st));
  BHIPC(hipMemcpyAsync(h_w.data(), w_cat, h_w.size() * 4, hipMemcpyDeviceToHost, st));
  BHIPC(hipStreamSynchronize(st));
  std::vector<double> sumw(count);
  std::vector<int32_t> shape(count), deg(good_off[count], 0), dmaxv(count);
  for (int b = 0; b < count; ++b) {
    const int32_t rc = pdhcg_validate_host(n[b], m[b], h_rp[rp_off[b] + n[b]], h_rp.data() + rp_off[b],
                                           h_col.data() + edge_off[b], h_u.data() + edge_off[b],
                                           h_w.data() + row_off[b]);
    if (rc != PDHCG_OK) {
      return bfail(rc, "market " + std::to_string(b) + ": " + pdhcg_last_error());
    }
    double s = 0.0;
    int dmax = 0;
    for (int i = 0; i < n[b]; ++i) {
      s += h_w[row_off[b] + i];
      dmax = std::max(dmax, h_rp[rp_off[b] + i + 1] - h_rp[rp_off[b] + i]);
    }
    for (int64_t k = edge_off[b]; k < edge_off[b + 1]; ++k) deg[good_off[b] + h_col[k]] += 1;
    sumw[b] = s;
    dmaxv[b] = dmax;
    shape[b] = batch_shape(dmax, 0);
  }
  std::vector<int32_t> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return edge_off[a + 1] - edge_off[a] > edge_off[b + 1] - edge_off[b];
  });

  pdhcg_batch bt = new (std::nothrow) pdhcg_batch_s();
  if (!bt) return bfail(PDHCG_ERR_OOM, "host allocation failed");
  bt->count = count;
  bt->stream = st;
  bt->h_n.assign(n, n + count);
  bt->h_m.assign(m, m + count);
  bt->h_rp_off = rp_off;
  bt->h_row_off = row_off;
  bt->h_good_off = good_off;
  bt->h_edge_off = edge_off;
  bt->total_rows = row_off[count];
  bt->total_goods = good_off[count];
  bt->total_edges = E;
  bt->h_dmax = dmaxv;
  bt->h_order = order;
  if (const char *gv = std::getenv("PDHCG_BATCH_GANG")) bt->gang_mode = std::max(0, std::atoi(gv));
  auto cleanup = [&](int32_t code) {
    pdhcg_batch_destroy(bt);
    return code;
  };
#define BK(call)                                                                     \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) {                                                          \
      bfail(e_ == hipErrorOutOfMemory ? PDHCG_ERR_OOM : PDHCG_ERR_HIP,               \
            std::string(#call) + ": " + hipGetErrorString(e_));                      \
      return cleanup(e_ == hipErrorOutOfMemory ? PDHCG_ERR_OOM : PDHCG_ERR_HIP);     \
    }                                                                                \
  } while (0)
  BK(balloc(&bt->order, count)); BK(balloc(&bt->n, count)); BK(balloc(&bt->m, count));
  BK(balloc(&bt->shape, count)); BK(balloc(&bt->rp_off, count + 1));
  BK(balloc(&bt->row_off, count + 1)); BK(balloc(&bt->good_off, count + 1));
  BK(balloc(&bt->edge_off, count + 1)); BK(balloc(&bt->sumw, count));
  BK(balloc(&bt->row_ptr, rp_off[count])); BK(balloc(&bt->col, E)); BK(balloc(&bt->deg, good_off[count]));
  BK(balloc(&bt->uh, E)); BK(balloc(&bt->w, row_off[count])); BK(balloc(&bt->rowmax, row_off[count]));
  BK(balloc(&bt->u, E));
  for (int q = 0; q < 3; ++q) {
    BK(balloc(&bt->X[q], E));
    BK(balloc(&bt->P[q], good_off[count]));
    BK(balloc(&bt->C[q], good_off[count]));
  }
  BK(balloc(&bt->XA, E)); BK(balloc(&bt->PA, good_off[count]));
  BK(balloc(&bt->info, count)); BK(balloc(&bt->queue, 1)); BK(balloc(&bt->args, 1));
  // normalised utilities (Sec. 5 preprocessing), on the host copy
  std::vector<float> h_uh(E), h_rowmax(row_off[count]);
  for (int b = 0; b < count; ++b)
    for (int i = 0; i < n[b]; ++i) {
      const int64_t r0 = edge_off[b] + h_rp[rp_off[b] + i], r1 = edge_off[b] + h_rp[rp_off[b] + i + 1];
      float mx = 0.0f;
      for (int64_t k = r0; k < r1; ++k) mx = std::max(mx, h_u[k]);
      h_rowmax[row_off[b] + i] = mx;
      for (int64_t k = r0; k < r1; ++k) h_uh[k] = h_u[k] / mx;
    }
  BK(hipMemcpyAsync(bt->order, order.data(), count * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->n, n, count * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->m, m, count * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->shape, shape.data(), count * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->rp_off, rp_off.data(), (count + 1) * 8, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->row_off, row_off.data(), (count + 1) * 8, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->good_off, good_off.data(), (count + 1) * 8, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->edge_off, edge_off.data(), (count + 1) * 8, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->sumw, sumw.data(), count * 8, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->row_ptr, row_ptr_cat, rp_off[count] * 4, hipMemcpyDeviceToDevice, st));
  BK(hipMemcpyAsync(bt->col, col_cat, E * 4, hipMemcpyDeviceToDevice, st));
  BK(hipMemcpyAsync(bt->deg, deg.data(), deg.size() * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->uh, h_uh.data(), E * 4, hipMemcpyHostToDevice, st));
  BK(hipMemcpyAsync(bt->u, u_cat, E * 4, hipMemcpyDeviceToDevice, st));
  BK(hipMemcpyAsync(bt->w, w_cat, row_off[count] * 4, hipMemcpyDeviceToDevice, st));
  BK(hipMemcpyAsync(bt->rowmax, h_rowmax.data(), row_off[count] * 4, hipMemcpyHostToDevice, st));
  BK(hipStreamSynchronize(st));
#undef BK
  *out = bt;
  return PDHCG_OK;
}

namespace {

BatchParamsDev batch_params(const pdhcg_params *p) {
  BatchParamsDev d;
  d.tol = p->tol;
  d.max_iter = p->max_iter;
  d.eval_every = p->eval_every;
  d.max_rounds = p->max_search_rounds;
  d.step_mode = p->step_mode;
  d.restart = p->restart;
  d.rtol = p->search_rtol;
  d.beta_suff = p->beta_sufficient;
  d.beta_nec = p->beta_necessary;
  d.beta_art = p->beta_artificial;
  d.theta = p->theta;
  d.omega_bound = p->omega_bound;
  d.eta0 = p->eta0;
  d.omega0 = p->omega0;
  d.omega_check_every = p->omega_check_every;
  d.output = p->output;
  return d;
}

BatchDev batch_view(pdhcg_batch bt) {
  BatchDev bd;
  bd.count = bt->count;
  bd.order = bt->order; bd.n = bt->n; bd.m = bt->m; bd.shape = bt->shape;
  bd.rp_off = bt->rp_off; bd.row_off = bt->row_off; bd.good_off = bt->good_off;
  bd.edge_off = bt->edge_off; bd.sumw = bt->sumw;
  bd.row_ptr = bt->row_ptr; bd.col = bt->col; bd.deg = bt->deg;
  bd.uh = bt->uh; bd.w = bt->w; bd.rowmax = bt->rowmax;
  bd.X0 = bt->X[0]; bd.X1 = bt->X[1]; bd.X2 = bt->X[2]; bd.XA = bt->XA;
  bd.P0 = bt->P[0]; bd.P1 = bt->P[1]; bd.P2 = bt->P[2]; bd.PA = bt->PA;
  bd.C0 = bt->C[0]; bd.C1 = bt->C[1]; bd.C2 = bt->C[2];
  bd.info = bt->info; bd.queue = bt->queue;
  bd.tickets = reinterpret_cast<const int4 *>(bt->tickets);
  bd.ntickets = bt->ntickets;
  bd.ngangs = bt->ngangs;
  bd.gang_cnt = bt->gang_cnt;
  bd.gang_off = bt->gang_off;
  bd.gang_buf = bt->gang_buf;
  return bd;
}

int32_t check_params(const pdhcg_params *p) {
  if (!(p->tol >= 0.0) || p->max_iter < 0 || p->eval_every <= 0 || p->max_search_rounds < 1)
    return bfail(PDHCG_ERR_ARG, "invalid parameters");
  if (p->search != PDHCG_SEARCH_ACTIVESET)
    return bfail(PDHCG_ERR_UNSUPPORTED, "the batched solver uses the active-set search");
  return PDHCG_OK;
}

constexpr int kGangMax = 4;  // workgroups per market in the automatic plan

// Gang plan for P resident workgroups.  Automatic: a market holding more
// than half of the mean load per workgroup (E / P edges) is split over
// ceil(nnz / (E / 2P)) workgroups, at most kGangMax and at most one per row,
// largest markets first, while the gangs' workgroups fit in P (so that all
// of them are resident together).  The gangs' tickets come first, then the
// single markets', each group largest first.
int32_t batch_plan(pdhcg_batch bt, int P) {
  if (bt->plan_P == P) return PDHCG_OK;
  const int count = bt->count;
  const double thr = 0.5 * (double)bt->total_edges / (double)std::max(P, 1);
  std::vector<int32_t> G(count, 1);
  int used = 0;
  for (int t = 0; t < count; ++t) {
    const int b = bt->h_order[t];
    const int64_t nnz = bt->h_edge_off[b + 1] - bt->h_edge_off[b];
    int gb = 1;
    if (bt->gang_mode >= 2) gb = bt->gang_mode;
    else if (bt->gang_mode < 0 && (double)nnz > thr)
      gb = (int)std::min<double>(kGangMax, std::ceil((double)nnz / thr));
    gb = std::min(gb, bt->h_n[b]);
    if (gb > 1 && used + gb > P) gb = 1;
    if (gb > 1) used += gb;
    G[b] = gb;
  }
  std::vector<int32_t> tk;
  std::vector<int64_t> goff;
  int64_t area = 0;
  int gmax = 1;
  for (int pass = 0; pass < 2; ++pass)
    for (int t = 0; t < count; ++t) {
      const int b = bt->h_order[t];
      if ((G[b] > 1) != (pass == 0)) continue;
      if (G[b] == 1) {
        tk.insert(tk.end(), {b, 0, 1, -1});
        continue;
      }
      const int gi = (int)goff.size();
      goff.push_back(area);
      area += gang_area(G[b], bt->h_m[b]);
      gmax = std::max(gmax, G[b]);
      for (int r = 0; r < G[b]; ++r) tk.insert(tk.end(), {b, r, G[b], gi});
    }
  const int64_t nt = (int64_t)tk.size() / 4, ng = (int64_t)goff.size();
  if (nt > bt->cap_tickets) {
    if (bt->tickets) (void)hipFree(bt->tickets);
    bt->tickets = nullptr;
    bt->cap_tickets = 0;
    BHIPC(balloc(&bt->tickets, (size_t)nt * 4));
    bt->cap_tickets = nt;
  }
  if (ng > bt->cap_gangs) {
    if (bt->gang_cnt) (void)hipFree(bt->gang_cnt);
    if (bt->gang_off) (void)hipFree(bt->gang_off);
    bt->gang_cnt = nullptr;
    bt->gang_off = nullptr;
    bt->cap_gangs = 0;
    BHIPC(balloc(&bt->gang_cnt, (size_t)ng));
    BHIPC(balloc(&bt->gang_off, (size_t)ng));
    bt->cap_gangs = ng;
  }
  if (area > bt->cap_gang_buf) {
    if (bt->gang_buf) (void)hipFree(bt->gang_buf);
    bt->gang_buf = nullptr;
    bt->cap_gang_buf = 0;
    BHIPC(balloc(&bt->gang_buf, (size_t)area));
    bt->cap_gang_buf = area;
  }
  BHIPC(hipMemcpyAsync(bt->tickets, tk.data(), tk.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       bt->stream));
  if (ng > 0)
    BHIPC(hipMemcpyAsync(bt->gang_off, goff.data(), goff.size() * sizeof(int64_t),
                         hipMemcpyHostToDevice, bt->stream));
  BHIPC(hipStreamSynchronize(bt->stream));
  bt->ntickets = (int32_t)nt;
  bt->ngangs = (int32_t)ng;
  bt->max_gang = gmax;
  bt->plan_P = P;
  bt->plan_version += 1;
  return PDHCG_OK;
}

// Resident workgroups of the persistent kernel: wg_per_cu per CU (0: as
// many as fit), at most one per ticket; plans the gangs for them.
int32_t batch_grid(pdhcg_batch bt, int wg_per_cu, int *grid) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  int fit = 0;
  BHIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, k_batch_solve, kBatchBlock, 0));
  fit = std::max(fit, 1);
  const int per_cu = wg_per_cu > 0 ? std::min(wg_per_cu, fit) : fit;
  const int P = cus * per_cu;
  const int32_t rc = batch_plan(bt, P);
  if (rc != PDHCG_OK) return rc;
  *grid = (int)std::min<int64_t>(P, bt->ntickets);
  return PDHCG_OK;
}

// (Re)build the solve graph for `grid` workgroups: a queue reset kernel,
// then the persistent kernel (no memset node: the queue is cleared by a
// kernel).
int32_t batch_graph(pdhcg_batch bt, int grid) {
  if (bt->exec && bt->graph_grid == grid && bt->graph_plan == bt->plan_version) return PDHCG_OK;
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  bt->exec = nullptr;
  bt->graph = nullptr;
  BHIPC(hipGraphCreate(&bt->graph, 0));
  uint32_t *queue = bt->queue;
  uint32_t *gang_cnt = bt->gang_cnt;
  int ngangs = bt->ngangs;
  void *a0[] = {&queue, &gang_cnt, &ngangs};
  hipKernelNodeParams k0 = {};
  k0.func = reinterpret_cast<void *>(k_batch_reset);
  k0.gridDim = dim3(1);
  k0.blockDim = dim3(64);
  k0.sharedMemBytes = 0;
  k0.kernelParams = a0;
  k0.extra = nullptr;
  hipGraphNode_t n0, n1;
  BHIPC(hipGraphAddKernelNode(&n0, bt->graph, nullptr, 0, &k0));
  BatchDev bd = batch_view(bt);
  const BatchArgs *args = bt->args;
  void *a1[] = {&bd, &args};
  hipKernelNodeParams k1 = {};
  k1.func = reinterpret_cast<void *>(k_batch_solve);
  k1.gridDim = dim3(grid);
  k1.blockDim = dim3(kBatchBlock);
  k1.sharedMemBytes = 0;
  k1.kernelParams = a1;
  k1.extra = nullptr;
  BHIPC(hipGraphAddKernelNode(&n1, bt->graph, &n0, 1, &k1));
  BHIPC(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
  bt->graph_grid = grid;
  bt->graph_plan = bt->plan_version;
  return PDHCG_OK;
}

// One solve of the whole batch with the current schedule; per-market
// results into hi.  PDHCG_BATCH_EAGER=1 launches the two kernels directly
// instead of the graph.
int32_t batch_run(pdhcg_batch bt, const pdhcg_params *p, float *p_cat, float *x_cat,
                  std::vector<BatchInfoDev> &hi, double *secs) {
  BatchArgs ha;
  ha.prm = batch_params(p);
  ha.p_out = p_cat;
  ha.x_out = x_cat;
  int grid = 0;
  int32_t rc = batch_grid(bt, bt->wg_per_cu, &grid);
  if (rc != PDHCG_OK) return rc;
  const char *eg = std::getenv("PDHCG_BATCH_EAGER");
  const bool eager = eg && std::atoi(eg) != 0;
  if (!eager) {
    rc = batch_graph(bt, grid);
    if (rc != PDHCG_OK) return rc;
  }
  BHIPC(hipMemcpyAsync(bt->args, &ha, sizeof(ha), hipMemcpyHostToDevice, bt->stream));
  const auto t0 = std::chrono::steady_clock::now();
  if (eager) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, bt->stream, bt->queue, bt->gang_cnt,
                       bt->ngangs);
    BHIPC(hipGetLastError());
    const BatchArgs *args = bt->args;
    hipLaunchKernelGGL(k_batch_solve, dim3(grid), dim3(kBatchBlock), 0, bt->stream, batch_view(bt),
                       args);
    BHIPC(hipGetLastError());
  } else {
    BHIPC(hipGraphLaunch(bt->exec, bt->stream));
  }
  hi.resize(bt->count);
  BHIPC(hipMemcpyAsync(hi.data(), bt->info, hi.size() * sizeof(BatchInfoDev),
                       hipMemcpyDeviceToHost, bt->stream));
  BHIPC(hipStreamSynchronize(bt->stream));
  *secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return PDHCG_OK;
}

double tick_seconds() {
  int dev = 0, khz = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  return 1.0 / (1e3 * (double)khz);
}

int32_t set_shape_policy(pdhcg_batch bt, int policy) {
  if (policy == bt->shape_policy) return PDHCG_OK;
  std::vector<int32_t> shape(bt->count);
  for (int b = 0; b < bt->count; ++b) shape[b] = batch_shape(bt->h_dmax[b], policy);
  BHIPC(hipMemcpyAsync(bt->shape, shape.data(), shape.size() * 4, hipMemcpyHostToDevice,
                       bt->stream));
  BHIPC(hipStreamSynchronize(bt->stream));
  bt->shape_policy = policy;
  return PDHCG_OK;
}

}  // namespace

extern "C" int32_t pdhcg_batch_solve(pdhcg_batch bt, const pdhcg_params *params, float *p_cat,
                                     float *x_cat, pdhcg_info *infos) {
  if (!bt || !p_cat || !x_cat) return bfail(PDHCG_ERR_ARG, "null argument");
  pdhcg_params dflt;
  pdhcg_default_params(&dflt);
  const pdhcg_params *p = params ? params : &dflt;
  int32_t rc = check_params(p);
  if (rc != PDHCG_OK) return rc;
  std::vector<BatchInfoDev> hi;
  double secs = 0.0;
  rc = batch_run(bt, p, p_cat, x_cat, hi, &secs);
  if (rc != PDHCG_OK) return rc;
  const double tick = tick_seconds();
  int32_t worst = PDHCG_OK;
  for (int b = 0; b < bt->count; ++b) {
    if (hi[b].status < 0) worst = std::min(worst, hi[b].status);
    else if (hi[b].status == PDHCG_MAX_ITER && worst == PDHCG_OK) worst = PDHCG_MAX_ITER;
    if (infos) {
      pdhcg_info &I = infos[b];
      std::memset(&I, 0, sizeof(I));
      I.rel_primal = hi[b].kkt[0];
      I.rel_dual = hi[b].kkt[1];
      I.rel_gap = hi[b].kkt[2];
      I.rel_kkt = hi[b].rel_kkt;
      I.eta = hi[b].eta;
      I.omega = hi[b].omega;
      I.iters = hi[b].iters;
      I.accepted = hi[b].accepted;
      I.restarts = hi[b].restarts;
      I.status = hi[b].status;
      I.evals = hi[b].evals;
      I.seconds = (double)hi[b].ticks * tick;  // this market's solve on its workgroup
      I.row_pass_seconds = secs;               // the whole launch
    }
  }
  return worst;
}

extern "C" int32_t pdhcg_batch_autotune(pdhcg_batch bt, const pdhcg_params *params,
                                        int32_t trial_iters, pdhcg_batch_schedule *out) {
  if (!bt) return bfail(PDHCG_ERR_ARG, "null batch");
  if (trial_iters < 1) return bfail(PDHCG_ERR_ARG, "trial_iters must be >= 1");
  pdhcg_params p;
  if (params) p = *params;
  else pdhcg_default_params(&p);
  p.tol = 0.0;  // every market runs trial_iters iterations
  p.max_iter = trial_iters;
  int32_t rc = check_params(&p);
  if (rc != PDHCG_OK) return rc;
  int fit = 0;
  BHIPC(hipOccupancyMaxActiveBlocksPerMultiprocessor(&fit, k_batch_solve, kBatchBlock, 0));
  fit = std::max(fit, 1);
  const int old_wg = bt->wg_per_cu, old_policy = bt->shape_policy;
  double best = INFINITY;
  int best_wg = fit, best_policy = 0, trials = 0;
  std::vector<BatchInfoDev> hi;
  for (int policy = 0; policy < 2; ++policy) {
    rc = set_shape_policy(bt, policy);
    if (rc != PDHCG_OK) break;
    for (int wg = 1; wg <= fit; ++wg) {
      bt->wg_per_cu = wg;
      double secs = 0.0;
      rc = batch_run(bt, &p, nullptr, nullptr, hi, &secs);
      if (rc != PDHCG_OK) break;
      ++trials;
      if (secs < best) {
        best = secs;
        best_wg = wg;
        best_policy = policy;
      }
    }
    if (rc != PDHCG_OK) break;
  }
  if (rc != PDHCG_OK) {
    bt->wg_per_cu = old_wg;
    (void)set_shape_policy(bt, old_policy);
    return rc;
  }
  bt->wg_per_cu = best_wg;
  rc = set_shape_policy(bt, best_policy);
  if (rc != PDHCG_OK) return rc;
  if (out) {
    out->wg_per_cu = best_wg;
    out->shape_policy = best_policy;
    out->trials = trials;
    out->best_trial_seconds = best;
  }
  return PDHCG_OK;
}

extern "C" int32_t pdhcg_batch_backward(pdhcg_batch bt, const float *x_cat, const float *p_cat,
                                        const double *omega, int32_t unroll, int32_t ckpt_every,
                                        const float *dL_dp_cat, float *dL_du_cat,
                                        float *dL_dw_cat) {
  if (!bt || !x_cat || !p_cat || !omega || !dL_dp_cat || !dL_du_cat || !dL_dw_cat)
    return bfail(PDHCG_ERR_ARG, "null argument");
  if (unroll < 1 || ckpt_every < 1) return bfail(PDHCG_ERR_ARG, "unroll and ckpt_every must be >= 1");
  for (int b = 0; b < bt->count; ++b)
    if (!(omega[b] > 0.0) || !std::isfinite(omega[b]))
      return bfail(PDHCG_ERR_ARG, "omega of market " + std::to_string(b) + " must be finite and > 0");
  const int K = unroll, L = std::min(ckpt_every, unroll);
  const int nck = (K + L - 1) / L;
  const int64_t E = bt->total_edges, G = bt->total_goods;
  // workspace of this call, freed on every exit path
  struct Owned {
    std::vector<void *> p;
    ~Owned() {
      for (void *q : p)
        if (q) (void)hipFree(q);
    }
  } own;
  auto get = [&](auto **ptr, size_t count) -> hipError_t {
    hipError_t e = balloc(ptr, count);
    if (e == hipSuccess) own.p.push_back(*ptr);
    return e;
  };
  BatchAdjArgs a = {};
  a.x_in = x_cat;
  a.p_in = p_cat;
  a.dL_dp = dL_dp_cat;
  a.dL_du = dL_du_cat;
  a.dL_dw = dL_dw_cat;
  double *d_omega = nullptr;
  BHIPC(get(&d_omega, (size_t)bt->count));
  BHIPC(get(&a.ck_x, (size_t)nck * E));
  BHIPC(get(&a.seg_x, (size_t)L * E));
  BHIPC(get(&a.R0, (size_t)E));
  BHIPC(get(&a.R1, (size_t)E));
  BHIPC(get(&a.ck_pcc, (size_t)3 * nck * G));
  BHIPC(get(&a.err, (size_t)1));
  BHIPC(hipMemsetAsync(a.err, 0, sizeof(int32_t), bt->stream));
  BHIPC(hipMemcpyAsync(d_omega, omega, (size_t)bt->count * sizeof(double), hipMemcpyHostToDevice,
                       bt->stream));
  a.omega = d_omega;
  a.nnz_total = E;
  a.m_total = G;
  a.K = K;
  a.L = L;
  a.nck = nck;
  a.max_rounds = 16;
  a.rtol = 1e-10;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const size_t shm = (size_t)7 * kBatchMaxGoods * sizeof(double);
  // one workgroup per CU (the LDS of the kernel), gangs planned for them
  int32_t rc = batch_plan(bt, cus);
  if (rc != PDHCG_OK) return rc;
  const int grid = (int)std::min<int64_t>(cus, bt->ntickets);
  BatchDev bd = batch_view(bt);
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, bt->stream, bt->queue, bt->gang_cnt,
                     bt->ngangs);
  BHIPC(hipGetLastError());
  hipLaunchKernelGGL(k_batch_backward, dim3(grid), dim3(kBatchBlock), shm, bt->stream, bd, a);
  BHIPC(hipGetLastError());
  int32_t herr = 0;
  BHIPC(hipMemcpyAsync(&herr, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, bt->stream));
  BHIPC(hipStreamSynchronize(bt->stream));  // the workspace is freed on return
  if (herr != 0) return bfail(PDHCG_ERR_HIP, "a gang of workgroups timed out waiting for a member");
  return PDHCG_OK;
}

extern "C" int32_t pdhcg_batch_layout(pdhcg_batch bt, int64_t *good_off, int64_t *edge_off) {
  if (!bt) return bfail(PDHCG_ERR_ARG, "null batch");
  for (int b = 0; b <= bt->count; ++b) {
    if (good_off) good_off[b] = bt->h_good_off[b];
    if (edge_off) edge_off[b] = bt->h_edge_off[b];
  }
  return PDHCG_OK;
}
