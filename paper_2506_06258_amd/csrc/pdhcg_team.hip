// Rows of 513 to kTeamMaxRow entries held in registers by a team of waves:
// the row prox (Sec. 2.2, active-set search inside the Alg. 3 bracket),
// the lagged fold of the kept allocation into its average (Alg. 2), |dx|^2
// and column sums, with the row read from memory once.  A 512-thread
// workgroup runs T = 512 / TEAM teams side by side, each on its own row
// (TEAM threads x E entries per thread hold the row); the teams reduce
// their sums through LDS between workgroup barriers and run the search
// rounds in lockstep (a team whose row is solved idles until the last one
// is), so T rows' loads are in flight at once.
//
// Goods beyond the LDS (relabelled markets, LDS mode 7): the entries of
// these goods are written, with their good's index inside its panel, to
// the panel buffers (pval / pid), where every long row owns a run per
// panel of kPanelW goods; the other row kernels write their entries of
// these goods to fixed slots (cslot) after the runs.  The buffers are laid
// out panel by panel, so that k_panel_part reads each panel's entries
// contiguously and sums them in an LDS copy of the panel, and k_panel_sum
// writes the panels' sums as the column sums of these goods.
//
// The LDS conventions (bit 1: float64 column partials, bit 2: float64
// prices, bit 4: only the goods below hot in LDS; workgroup partials
// written to their slot of the partial arrays) are those of the other row
// kernels, so a market may mix them.
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pdhcg {

namespace {

// Sums (kind 0), maxima (kind 1) or the sum of x and the maximum of y
// (kind 2) of two values over each team: every
// wave reduces its own, the wave leaders write them to red, and every
// thread combines its team's waves.  Returns, in nact, the number of teams
// whose flag is set (the same in every thread).  Contains two workgroup
// barriers; every thread of the workgroup must call it.
template <int W>
__device__ __forceinline__ void team_reduce2(double &x, double &y, int kind, bool flag, int &nact,
                                             double (*red)[3]) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int team = wave / W;
  constexpr int kWaves = kTeamBlock / kWave;
  x = kind == 1 ? wave_max_d(x) : wave_sum_d(x);
  y = kind ? wave_max_d(y) : wave_sum_d(y);
  __syncthreads();  // earlier readers of red are done
  if (lane == 0) {
    red[wave][0] = x;
    red[wave][1] = y;
    red[wave][2] = flag ? 1.0 : 0.0;
  }
  __syncthreads();
  double sx = red[team * W][0], sy = red[team * W][1];
#pragma unroll
  for (int w = 1; w < W; ++w) {
    const double vx = red[team * W + w][0], vy = red[team * W + w][1];
    sx = kind == 1 ? fmax(sx, vx) : sx + vx;
    sy = kind ? fmax(sy, vy) : sy + vy;
  }
  int c = 0;
#pragma unroll
  for (int t = 0; t < kWaves / W; ++t) c += red[t * W][2] != 0.0 ? 1 : 0;
  x = sx;
  y = sy;
  nact = c;
}

}  // namespace

template <int TEAM, int E, int LDS_MODE>
__global__ __launch_bounds__(kTeamBlock) void k_row_team(MarketDev md, BinDev bin, RowIO io) {
  extern __shared__ double lds_d[];
  constexpr int kChunk = E < 16 ? E : 16;  // entries loaded together per thread
  static_assert(E % kChunk == 0, "E must be a multiple of the chunk");
  constexpr int W = TEAM / kWave;        // waves per team
  constexpr int T = kTeamBlock / TEAM;   // teams (rows in flight)
  __shared__ double red[kTeamBlock / kWave][3];
  __shared__ int lslot[T][kMaxPanels];   // next free slot of each panel run of the team's row
  __shared__ uint32_t r_max, r_sum, r_cnt;
  const int m = md.m;
  const float *xin = io.xin;
  const double *pp = io.p;
  float *xout = io.xout;
  float *xavg = io.xavg;
  double tau = io.tau;
  float wfold = io.wfold;
  double *cglob = io.csum;
  if (io.use_state) {
    const DevState *S = md.S;
    xin = pick3<float *>(md.X0, md.X1, md.X2, S->ix[0]);
    xout = pick3<float *>(md.X0, md.X1, md.X2, S->ix[1]);
    xavg = pick3<float *>(md.X0, md.X1, md.X2, S->ix[2]);
    pp = pick3<double *>(md.P0, md.P1, md.P2, S->ip[1]);
    cglob = pick3<double *>(md.C0, md.C1, md.C2, S->ic[2]);
    tau = S->tau;
    wfold = S->fold ? (float)(1.0 / (double)S->k_in) : 0.0f;
  }
  const int hot = (LDS_MODE & 4) ? md.hot : ((LDS_MODE & 3) ? m : 0);
  double *lp = lds_d;
  double *lc = (LDS_MODE & 2) ? lds_d + hot : lds_d;
  if (threadIdx.x == 0) {
    r_max = 0;
    r_sum = 0;
    r_cnt = 0;
  }
  if (LDS_MODE != 0) {
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      if (LDS_MODE & 2) lp[j] = pp[j];
      if (LDS_MODE & 1) lc[j] = 0.0;
    }
  }
  __syncthreads();
  // price of good c: one load through a generic pointer, from LDS for the
  // goods below hot and from global memory (L2) above
  auto pget = [&](int c) {
    if (!(LDS_MODE & 2)) return pp[c];
    if (!(LDS_MODE & 4)) return lp[c];
    const double *src = c < hot ? lp + c : pp + c;
    return *src;
  };
  const int wave = threadIdx.x / kWave;
  const int team = wave / W;
  const int tt = threadIdx.x - team * TEAM;  // thread index inside the team
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  const bool fold = wfold != 0.0f;
  const bool fold_read = fold && wfold != 1.0f;  // weight 1 replaces the average
  // cold entries go to the panel buffers (column sums of relabelled markets)
  const bool panels = (LDS_MODE & 4) && io.colsum && md.npanel > 0;
  double dx2 = 0.0;
  uint32_t rmax = 0, rsum = 0, rcount = 0;
  for (int base = row_lo; base < row_hi; base += T) {
    const int slot = base + team;
    const bool rv = slot < row_hi;
    const int i = rv ? (bin.rows ? bin.rows[slot] : slot) : 0;
    const int beg = rv ? md.row_ptr[i] : 0;
    const int d = rv ? md.row_ptr[i + 1] - beg : 0;
    const double tw = rv ? tau * (double)md.w[i] : 0.0;
    // ---- the row into registers (slots past the row end load nothing)
    // registers hold u and a = x^k - tau p per entry; the good ids and
    // x^k are loaded in chunks of kChunk entries and read again (from
    // cache) for the final sweep
    float u[E];
    double a[E];
    double s0 = 0.0;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += kChunk) {
      int cc[kChunk];
      float xk[kChunk], y[kChunk];
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int k = tt + TEAM * (e0 + e);
        const bool okk = k < d;
        const int q = beg + k;
        u[e0 + e] = okk ? md.uh[q] : 0.0f;
        cc[e] = okk ? md.col[q] : 0;
        xk[e] = okk ? xin[q] : 0.0f;
        y[e] = (okk && fold_read) ? xavg[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int k = tt + TEAM * (e0 + e);
        a[e0 + e] = fma(-tau, pget(cc[e]), (double)xk[e]);
        if (k < d) {
          if (fold) xavg[beg + k] = fold_read ? fmaf(xk[e] - y[e], wfold, y[e]) : xk[e];
          s0 = fma((double)u[e0 + e], (double)xk[e], s0);
        } else {
          u[e0 + e] = 0.0f;
        }
      }
    }
    // ---- trial point (Alg. 3): the row's previous root in solver passes,
    // else s = u^T x^k, else the best single-good lower bound
    const double s_prev = (rv && io.use_state && md.srow) ? (double)md.srow[i] : 0.0;
    // without a previous root, the lower bound is formed alongside u^T x^k
    // (both reduced at once; it is used only when u^T x^k = 0)
    double lb = 0.0;
    if (rv && !(s_prev > 0.0)) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        if (u[e] > 0.0f) {
          const double uu = (double)u[e];
          lb = fmax(lb, pos_root_d(uu * a[e], tw * uu * uu));
        }
    }
    int nact = 0;
    team_reduce2<W>(s0, lb, 2, false, nact, red);
    double s = s_prev > 0.0 ? s_prev : (s0 > 0.0 ? s0 : (lb > 0.0 ? lb : 1.0));
    // ---- search rounds in lockstep
    double L = 0.0, U = INFINITY, sfin = s;
    bool active = rv, found = false;
    int rounds = 0;
    for (int it = 0; it < io.max_rounds; ++it) {
      const double inv = active ? fast_rcp(s) : 0.0, ti = tw * inv;
      double A = 0.0, Q = 0.0;
      if (active) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double uu = (double)u[e];
          const double on = fma(uu, ti, a[e]) > 0.0 ? uu : 0.0;
          A = fma(on, a[e], A);
          Q = fma(on, uu, Q);
        }
      }
      team_reduce2<W>(A, Q, 0, active, nact, red);
      if (nact == 0) break;
      const double B = tw * Q, g = fma(B, inv, A);
      const double sA = active ? pos_root_d(A, B) : 0.0;
      double diff = 0.0, unused3 = 0.0;
      if (active && sA > 0.0) {
        const double tA = tw * fast_rcp(sA);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double uu = (double)u[e];
          if ((fma(uu, ti, a[e]) > 0.0) != (fma(uu, tA, a[e]) > 0.0)) diff = 1.0;
        }
      }
      int nd = 0;
      team_reduce2<W>(diff, unused3, 1, false, nd, red);
      if (active) {
        const bool same = sA > 0.0 && diff == 0.0;
        ++rounds;
        U = fmin(U, fmax(s, g));
        L = fmax(L, fmin(s, g));
        if (sA > 0.0) L = fmax(L, sA);
        if (same || sA == s) {
          sfin = sA;
          found = true;
          active = false;
        } else if (U - L <= io.rtol * U) {
          sfin = 0.5 * (L + U);
          found = true;
          active = false;
        } else {
          s = (L > 0.0) ? L : 0.5 * U;
          sfin = s;
        }
      }
    }
    if (rv && !found && U < INFINITY) sfin = 0.5 * (L + U);
    if (rv && tt == 0) {
      if (io.use_state && md.srow) md.srow[i] = (float)sfin;
      if (io.s_out) io.s_out[i] = (float)sfin;
      rmax = max(rmax, (uint32_t)rounds);
      rsum += (uint32_t)rounds;
      rcount += 1;
    }
    // ---- the allocation at the root, |dx|^2, column sums
    if (panels) {
      for (int p = tt; p < md.npanel; p += TEAM)
        lslot[team][p] = rv ? md.proff[(size_t)(bin.team_off + slot) * md.npanel + p] : 0;
      __syncthreads();
    }
    const double tf = rv ? tw * fast_rcp(sfin) : 0.0;
    // the sweep's indices pass through an empty asm statement, so that the
    // compiler forms their addresses here instead of keeping those of the
    // loads above alive through the search (which ran out of registers)
    int tt2 = tt, beg2 = beg;
    asm volatile("" : "+v"(tt2), "+v"(beg2));
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += kChunk) {
      int cc[kChunk];
      float xk[kChunk];
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int k = tt2 + TEAM * (e0 + e);
        const bool okk = k < d;
        const int q = beg2 + k;
        cc[e] = okk ? md.col[q] : 0;
        xk[e] = okk ? xin[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kChunk; ++e) {
        const int k = tt2 + TEAM * (e0 + e);
        if (k < d) {
          const int q = beg2 + k;
          const float xn = (float)fmax(fma((double)u[e0 + e], tf, a[e0 + e]), 0.0);
          xout[q] = xn;
          const double df = (double)xn - (double)xk[e];
          dx2 = fma(df, df, dx2);
          if (io.colsum) {
            const int cj = cc[e];
            if (!(LDS_MODE & 4) || cj < hot) {
              atomicAdd(((LDS_MODE & 1) && cj < hot) ? &lc[cj] : &cglob[cj], (double)xn);
            } else if (panels) {
              const int gj = cj - hot;
              const int at = atomicAdd(&lslot[team][gj >> kPanelShift], 1);
              md.pval[at] = xn;
              md.pid[at] = (uint16_t)(gj & (kPanelW - 1));
            }
          }
        }
      }
    }
    if (panels) __syncthreads();  // lslot is rewritten for the next rows
  }
  // ---- workgroup partials
  const int lane = threadIdx.x & (kWave - 1);
  const double dsum = wave_sum_d(dx2);
  __syncthreads();
  if (lane == 0) {
    red[wave][0] = dsum;
    if (rcount) {
      atomicMax(&r_max, rmax);
      atomicAdd(&r_sum, rsum);
      atomicAdd(&r_cnt, rcount);
    }
  }
  __syncthreads();
  const int slotw = bin.wg_offset + wg;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kTeamBlock / kWave; ++q) t += red[q][0];
    if (md.rowpart) md.rowpart[(size_t)slotw * kRowStats + 0] = t;
    if (io.use_state) {
      atomicMax(&md.S->rounds_max, r_max);
      atomicAdd((unsigned long long *)&md.S->rounds_sum, (unsigned long long)r_sum);
      atomicAdd((unsigned long long *)&md.S->rows_searched, (unsigned long long)r_cnt);
    }
  }
  if ((LDS_MODE & 1) && io.colsum) {
    double *dst = md.colpart + (size_t)slotw * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) dst[j] = lc[j];
  }
}

// Panel P's entries split into gridDim.x chunks: block (r, P) sums chunk r
// into an LDS copy of the panel (float64) and writes it to
// part[(P * nchunk + r) * kPanelW ...].
__global__ __launch_bounds__(1024) void k_panel_part(const float *val, const uint16_t *id,
                                                     const int64_t *pbeg, double *part) {
  extern __shared__ double acc[];
  const int P = blockIdx.y, r = blockIdx.x, nchunk = gridDim.x;
  for (int j = threadIdx.x; j < kPanelW; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  const int64_t b = pbeg[P], len = pbeg[P + 1] - b;
  const int64_t k0 = b + len * r / nchunk, k1 = b + len * (r + 1) / nchunk;
  constexpr int U = 8;  // entries per thread in flight
  for (int64_t k = k0 + threadIdx.x; k < k1; k += (int64_t)U * blockDim.x) {
    float v[U];
    uint16_t g[U];
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const int64_t q = min(k + (int64_t)e * blockDim.x, k1 - 1);
      v[e] = val[q];
      g[e] = id[q];
    }
#pragma unroll
    for (int e = 0; e < U; ++e)
      if (k + (int64_t)e * blockDim.x < k1) atomicAdd(&acc[g[e]], (double)v[e]);
  }
  __syncthreads();
  double *dst = part + ((size_t)P * nchunk + r) * kPanelW;
  for (int j = threadIdx.x; j < kPanelW; j += blockDim.x) dst[j] = acc[j];
}

// out[hot + g] (+)= the panel partial sums of good hot + g (in chunk order):
// added to what k_cold_sums wrote when some of these goods' entries are
// gathered by column, written otherwise.
__global__ __launch_bounds__(256) void k_panel_sum(MarketDev md, int use_state, double *out,
                                                   const double *part, int nchunk, int accumulate) {
  if (use_state) out = pick3<double *>(md.C0, md.C1, md.C2, md.S->ic[2]);
  const int ncold = md.m - md.hot;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ncold) return;
  const int P = g >> kPanelShift, j = g & (kPanelW - 1);
  const double *src = part + (size_t)P * nchunk * kPanelW + j;
  double s = 0.0;
  for (int r = 0; r < nchunk; ++r) s += src[(size_t)r * kPanelW];
  out[md.hot + g] = accumulate ? out[md.hot + g] + s : s;
}

// ------------------------------------------------------------- launchers --

// Team shapes (TEAM threads x E entries per thread) by code, 1..5: more
// rows in flight for the shorter rows.
int team_code(int d) {
  if (d <= 1024) return 1;         // 128 x 8, 4 rows per workgroup
  if (d <= 2048) return 2;         // 128 x 16, 4 rows
  if (d <= 4096) return 3;         // 128 x 32, 4 rows
  if (d <= 8192) return 4;         // 256 x 32, 2 rows
  if (d <= kTeamMaxRow) return 5;  // 512 x 32, 1 row
  return 0;
}

template <int TEAM, int E>
static hipError_t team_launch_t(const MarketDev &md, const BinDev &bin, int lds_mode,
                                const RowIO &io, int nwg, hipStream_t st) {
  const size_t lh = (lds_mode & 4) ? (size_t)md.hot : (size_t)md.m;
  const size_t shm = lh * (((lds_mode & 2) ? sizeof(double) : 0) +
                           ((lds_mode & 1) ? sizeof(double) : 0));
  switch (lds_mode) {
    case 0: hipLaunchKernelGGL((k_row_team<TEAM, E, 0>), dim3(nwg), dim3(kTeamBlock), shm, st, md, bin, io); break;
    case 1: hipLaunchKernelGGL((k_row_team<TEAM, E, 1>), dim3(nwg), dim3(kTeamBlock), shm, st, md, bin, io); break;
    case 3: hipLaunchKernelGGL((k_row_team<TEAM, E, 3>), dim3(nwg), dim3(kTeamBlock), shm, st, md, bin, io); break;
    case 7: hipLaunchKernelGGL((k_row_team<TEAM, E, 7>), dim3(nwg), dim3(kTeamBlock), shm, st, md, bin, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_row_team(const MarketDev &md, const BinDev &bin, int code, int lds_mode,
                           const RowIO &io, int nwg, hipStream_t st) {
  switch (code) {
    case 1: return team_launch_t<128, 8>(md, bin, lds_mode, io, nwg, st);
    case 2: return team_launch_t<128, 16>(md, bin, lds_mode, io, nwg, st);
    case 3: return team_launch_t<128, 32>(md, bin, lds_mode, io, nwg, st);
    case 4: return team_launch_t<256, 32>(md, bin, lds_mode, io, nwg, st);
    case 5: return team_launch_t<512, 32>(md, bin, lds_mode, io, nwg, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_panel_sums(const MarketDev &md, int use_state, double *out, const float *pval,
                             const uint16_t *pid, const int64_t *pbeg, double *part, int nchunk,
                             int accumulate, int sum, hipStream_t st) {
  const int ncold = md.m - md.hot;
  if (md.npanel <= 0 || ncold <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_panel_part, dim3(nchunk, md.npanel), dim3(1024), kPanelW * sizeof(double), st,
                     pval, pid, pbeg, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sum) return e;
  hipLaunchKernelGGL(k_panel_sum, dim3((ncold + 255) / 256), dim3(256), 0, st, md, use_state, out,
                     part, nchunk, accumulate);
  return hipGetLastError();
}

}  // namespace pdhcg
