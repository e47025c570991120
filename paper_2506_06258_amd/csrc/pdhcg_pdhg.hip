// HIP kernels (gfx950) of restarted PDHG (Alg. 1, Sec. 2.1) on the
// reformulated Eisenberg-Gale program, the paper's baseline method:
// primal (x, t), dual (p, y) of
//   L = -sum_i w_i log t_i + p^T (1^T x - 1) + y^T (t - U x)
// (eq. primal-dual-formulation).  One iteration is
//   k_pstep      p_try = p + sigma (2 c - c_prev - 1)        (eq. update:py),
//                shared with PDHCG;
//   k_pdhg_row   per buyer: y_try = y + sigma (2 g - g_prev)  (eq. update:py),
//                t_try by the closed form of eq. update:t, and per edge
//                x_try = max(0, x - tau (p_try_j - u_ij y_try_i)) (eq.
//                update:x); g_try = t_try - U x_try, the lagged folds of the
//                kept (x, t, y) into their averages, the step-rule sums and
//                per-workgroup column partials of x_try;
//   k_col_chunks / k_col_decide / k_step_rule, shared with PDHCG (the rule
//                adds the buyers' terms).
// There is no root search: every entry is one fused multiply-add and a
// clamp, so the pass is a pure stream (u, good id, x read, x written, the
// average read and written) plus O(n + m) vectors.
//
// Scope: markets whose goods all keep their prices and column partials in
// LDS (LDS mode 3, 2-byte good ids) and rows of at most 512 entries; the
// host returns PDHCG_ERR_UNSUPPORTED otherwise.
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pdhcg {

namespace {

constexpr uint32_t kOOR = 0x80000000u;      // offsets from here on are dropped / read 0
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw 32-bit buffer (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           (int)kRsrcWord3);
}
__device__ __forceinline__ float ld_f(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ int ld_u16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (int)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}
__device__ __forceinline__ void st_f(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}

// Entries of one pass held by a lane, and its row's scalars.
template <int E>
struct Pass {
  float u[E], x[E];
  int c[E];
  int id, lo, d;
  float w;
  double t, y, g, gp;
};

}  // namespace

// Two register sets alternate: while one pass is computed and stored, the
// next pass's entries and row scalars are loading (each wave keeps a pass of
// loads in flight through its compute), as in the PDHCG row kernel.
template <int G, int E>
__global__ __launch_bounds__(kRowBlock) void k_pdhg_row(MarketDev md, PdhgDev pd, BinDev bin) {
  extern __shared__ double lds_d[];
  const int m = md.m;
  const DevState *S = md.S;
  const float *xin = pick3<float *>(md.X0, md.X1, md.X2, S->ix[0]);
  float *xout = pick3<float *>(md.X0, md.X1, md.X2, S->ix[1]);
  float *xavg = pick3<float *>(md.X0, md.X1, md.X2, S->ix[2]);
  const double *pp = pick3<double *>(md.P0, md.P1, md.P2, S->ip[1]);
  const double *tcur = pick3<double *>(pd.T0, pd.T1, pd.T2, S->ix[0]);
  double *ttry = pick3<double *>(pd.T0, pd.T1, pd.T2, S->ix[1]);
  double *tavg = pick3<double *>(pd.T0, pd.T1, pd.T2, S->ix[2]);
  const double *ycur = pick3<double *>(pd.Y0, pd.Y1, pd.Y2, S->ip[0]);
  double *ytry = pick3<double *>(pd.Y0, pd.Y1, pd.Y2, S->ip[1]);
  double *yavg = pick3<double *>(pd.Y0, pd.Y1, pd.Y2, S->ip[2]);
  const double *gprev = pick3<double *>(pd.G0, pd.G1, pd.G2, S->ic[0]);
  const double *gcur = pick3<double *>(pd.G0, pd.G1, pd.G2, S->ic[1]);
  double *gtry = pick3<double *>(pd.G0, pd.G1, pd.G2, S->ic[2]);
  const double tau = S->tau, sigma = S->sigma;
  const bool fold = S->fold != 0;
  const double wfd = fold ? 1.0 / (double)S->k_in : 0.0;
  const float wf = (float)wfd;
  const bool fold_read = fold && S->k_in > 1;  // weight 1 replaces the average

  double *lp = lds_d;      // [m] trial prices
  double *lc = lds_d + m;  // [m] column partials of x_try
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    lp[j] = pp[j];
    lc[j] = 0.0;
  }
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int r = lane & (G - 1);
  const int seg = lane / G;
  constexpr int kSeg = kWave / G;
  constexpr int kWaves = kRowBlock / kWave;
  constexpr int kStep = kWaves * kSeg;
  const int rows = bin.nrows;
  const int stride = (int)gridDim.x * kStep;
  const uint32_t eb = (uint32_t)md.nnz * 4u;
  const __amdgpu_buffer_rsrc_t ru = rsrc(md.uh, eb);
  const __amdgpu_buffer_rsrc_t rc = rsrc(md.col16, (uint32_t)md.nnz * 2u);
  const __amdgpu_buffer_rsrc_t rx = rsrc(xin, eb);
  const __amdgpu_buffer_rsrc_t ro = rsrc(xout, eb);
  const __amdgpu_buffer_rsrc_t ra = rsrc(xavg, fold_read ? eb : 0u);
  const __amdgpu_buffer_rsrc_t raw = rsrc(xavg, fold ? eb : 0u);

  double px2 = 0.0, dy2 = 0.0, iy = 0.0;  // |dx|^2 + |dt|^2, |dy|^2, dy^T (dt - U dx)

  auto load = [&](int slot, Pass<E> &P) {
    const bool rv = slot < rows;
    const int sl = rv ? slot : rows - 1;
    P.id = bin.rows ? bin.rows[sl] : sl;
    P.lo = bin.rlo[sl];
    P.d = rv ? bin.rhi[sl] - P.lo : 0;
    const uint32_t off = 4u * (uint32_t)(P.lo + r);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t o = (r + G * e < P.d) ? off + 4u * G * e : kOOR;
      P.u[e] = ld_f(ru, o);
      P.x[e] = ld_f(rx, o);
      P.c[e] = ld_u16(rc, o == kOOR ? kOOR : o >> 1);
    }
    P.w = md.w[P.id];
    P.t = tcur[P.id];
    P.y = ycur[P.id];
    P.g = gcur[P.id];
    P.gp = gprev[P.id];
  };

  auto compute = [&](const Pass<E> &P, int slot) {
    const bool rv = slot < rows;
    const uint32_t off = 4u * (uint32_t)(P.lo + r);
    // averages of the kept iterate (lagged fold), read before any store
    float xa[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t o = (r + G * e < P.d) ? off + 4u * G * e : kOOR;
      xa[e] = ld_f(ra, o);
    }
    double ta = 0.0, ya = 0.0;
    if (fold_read && rv && r == 0) {
      ta = tavg[P.id];
      ya = yavg[P.id];
    }
    // dual step of the buyer (eq. update:py) and its utility (eq. update:t)
    const double y2 = P.y + sigma * (2.0 * P.g - P.gp);
    const double b = fma(tau, y2, -P.t);
    const double t2 = 0.5 * (fast_sqrt(fma(b, b, 4.0 * tau * (double)P.w)) - b);
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool ok = r + G * e < P.d;
      const uint32_t o = ok ? off + 4u * G * e : kOOR;
      const double uy = (double)P.u[e] * y2;
      const float xn = (float)fmax(fma(-tau, lp[P.c[e]] - uy, (double)P.x[e]), 0.0);
      st_f(ro, o, xn);
      st_f(raw, o, fold_read ? fmaf(P.x[e] - xa[e], wf, xa[e]) : P.x[e]);
      const double df = ok ? (double)xn - (double)P.x[e] : 0.0;
      px2 = fma(df, df, px2);
      s = fma((double)P.u[e], ok ? (double)xn : 0.0, s);
      atomicAdd(&lc[P.c[e]], ok ? (double)xn : 0.0);
    }
    s = seg_sum_d<G>(s);
    if (rv && r == 0) {
      const double g2 = t2 - s;
      ttry[P.id] = t2;
      ytry[P.id] = y2;
      gtry[P.id] = g2;
      if (fold) {
        tavg[P.id] = fold_read ? ta + (P.t - ta) * wfd : P.t;
        yavg[P.id] = fold_read ? ya + (P.y - ya) * wfd : P.y;
      }
      const double dt = t2 - P.t, dy = y2 - P.y;
      px2 = fma(dt, dt, px2);
      dy2 = fma(dy, dy, dy2);
      iy = fma(dy, g2 - P.g, iy);
    }
  };

  int base = blockIdx.x * kStep + wave * kSeg;
  Pass<E> A, B;
  if (base < rows) load(base + seg, A);
  while (base < rows) {
    const int nb = base + stride;
    if (nb < rows) load(nb + seg, B);
    compute(A, base + seg);
    base = nb;
    if (base >= rows) break;
    const int nb2 = base + stride;
    if (nb2 < rows) load(nb2 + seg, A);
    compute(B, base + seg);
    base = nb2;
  }

  __shared__ double red[3][kWaves];
  const double v0 = wave_sum_d(px2), v1 = wave_sum_d(dy2), v2 = wave_sum_d(iy);
  if (lane == 0) {
    red[0][wave] = v0;
    red[1][wave] = v1;
    red[2][wave] = v2;
  }
  __syncthreads();
  const int slot = bin.wg_offset + blockIdx.x;
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[threadIdx.x][q];
    md.rowpart[(size_t)slot * kRowStats + threadIdx.x] = t;
  }
  double *dst = md.colpart + (size_t)slot * m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) dst[j] = lc[j];
}

// KKT pass of PDHG (Sec. 5 Criteria on (x, t, p, y)) over the current point
// and, when io.xa is set, the averaged one, with the lagged fold of the kept
// iterate into the averages (x, t, y here; p in k_eval_col).  Per
// workgroup: the column maxima of u_ij y_i - p_j (ord_key keys) of both
// points and the column sums of the averaged point (of the current one with
// io.want_cc) in LDS, and the row statistics
//   [0 + 8z] max |t - Ux|, [1 + 8z] max |w/t - y|, [2 + 8z] max |w/t|,
//   [3 + 8z] max |y|, [4 + 8z] max x (p - u y)_+, [5 + 8z] max (p - u y)_+,
//   [6 + 8z] max |x|    (z = 0 current, 1 average),
//   [16 + z] |x - x_anchor|^2 + |t - t_anchor|^2, [18 + z] |y - y_anchor|^2.
// g_avg (nullable) receives t - Ux of the averaged point.
template <int G, int E>
__global__ __launch_bounds__(kRowBlock) void k_pdhg_eval(MarketDev md, PdhgDev pd, BinDev bin,
                                                        EvalIO io, const double *tc,
                                                        const double *yc, double *ta, double *ya,
                                                        double *g_avg, int total_wg) {
  extern __shared__ double lds_e[];
  const int m = md.m;
  const bool has_avg = io.xa != nullptr;
  const bool sum_avg = has_avg && !io.want_cc;
  double *lcs = lds_e;
  unsigned int *lMc = reinterpret_cast<unsigned int *>(lds_e + m);
  unsigned int *lMa = lMc + m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    lcs[j] = 0.0;
    lMc[j] = 0u;
    lMa[j] = 0u;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int r = lane & (G - 1);
  const int seg = lane / G;
  constexpr int kSeg = kWave / G;
  constexpr int kWaves = kRowBlock / kWave;
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  const float wf = io.wfold;
  const double wfd = (double)wf;
  const double *tanc = pd.TA, *yanc = pd.YA;

  double st[kPdhgEvalStats];
#pragma unroll
  for (int q = 0; q < kPdhgEvalStats; ++q) st[q] = 0.0;

  for (int base = row_lo + wave * kSeg; base < row_hi; base += kWaves * kSeg) {
    const int slot = base + seg;
    const bool rv = slot < row_hi;
    const int i = rv ? (bin.rows ? bin.rows[slot] : slot) : 0;
    const int beg = rv ? md.row_ptr[i] : 0;
    const int d = rv ? md.row_ptr[i + 1] - beg : 0;
    const double wi = rv ? (double)md.w[i] : 0.0;
    float uh[E], xc[E], xa[E], xz[E];
    double pcj[E], paj[E];
    int cj[E];
    bool ok[E];
    // every load of the pass first, then the gathers, then fold and stores
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = r + G * e;
      ok[e] = idx < d;
      const int k = beg + (ok[e] ? idx : 0);
      uh[e] = md.uh[k];
      xc[e] = io.xc[k];
      cj[e] = md.col[k];
      xa[e] = has_avg ? io.xa[k] : 0.0f;
      xz[e] = io.xanc ? io.xanc[k] : 0.0f;
    }
    const double t0 = rv ? tc[i] : 1.0, y0 = rv ? yc[i] : 0.0;
    double t1 = (rv && has_avg) ? ta[i] : 1.0, y1 = (rv && has_avg) ? ya[i] : 0.0;
    const double tz = (rv && io.xanc) ? tanc[i] : 0.0, yz = (rv && io.xanc) ? yanc[i] : 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      pcj[e] = io.pc[cj[e]];
      paj[e] = has_avg ? io.pa[cj[e]] : 0.0;
    }
    if (has_avg && wf != 0.0f) {
      t1 = (wf == 1.0f) ? t0 : t1 + (t0 - t1) * wfd;
      y1 = (wf == 1.0f) ? y0 : y1 + (y0 - y1) * wfd;
    }
    double sc = 0.0, sa = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!ok[e]) {
        uh[e] = 0.0f;
        xc[e] = 0.0f;
        xa[e] = 0.0f;
        continue;
      }
      const float x = xc[e];
      float y = xa[e];
      double q = paj[e];
      if (has_avg && wf != 0.0f) {
        y = (wf == 1.0f) ? x : fmaf(x - y, wf, y);
        io.xa[beg + r + G * e] = y;
        q = (wf == 1.0f) ? pcj[e] : q + (pcj[e] - q) * wfd;
      }
      xa[e] = y;
      paj[e] = q;
      if (io.xanc) {
        const float z = xz[e];
        st[16] += (double)(x - z) * (double)(x - z);
        if (has_avg) st[17] += (double)(y - z) * (double)(y - z);
      }
      sc += (double)uh[e] * (double)x;
      sa += (double)uh[e] * (double)y;
    }
    sc = seg_sum_d<G>(sc);
    sa = seg_sum_d<G>(sa);
    if (rv && r == 0) {
      const double q0 = wi / t0;
      st[0] = fmax(st[0], fabs(t0 - sc));
      st[1] = fmax(st[1], fabs(q0 - y0));
      st[2] = fmax(st[2], fabs(q0));
      st[3] = fmax(st[3], fabs(y0));
      if (io.tc) io.tc[i] = (float)(t0 * (double)io.rowscale[i]);
      if (io.xanc) {
        st[16] += (t0 - tz) * (t0 - tz);
        st[18] += (y0 - yz) * (y0 - yz);
      }
      if (has_avg) {
        const double q1 = wi / t1;
        st[8] = fmax(st[8], fabs(t1 - sa));
        st[9] = fmax(st[9], fabs(q1 - y1));
        st[10] = fmax(st[10], fabs(q1));
        st[11] = fmax(st[11], fabs(y1));
        if (wf != 0.0f) {
          ta[i] = t1;
          ya[i] = y1;
        }
        if (g_avg) g_avg[i] = t1 - sa;
        if (io.ta) io.ta[i] = (float)(t1 * (double)io.rowscale[i]);
        if (io.xanc) {
          st[17] += (t1 - tz) * (t1 - tz);
          st[19] += (y1 - yz) * (y1 - yz);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!ok[e]) continue;
      const int c = cj[e];
      const double vc = (double)uh[e] * y0;
      const double rc = pcj[e] - vc;
      if (rc > 0.0) {
        st[5] = fmax(st[5], rc);
        st[4] = fmax(st[4], (double)xc[e] * rc);
      }
      st[6] = fmax(st[6], fabs((double)xc[e]));
      atomicMax(&lMc[c], ord_key((float)(vc - pcj[e])));
      if (has_avg) {
        const double va = (double)uh[e] * y1;
        const double ra = paj[e] - va;
        if (ra > 0.0) {
          st[13] = fmax(st[13], ra);
          st[12] = fmax(st[12], (double)xa[e] * ra);
        }
        st[14] = fmax(st[14], fabs((double)xa[e]));
        atomicMax(&lMa[c], ord_key((float)(va - paj[e])));
      }
      if (sum_avg || io.want_cc) atomicAdd(&lcs[c], io.want_cc ? (double)xc[e] : (double)xa[e]);
    }
  }
  __shared__ double red[kWaves][kPdhgEvalStats];
#pragma unroll
  for (int q = 0; q < kPdhgEvalStats; ++q) {
    const double v = (q >= 16) ? wave_sum_d(st[q]) : wave_max_d(st[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  const int slot = bin.wg_offset + wg;
  if (threadIdx.x < kPdhgEvalStats) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int w = 1; w < kWaves; ++w) v = (q >= 16) ? v + red[w][q] : fmax(v, red[w][q]);
    md.rowpart[(size_t)slot * kPdhgEvalStats + q] = v;
  }
  const size_t TW = (size_t)total_wg * m;
  unsigned int *dMc = reinterpret_cast<unsigned int *>(io.evalpart) + (size_t)slot * m;
  unsigned int *dMa = reinterpret_cast<unsigned int *>(io.evalpart + TW) + (size_t)slot * m;
  double *dcs = io.evalcs + (size_t)slot * m;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    dMc[j] = lMc[j];
    dMa[j] = lMa[j];
    dcs[j] = lcs[j];
  }
}

// Relative KKT error of PDHG (Sec. 5 Criteria) from the column statistics
// of k_eval_col (max |c - 1|, max |c|, max (M - p)_+, max (p - M) per point,
// |p - p_anchor|^2) and the row statistics of k_pdhg_eval, in one block.
__global__ __launch_bounds__(kColBlock) void k_pdhg_eval_final(MarketDev md, int total_wg,
                                                               int tiles) {
  DevState *S = md.S;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  constexpr int NC = 10, NR = kPdhgEvalStats;
  double c[NC], rw[NR];
  for (int q = 0; q < NC; ++q) c[q] = (q == 3 || q == 7) ? -INFINITY : 0.0;
  for (int q = 0; q < NR; ++q) rw[q] = 0.0;
  for (int b = threadIdx.x; b < tiles; b += blockDim.x)
    for (int q = 0; q < NC; ++q) {
      const double v = md.colblk[(size_t)b * kEvalColStats + q];
      c[q] = (q >= 8) ? c[q] + v : fmax(c[q], v);
    }
  for (int b = threadIdx.x; b < total_wg; b += blockDim.x)
    for (int q = 0; q < NR; ++q) {
      const double v = md.rowpart[(size_t)b * kPdhgEvalStats + q];
      rw[q] = (q >= 16) ? rw[q] + v : fmax(rw[q], v);
    }
  __shared__ double fc[kColBlock / kWave][NC];
  __shared__ double fr[kColBlock / kWave][NR];
  for (int q = 0; q < NC; ++q) {
    const double v = (q >= 8) ? wave_sum_d(c[q]) : wave_max_d(c[q]);
    if (lane == 0) fc[wave][q] = v;
  }
  for (int q = 0; q < NR; ++q) {
    const double v = (q >= 16) ? wave_sum_d(rw[q]) : wave_max_d(rw[q]);
    if (lane == 0) fr[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 0; q < NC; ++q) {
    c[q] = fc[0][q];
    for (int w = 1; w < kColBlock / kWave; ++w)
      c[q] = (q >= 8) ? c[q] + fc[w][q] : fmax(c[q], fc[w][q]);
  }
  for (int q = 0; q < NR; ++q) {
    rw[q] = fr[0][q];
    for (int w = 1; w < kColBlock / kWave; ++w)
      rw[q] = (q >= 16) ? rw[q] + fr[w][q] : fmax(rw[q], fr[w][q]);
  }
  //   r_primal = max(max|c - 1|, max|t - Ux|) / (1 + max(max|c|, max|t - Ux|, 1))
  //   r_dual   = max(max|w/t - y|, max (M - p)_+)
  //              / (1 + max(max|w/t|, max|y|, max (p - M)))
  //   r_gap    = max x (p - u y)_+ / (1 + max(max|x|, max (p - u y)_+))
  for (int z = 0; z < 2; ++z) {
    const int oc = 4 * z, orr = 8 * z;
    const double tr = rw[orr + 0];
    S->kkt[z][0] = fmax(c[oc + 0], tr) / (1.0 + fmax(fmax(c[oc + 1], tr), 1.0));
    S->kkt[z][1] = fmax(rw[orr + 1], c[oc + 2]) /
                   (1.0 + fmax(fmax(rw[orr + 2], rw[orr + 3]), c[oc + 3]));
    S->kkt[z][2] = rw[orr + 4] / (1.0 + fmax(rw[orr + 6], rw[orr + 5]));
  }
  S->dxa2[0] = rw[16];
  S->dxa2[1] = rw[17];
  S->dpa2[0] = c[8] + rw[18];
  S->dpa2[1] = c[9] + rw[19];
}

// Buyers' state from an allocation: r = U x (normalised), t = t_in / rowmax
// (t_in null: t = r), y = y_in * rowmax (y_in null: y = w / t), and
// g0 = g1 = t - r.  One wave per buyer.
__global__ void k_pdhg_rows_init(MarketDev md, const float *x, const float *t_in,
                                 const float *y_in, const float *rowmax, double *t, double *y,
                                 double *g0, double *g1) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= md.n) return;
  const int b = md.row_ptr[i], e = md.row_ptr[i + 1];
  double s = 0.0;
  for (int k = b + lane; k < e; k += kWave) s += (double)md.uh[k] * (double)x[k];
  s = wave_sum_d(s);
  if (lane == 0) {
    const double ti = t_in ? (double)t_in[i] / (double)rowmax[i] : s;
    const double yi = y_in ? (double)y_in[i] * (double)rowmax[i] : (double)md.w[i] / ti;
    t[i] = ti;
    y[i] = yi;
    g0[i] = ti - s;
    g1[i] = ti - s;
  }
}

// t and y back in the caller's units: t * rowmax, y / rowmax.
__global__ void k_pdhg_rows_out(const double *t, const double *y, const float *rowmax,
                                float *t_out, float *y_out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (t_out) t_out[i] = (float)(t[i] * (double)rowmax[i]);
  if (y_out) y_out[i] = (float)(y[i] / (double)rowmax[i]);
}

// ---------------------------------------------------------------- launchers --

template <int G, int E>
static hipError_t pdhg_row_t(const MarketDev &md, const PdhgDev &pd, const BinDev &bin, int nwg,
                             hipStream_t st) {
  const size_t shm = (size_t)md.m * 2 * sizeof(double);
  hipLaunchKernelGGL((k_pdhg_row<G, E>), dim3(nwg), dim3(kRowBlock), shm, st, md, pd, bin);
  return hipGetLastError();
}

hipError_t launch_pdhg_row(const MarketDev &md, const PdhgDev &pd, const BinDev &bin, int G, int E,
                           int nwg, hipStream_t st) {
#define PDHG_ROW_DISPATCH(g, e) \
  if (G == g && E == e) return pdhg_row_t<g, e>(md, pd, bin, nwg, st);
  PDHCG_ROW_VARIANTS(PDHG_ROW_DISPATCH)
#undef PDHG_ROW_DISPATCH
  return hipErrorInvalidValue;
}

template <int G, int E>
static hipError_t pdhg_eval_t(const MarketDev &md, const PdhgDev &pd, const BinDev &bin,
                              const EvalIO &io, const double *tc, const double *yc, double *ta,
                              double *ya, double *g_avg, int nwg, int total_wg, hipStream_t st) {
  const size_t shm = (size_t)md.m * (sizeof(double) + 2 * sizeof(uint32_t));
  hipLaunchKernelGGL((k_pdhg_eval<G, E>), dim3(nwg), dim3(kRowBlock), shm, st, md, pd, bin, io,
                     tc, yc, ta, ya, g_avg, total_wg);
  return hipGetLastError();
}

hipError_t launch_pdhg_eval(const MarketDev &md, const PdhgDev &pd, const BinDev &bin, int G,
                            int E, const EvalIO &io, const double *tc, const double *yc,
                            double *ta, double *ya, double *g_avg, int nwg, int total_wg,
                            hipStream_t st) {
#define PDHG_EVAL_DISPATCH(g, e) \
  if (G == g && E == e)          \
    return pdhg_eval_t<g, e>(md, pd, bin, io, tc, yc, ta, ya, g_avg, nwg, total_wg, st);
  PDHCG_ROW_VARIANTS(PDHG_EVAL_DISPATCH)
#undef PDHG_EVAL_DISPATCH
  return hipErrorInvalidValue;
}

hipError_t launch_pdhg_eval_final(const MarketDev &md, int total_wg, hipStream_t st) {
  const int tiles = (md.m + kColBlock - 1) / kColBlock;
  hipLaunchKernelGGL(k_pdhg_eval_final, dim3(1), dim3(kColBlock), 0, st, md, total_wg, tiles);
  return hipGetLastError();
}

hipError_t launch_pdhg_rows_init(const MarketDev &md, const float *x, const float *t_in,
                                 const float *y_in, const float *rowmax, double *t, double *y,
                                 double *g0, double *g1, hipStream_t st) {
  const int per = 256 / kWave;
  hipLaunchKernelGGL(k_pdhg_rows_init, dim3((md.n + per - 1) / per), dim3(256), 0, st, md, x,
                     t_in, y_in, rowmax, t, y, g0, g1);
  return hipGetLastError();
}

hipError_t launch_pdhg_rows_out(const double *t, const double *y, const float *rowmax, float *t_out,
                                float *y_out, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_pdhg_rows_out, dim3((n + 255) / 256), dim3(256), 0, st, t, y, rowmax, t_out,
                     y_out, n);
  return hipGetLastError();
}

}  // namespace pdhcg
