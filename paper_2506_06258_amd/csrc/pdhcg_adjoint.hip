// Reverse mode through fixed-step PDHCG iterations (gfx950).
//
// The forward map of one step (Alg. 2 with a fixed step, no restarts):
//   c^k = colsum(x^k),  p^{k+1} = p^k + sigma (2 c^k - c^{k-1} - 1)
//   (eq. update:py),  x^{k+1}_i = prox_i(x^k_i - tau p^{k+1}; w_i, uh_i)
//   (Sec. 2.2).
// The forward steps run with the row pass of pdhcg_kernels.hip in explicit
// mode.  The reverse of one step, for an incoming adjoint
// g = dL/dx^{k+1} = R + B[col] (R per entry, B per good):
//   on the active set A of row i (x^{k+1}_ij > 0), with s = sum_A uh x^{k+1},
//   D = 1 + tau w_i sum_A uh^2 / s^2 and h = (tau w_i / s^2) sum_A g uh / D,
//   r_j = g_j - h uh_j on A (0 off A) is dL/d(x^k - tau p^{k+1}),
//   dL/dw_i += (tau / s) sum_A r uh,  dL/duh_j += r_j tau w_i / s - h x_j;
// then with Pt = dL/dp^{k+1} - tau colsum(r):
//   dL/dp^k = Pt,  dL/dx^k = r + (2 sigma Pt + Cn)[col],  Cn' = -sigma Pt,
// where Cn = dL/dc^k carried from the step after.  (x_j = a_j + tau w uh_j/s
// on A, s = sum_A uh x; differentiating and solving for ds gives D.)
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pdhcg {

namespace {

int grid_1d(int64_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

// Buyers per good on the support of x: cnt[col[k]] += (x[k] > 0), then the
// largest count into *out (both zeroed by the caller).
__global__ void k_active_count(const int32_t *col, const float *x, int64_t nnz, int32_t *cnt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz && x[k] > 0.0f) atomicAdd(&cnt[col[k]], 1);
}

__global__ void k_int_max(const int32_t *cnt, int m, int32_t *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int v = j < m ? cnt[j] : 0;
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
  if ((threadIdx.x & (kWave - 1)) == 0 && v > 0) atomicMax(out, v);
}

__global__ void k_zero_i32(int32_t *a, int64_t len) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) a[k] = 0;
}

// p += sigma (2 c - cprev - 1), float64.
__global__ void k_adj_pstep(double *p, const double *c, const double *cprev, double sigma,
                            int m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) p[j] += sigma * (2.0 * c[j] - cprev[j] - 1.0);
}

// Per-workgroup column partials [rows][hot] summed in kColChunks chunks of
// rows, each chunk in a fixed order: chunk[q][j] (j < hot, row stride m).
__global__ __launch_bounds__(kColBlock) void k_sum_partials(const double *part, int rows, int hot,
                                                            int m, double *chunk) {
  const int j = blockIdx.x * kColBlock + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= hot) return;
  const int per = (rows + kColChunks - 1) / kColChunks;
  const int b0 = q * per, b1 = min(rows, b0 + per);
  double c = 0.0;
  for (int b = b0; b < b1; ++b) c += part[(size_t)b * hot + j];
  chunk[(size_t)q * m + j] = c;
}

// out[j] = sum_q chunk[q][j] in order for j < hot; out[j] = cold[j] above.
__global__ void k_finish_colsum(const double *chunk, const double *cold, int hot, int m,
                                double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double c = 0.0;
  if (j < hot) {
    for (int q = 0; q < kColChunks; ++q) c += chunk[(size_t)q * m + j];
  } else {
    c = cold[j];
  }
  out[j] = c;
}

// Column sums of x by float64 device atomics (one-time use).
__global__ void k_colsum_atomic(const int32_t *col, const float *x, int64_t nnz, double *out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&out[col[k]], (double)x[k]);
}

__global__ void k_zero_f64(double *a, int64_t len) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) a[k] = 0.0;
}

__global__ void k_zero_f32(float *a, int64_t len) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < len) a[k] = 0.0f;
}

// Reverse of the row prox for every row (see the file comment).  Lane r of
// a segment of G lanes handles entries r, r+G, ... of its row.  Column sums
// of r go to float64 LDS partials (LDS_MODE 1, written to md.colpart) or to
// io.csum by device atomics (LDS_MODE 0).
template <int G, int E, int LDS_MODE>
__global__ __launch_bounds__(kRowBlock) void k_adj_row(MarketDev md, BinDev bin, AdjIO io) {
  // LDS_MODE bit 1: column partials of r for goods [0, hot); bit 2: the
  // goods' b values as well (gathered from LDS instead of global memory)
  extern __shared__ double lcs[];
  const int hot = LDS_MODE ? md.hot : 0;
  double *lb = lcs + hot;
  if (LDS_MODE) {
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      lcs[j] = 0.0;
      if (LDS_MODE & 2) lb[j] = io.b[j];
    }
    __syncthreads();
  }
  auto bget = [&](int c) {
    if (!(LDS_MODE & 2)) return io.b[c];
    const bool h = c < hot;
    const double vl = lb[h ? c : 0];
    const double vg = io.b[h ? 0 : c];
    return h ? vl : vg;
  };
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int r = lane & (G - 1);
  const int seg = lane / G;
  constexpr int kSeg = kWave / G;
  constexpr int kWaves = kRowBlock / kWave;
  constexpr int kStep = kWaves * kSeg;  // rows per workgroup pass
  // passes interleaved over the workgroups (as in the forward row kernel);
  // NP passes per trip, all their loads issued before any is used
  constexpr int NP = 2;
  const int wg = blockIdx.x;
  const int stride = (int)gridDim.x * kStep;
  const double tau = io.tau;
  for (int base = wg * kStep + wave * kSeg; base < bin.nrows; base += NP * stride) {
    int i[NP], beg[NP], d[NP];
    double tw[NP];
    bool rv[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      const int slot = base + h * stride + seg;
      rv[h] = slot < bin.nrows;
      i[h] = rv[h] ? (bin.rows ? bin.rows[slot] : slot) : 0;
      beg[h] = rv[h] ? md.row_ptr[i[h]] : 0;
      d[h] = rv[h] ? md.row_ptr[i[h] + 1] - beg[h] : 0;
      tw[h] = rv[h] ? tau * (double)md.w[i[h]] : 0.0;
    }
    float uh[NP][E], xn[NP][E], du[NP][E], rin[NP][E];
    int cj[NP][E];
#pragma unroll
    for (int h = 0; h < NP; ++h)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = r + G * e;
        const int k = beg[h] + (idx < d[h] ? idx : 0);  // row start: in bounds
        uh[h][e] = md.uh[k];
        xn[h][e] = io.xn[k];
        cj[h][e] = md.col[k];
        du[h][e] = io.duh[k];
        rin[h][e] = io.r_in[k];
      }
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      double g[E];
      bool act[E];
      double s = 0.0, Q = 0.0, Gu = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool v = r + G * e < d[h];
        g[e] = v ? (double)rin[h][e] + bget(cj[h][e]) : 0.0;
        act[e] = v && xn[h][e] > 0.0f;
        const double u = act[e] ? (double)uh[h][e] : 0.0;
        s = fma(u, (double)xn[h][e], s);
        Q = fma(u, u, Q);
        Gu = fma(u, g[e], Gu);
      }
      s = seg_sum_d<G>(s);
      Q = seg_sum_d<G>(Q);
      Gu = seg_sum_d<G>(Gu);
      const bool live = rv[h] && s > 0.0;
      const double is = live ? fast_rcp(s) : 0.0;
      const double tws2 = tw[h] * is * is;
      const double hh = live ? tws2 * Gu / (1.0 + tws2 * Q) : 0.0;
      double ru = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int idx = r + G * e;
        if (idx < d[h]) {
          const int k = beg[h] + idx;
          const double rr = (live && act[e]) ? g[e] - hh * (double)uh[h][e] : 0.0;
          io.r_out[k] = (float)rr;
          if (live && act[e])
            io.duh[k] = du[h][e] + (float)(rr * tw[h] * is - hh * (double)xn[h][e]);
          ru = fma(rr, (double)uh[h][e], ru);
          atomicAdd(cj[h][e] < hot ? &lcs[cj[h][e]] : &io.csum[cj[h][e]], rr);
        }
      }
      ru = seg_sum_d<G>(ru);
      if (live && r == 0) io.dw[i[h]] += (float)(tau * is * ru);
    }
  }
  if (LDS_MODE) {
    __syncthreads();
    double *dst = md.colpart + (size_t)(bin.wg_offset + wg) * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) dst[j] = lcs[j];
  }
}

// Column part of the reverse step: Pt = P - tau colsum(r), B = 2 sigma Pt +
// Cn, Cn = -sigma Pt, P = Pt.  colsum(r) from chunk sums for goods below hot
// and from the atomic accumulator cold above.
__global__ void k_adj_col(const double *chunk, const double *cold, int hot, double *P, double *B,
                          double *Cn, double tau, double sigma, int m) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double cr = 0.0;
  if (j < hot) {
    for (int q = 0; q < kColChunks; ++q) cr += chunk[(size_t)q * m + j];
  } else {
    cr = cold[j];
  }
  const double pt = P[j] - tau * cr;
  B[j] = 2.0 * sigma * pt + Cn[j];
  Cn[j] = -sigma * pt;
  P[j] = pt;
}

// dL/du from dL/duh through uh = u / max_j u_ij: the row's first entry with
// uh == 1 is its first maximum.  One wave per row.
__global__ void k_adj_unnormalize(const int32_t *row_ptr, const float *uh, const float *rowmax,
                                  const float *duh, int n, float *du) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= n) return;
  const int beg = row_ptr[i], end = row_ptr[i + 1];
  double gs = 0.0;
  int first = end;
  for (int k = beg + lane; k < end; k += kWave) {
    gs = fma((double)uh[k], (double)duh[k], gs);
    if (uh[k] == 1.0f) first = min(first, k);
  }
  gs = wave_sum_d(gs);
  for (int o = 32; o >= 1; o >>= 1) first = min(first, __shfl_xor(first, o));
  const double inv = 1.0 / (double)rowmax[i];
  for (int k = beg + lane; k < end; k += kWave) {
    double v = (double)duh[k] * inv;
    if (k == first) v -= gs * inv;
    du[k] = (float)v;
  }
}

// ------------------------------------------------------------- launchers --

hipError_t launch_active_colmax(const int32_t *col, const float *x, int64_t nnz, int32_t *cnt,
                               int m, int32_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_i32, dim3(grid_1d(m + 1, 256)), dim3(256), 0, st, cnt, (int64_t)m);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, st, out, (int64_t)1);
  hipLaunchKernelGGL(k_active_count, dim3(grid_1d(nnz, 256)), dim3(256), 0, st, col, x, nnz, cnt);
  hipLaunchKernelGGL(k_int_max, dim3(grid_1d(m, 256)), dim3(256), 0, st, cnt, m, out);
  return hipGetLastError();
}

hipError_t launch_adj_pstep(double *p, const double *c, const double *cprev, double sigma, int m,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_adj_pstep, dim3(grid_1d(m, 256)), dim3(256), 0, st, p, c, cprev, sigma, m);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *part, int rows, int hot, int m, double *chunk,
                               hipStream_t st) {
  if (hot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_partials, dim3(grid_1d(hot, kColBlock), kColChunks), dim3(kColBlock),
                     0, st, part, rows, hot, m, chunk);
  return hipGetLastError();
}

hipError_t launch_finish_colsum(const double *chunk, const double *cold, int hot, int m,
                                double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_colsum, dim3(grid_1d(m, 256)), dim3(256), 0, st, chunk, cold, hot, m,
                     out);
  return hipGetLastError();
}

hipError_t launch_colsum_atomic(const int32_t *col, const float *x, int64_t nnz, double *out,
                                int m, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_1d(m, 256)), dim3(256), 0, st, out, (int64_t)m);
  hipLaunchKernelGGL(k_colsum_atomic, dim3(grid_1d(nnz, 256)), dim3(256), 0, st, col, x, nnz, out);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double *a, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_1d(len, 256)), dim3(256), 0, st, a, len);
  return hipGetLastError();
}

hipError_t launch_zero_f32(float *a, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f32, dim3(grid_1d(len, 256)), dim3(256), 0, st, a, len);
  return hipGetLastError();
}

template <int G, int E, int LDSM>
static hipError_t adj_launch_t(const MarketDev &md, const BinDev &bin, const AdjIO &io, int nwg,
                               hipStream_t st) {
  const size_t shm = (size_t)md.hot * (((LDSM & 1) ? sizeof(double) : 0) +
                                       ((LDSM & 2) ? sizeof(double) : 0));
  hipLaunchKernelGGL((k_adj_row<G, E, LDSM>), dim3(nwg), dim3(kRowBlock), shm, st, md, bin, io);
  return hipGetLastError();
}

hipError_t launch_adj_row(const MarketDev &md, const BinDev &bin, int G, int E, int lds,
                          const AdjIO &io, int nwg, hipStream_t st) {
  // lds: the market's LDS mode (bit 1 partials, bit 2 prices: then b too)
  if (G == 0) return launch_adj_long(md, bin, lds & 1, io, nwg, st);
#define PDHCG_ADJ_DISPATCH(g, e)                                              \
  if (G == g && E == e)                                                       \
    return (lds & 2) ? adj_launch_t<g, e, 3>(md, bin, io, nwg, st)            \
         : (lds & 1) ? adj_launch_t<g, e, 1>(md, bin, io, nwg, st)            \
                     : adj_launch_t<g, e, 0>(md, bin, io, nwg, st);
  PDHCG_ROW_VARIANTS(PDHCG_ADJ_DISPATCH)
#undef PDHCG_ADJ_DISPATCH
  return hipErrorInvalidValue;
}

hipError_t launch_adj_col(const double *chunk, const double *cold, int hot, double *P, double *B,
                          double *Cn, double tau, double sigma, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_col, dim3(grid_1d(m, 256)), dim3(256), 0, st, chunk, cold, hot, P, B,
                     Cn, tau, sigma, m);
  return hipGetLastError();
}

hipError_t launch_adj_unnormalize(const int32_t *row_ptr, const float *uh, const float *rowmax,
                                  const float *duh, int n, float *du, hipStream_t st) {
  const int rows_per_block = 256 / kWave;
  hipLaunchKernelGGL(k_adj_unnormalize, dim3(grid_1d(n, rows_per_block)), dim3(256), 0, st,
                     row_ptr, uh, rowmax, duh, n, du);
  return hipGetLastError();
}

}  // namespace pdhcg
