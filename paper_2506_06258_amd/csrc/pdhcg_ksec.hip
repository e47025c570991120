// The k-section row search of Sec. 2.2.1 mapped the way the paper maps it:
// one row per wave, the row staged in LDS, one lane per candidate.  A wave
// loads its row once (lane l takes entries l, l + 64, ...), forms
// a_j = x^k_j - tau p_j and keeps (a_j, u_j) in its slice of LDS; every
// round the first k lanes (k <= 64 on wave64) evaluate one candidate each,
//   s_l = L + l (U - L) / (k + 1),  g_l = sum_j u_j [a_j + u_j tau w / s_l]_+,
// reading the whole row from LDS (every lane the same address: a broadcast),
// and the bracket becomes U = min(U, min_l max(s_l, g_l)),
// L = max(L, max_l min(s_l, g_l)) by wave reductions.  The loading lanes
// then write x^{k+1} = [a + u tau w / s]_+ at the bracket midpoint from
// their registers.  A round costs every active lane one pass over the row,
// so per round the work is k d lane-steps on k lanes: the time per round
// is the same for any k <= 64, and the rounds needed fall as
// log(1/eps) / log(k + 1).
//
// Scope: rows of at most 512 entries (8 per lane) and column partials of
// every good in LDS beside the 8 waves' staging (m <= 14,000 on gfx950);
// prices are gathered from global memory (L2).
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pdhcg {

namespace {

constexpr int kPerLane = kKwaveMaxRow / kWave;  // entries per lane

__device__ __forceinline__ void wave_lds_sync() {
  // LDS writes of the wave are visible to its own later LDS reads
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ double wave_min_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

}  // namespace

__global__ __launch_bounds__(kRowBlock) void k_row_kwave(MarketDev md, RowIO io) {
  extern __shared__ double lds_k[];
  const int m = md.m;
  constexpr int kWaves = kRowBlock / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  double *lc = lds_k;                                          // [m] column partials
  double *sa = lds_k + m + (size_t)wave * kKwaveMaxRow;        // [512] a_j of this wave's row
  float *su = reinterpret_cast<float *>(lds_k + m + (size_t)kWaves * kKwaveMaxRow) +
              (size_t)wave * kKwaveMaxRow;                     // [512] u_j

  const float *xin = io.xin;
  const double *pp = io.p;
  float *xout = io.xout;
  float *xavg = io.xavg;
  double tau = io.tau;
  float wfold = io.wfold;
  if (io.use_state) {
    const DevState *S = md.S;
    xin = pick3<float *>(md.X0, md.X1, md.X2, S->ix[0]);
    xout = pick3<float *>(md.X0, md.X1, md.X2, S->ix[1]);
    xavg = pick3<float *>(md.X0, md.X1, md.X2, S->ix[2]);
    pp = pick3<double *>(md.P0, md.P1, md.P2, S->ip[1]);
    tau = S->tau;
    wfold = S->fold ? (float)(1.0 / (double)S->k_in) : 0.0f;
  }
  const bool fold = wfold != 0.0f && xavg != nullptr;
  const bool fold_read = fold && wfold != 1.0f;
  const int K = io.sections;
  const double rtol = io.rtol;
  if (io.colsum) {
    for (int j = threadIdx.x; j < m; j += blockDim.x) lc[j] = 0.0;
    __syncthreads();
  }

  double dx2 = 0.0;
  uint32_t rmax = 0, rsum = 0, rcount = 0;
  const int nw = (int)gridDim.x * kWaves;
  for (int i = blockIdx.x * kWaves + wave; i < md.n; i += nw) {
    const int beg = md.row_ptr[i];
    const int d = md.row_ptr[i + 1] - beg;
    const double tw = tau * (double)md.w[i];
    float u[kPerLane], xk[kPerLane], xa[kPerLane];
    int c[kPerLane];
    double a[kPerLane];
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int j = lane + kWave * q;
      const bool ok = j < d;
      const int k = beg + (ok ? j : 0);
      u[q] = ok ? md.uh[k] : 0.0f;
      xk[q] = ok ? xin[k] : 0.0f;
      c[q] = ok ? md.col[k] : 0;
      xa[q] = (ok && fold_read) ? xavg[k] : 0.0f;
    }
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      a[q] = fma(-tau, pp[c[q]], (double)xk[q]);
      s = fma((double)u[q], (double)xk[q], s);
      const int j = lane + kWave * q;
      if (j < d) {
        sa[j] = a[q];
        su[j] = u[q];
      }
    }
    s = wave_sum_d(s);
    // trial value s = u^T x^k (Alg. 3); if zero, the best single-good
    // lower bound, the positive root of s = u_j (a_j + u_j tau w / s)
    if (!(s > 0.0)) {
      double lb = 0.0;
#pragma unroll
      for (int q = 0; q < kPerLane; ++q)
        if (u[q] > 0.0f) {
          const double uu = (double)u[q];
          lb = fmax(lb, pos_root_d(uu * a[q], tw * uu * uu));
        }
      lb = wave_max_d(lb);
      s = lb > 0.0 ? lb : 1.0;
    }
    // bracket [min(s, g(s)), max(s, g(s))] (Alg. 3)
    double g = 0.0;
    {
      const double ti = tw * fast_rcp(s);
#pragma unroll
      for (int q = 0; q < kPerLane; ++q) {
        const double uu = (double)u[q];
        g = fma(uu, fmax(fma(uu, ti, a[q]), 0.0), g);
      }
      g = wave_sum_d(g);
    }
    double U = fmax(s, g), L = fmin(s, g);
    wave_lds_sync();
    int rounds = 0;
    while (rounds < io.max_rounds && U - L > rtol * U) {
      const bool cand = lane < K;
      const double sl = L + (double)(lane + 1) * ((U - L) / (double)(K + 1));
      double hi = INFINITY, lo = 0.0;
      if (cand) {
        const double ti = tw * fast_rcp(sl);
        double acc = 0.0;
        for (int j = 0; j < d; ++j) {
          const double uu = (double)su[j];
          acc = fma(uu, fmax(fma(uu, ti, sa[j]), 0.0), acc);
        }
        hi = fmax(sl, acc);
        lo = fmin(sl, acc);
      }
      U = fmin(U, wave_min_d(hi));
      L = fmax(L, wave_max_d(lo));
      ++rounds;
    }
    const double sfin = 0.5 * (L + U);
    const double tf = tw * fast_rcp(sfin);
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      const int j = lane + kWave * q;
      if (j < d) {
        const int k = beg + j;
        const float xn = (float)fmax(fma((double)u[q], tf, a[q]), 0.0);
        xout[k] = xn;
        if (fold) xavg[k] = fold_read ? fmaf(xk[q] - xa[q], wfold, xa[q]) : xk[q];
        const double df = (double)xn - (double)xk[q];
        dx2 = fma(df, df, dx2);
        if (io.colsum) atomicAdd(&lc[c[q]], (double)xn);
      }
    }
    if (io.s_out && lane == 0) io.s_out[i] = (float)sfin;
    if (lane == 0) {
      rmax = max(rmax, (uint32_t)rounds);
      rsum += (uint32_t)rounds;
      rcount += 1;
    }
    // the next row overwrites the staging only after every lane's reads
    wave_lds_sync();
  }

  __shared__ double red[kWaves];
  __shared__ uint32_t r_max, r_sum, r_cnt;
  if (threadIdx.x == 0) {
    r_max = 0;
    r_sum = 0;
    r_cnt = 0;
  }
  const double ds = wave_sum_d(dx2);
  __syncthreads();
  if (lane == 0) {
    red[wave] = ds;
    if (rcount) {
      atomicMax(&r_max, rmax);
      atomicAdd(&r_sum, rsum);
      atomicAdd(&r_cnt, rcount);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[q];
    if (md.rowpart) md.rowpart[(size_t)blockIdx.x * kRowStats] = t;
    if (io.use_state) {
      atomicMax(&md.S->rounds_max, r_max);
      atomicAdd((unsigned long long *)&md.S->rounds_sum, (unsigned long long)r_sum);
      atomicAdd((unsigned long long *)&md.S->rows_searched, (unsigned long long)r_cnt);
    }
  }
  if (io.colsum) {
    double *dst = md.colpart + (size_t)blockIdx.x * m;
    for (int j = threadIdx.x; j < m; j += blockDim.x) dst[j] = lc[j];
  }
}

size_t kwave_lds_bytes(int m) {
  return (size_t)m * sizeof(double) +
         (size_t)(kRowBlock / kWave) * kKwaveMaxRow * (sizeof(double) + sizeof(float));
}

hipError_t launch_row_kwave(const MarketDev &md, const RowIO &io, int nwg, hipStream_t st) {
  hipLaunchKernelGGL(k_row_kwave, dim3(nwg), dim3(kRowBlock), kwave_lds_bytes(md.m), st, md, io);
  return hipGetLastError();
}

}  // namespace pdhcg
