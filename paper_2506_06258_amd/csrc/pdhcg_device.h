// Device-side building blocks shared by the PDHCG kernels (single-market
// passes and the batched persistent solver).  Included by .hip sources only.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pdhcg_internal.h"

namespace pdhcg {

// ---------------------------------------------------------------- helpers --

template <typename T>
__device__ __forceinline__ T pick3(T a, T b, T c, int i) {
  return i == 0 ? a : (i == 1 ? b : c);
}

// Cross-lane exchange of one 32-bit value within a wave.  Lane masks below
// 16 use DPP moves (quad_perm / row mirrors; bound_ctrl with every row and
// bank enabled, so no lane keeps an old value and no copy is needed), 16
// uses ds_swizzle inside 32-lane halves, 32 uses ds_bpermute.  For a sum or
// max every pairing works as long as it combines disjoint partial results,
// which these do.
template <int MASK>
__device__ __forceinline__ int xchg32(int v) {
  if constexpr (MASK == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
  } else if constexpr (MASK == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  } else if constexpr (MASK == 4) {
    return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
  } else if constexpr (MASK == 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);  // row_mirror
  } else if constexpr (MASK == 16) {
    return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // lane ^ 16 within 32 lanes
  } else {
    return __shfl_xor(v, MASK);
  }
}

template <int MASK>
__device__ __forceinline__ double xchg64(double v) {
  const int lo = xchg32<MASK>(__double2loint(v));
  const int hi = xchg32<MASK>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Sum / max over the aligned segment of G lanes; every lane gets the result.
template <int G>
__device__ __forceinline__ double seg_sum_d(double v) {
  if constexpr (G >= 2) v += xchg64<1>(v);
  if constexpr (G >= 4) v += xchg64<2>(v);
  if constexpr (G >= 8) v += xchg64<4>(v);
  if constexpr (G >= 16) v += xchg64<8>(v);
  if constexpr (G >= 32) v += xchg64<16>(v);
  if constexpr (G >= 64) v += xchg64<32>(v);
  return v;
}

template <int G>
__device__ __forceinline__ double seg_max_d(double v) {
  if constexpr (G >= 2) v = fmax(v, xchg64<1>(v));
  if constexpr (G >= 4) v = fmax(v, xchg64<2>(v));
  if constexpr (G >= 8) v = fmax(v, xchg64<4>(v));
  if constexpr (G >= 16) v = fmax(v, xchg64<8>(v));
  if constexpr (G >= 32) v = fmax(v, xchg64<16>(v));
  if constexpr (G >= 64) v = fmax(v, xchg64<32>(v));
  return v;
}

// 1/x in float64 from the hardware reciprocal estimate and two
// Newton-Raphson steps (each step squares the relative error).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// sqrt(x) in float64 for a normal x > 0 (no range scaling; x = 0 gives
// NaN): the hardware 1/sqrt estimate y, then one coupled Newton step on
// (s, h) ~ (x y, y/2) and two residual corrections s += (x - s^2) h.
__device__ __forceinline__ double fast_sqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  s = fma(fma(-s, s, x), h, s);
  s = fma(fma(-s, s, x), h, s);
  return s;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Order-preserving 32-bit key of a float of any sign: unsigned comparison
// of keys matches the comparison of the floats, and key 0 lies below every
// float.  The KKT column maxima are taken over D = u y - p (the column max of
// u y shifted by the column's price), so that near equilibrium, where M and
// p almost cancel, the float32 key rounds the small difference rather than
// M itself.
__device__ __forceinline__ unsigned int ord_key(float f) {
  const unsigned int b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord_dec(unsigned int k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Bits of a segment inside a wave ballot.
template <int G>
__device__ __forceinline__ bool seg_any(bool pred) {
  const unsigned long long b = __ballot(pred);
  if constexpr (G == 64) {
    return b != 0ull;
  } else {
    const int lane = threadIdx.x & (kWave - 1);
    const int sh = lane & ~(G - 1);
    return ((b >> sh) & ((1ull << G) - 1ull)) != 0ull;
  }
}

// Positive root of s^2 - A s - B = 0 (B >= 0), float64, cancellation-free
// and branch-free: (A + d)/2 for A >= 0, 2B/(d - A) for A < 0, with
// d = sqrt(A^2 + 4B); 0 when A <= 0 and B = 0 (no positive root).
__device__ __forceinline__ double pos_root_d(double A, double B) {
  const double q = fabs(A) + fast_sqrt(fma(A, A, 4.0 * B));
  const double r = (A >= 0.0) ? 0.5 * q : 2.0 * B * fast_rcp(q);
  return (q > 0.0 && (A > 0.0 || B > 0.0)) ? r : 0.0;
}

// Precision: the streamed per-edge data (u_hat, col, x, x_avg) is float32;
// prices are float64 (O(m) values whose updates fall below float32
// resolution near the solution), and the row root is found in float64:
// x_new = x - tau p + tau w u / s subtracts two terms of size tau p to get
// a term of the size of x, which float32 cannot resolve once tau p >> x.
//
// LDS_MODE bits: 1 = float32 column partials in LDS (else float64 global
// atomics); 2 = float64 copy of the prices in LDS (else gathered from
// global memory, where they stay L2-resident).

// One row of the prox step (Sec. 2.2) for the segment of G lanes that owns
// it.  Lane r holds entries r, r+G, ... of the row: u_j, x^k_j and
// a_j = x^k_j - tau p_j (float64).  ok[e] marks the slots inside the row;
// slots past the row end must hold u = 0 (x and a are then ignored).
// With b_j = tau w_i u_j,
//   a_j + b_j/s = a_j + u_j (tau w_i / s),
//   g(s) = sum_j u_j [a_j + b_j/s]_+,   phi(s) = s - g(s),
// so b_j is never stored.  Returns the root s* of phi (or the midpoint of
// the final bracket if max_rounds ran out); the caller forms
// x_j = [a_j + u_j tau w_i / s*]_+.
template <int G, int E, int MODE>
__device__ __forceinline__ double prox_solve(bool rv, double tw, int max_rounds, double rtol,
                                             int K, const bool (&ok)[E], const double (&a)[E],
                                             const float (&uh)[E], const float (&xk)[E],
                                             int &rounds) {
  double s0 = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) s0 = fma((double)uh[e], (double)xk[e], s0);
  s0 = seg_sum_d<G>(s0);

  // Trial value: s = u^T x^k (Alg. 3); if zero, the best single-good lower
  // bound (the root of s = u_j (a_j + b_j/s) for one good j).
  double s = s0;
  if (!(s > 0.0)) {
    double lb = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (uh[e] > 0.0f) {
        const double u = (double)uh[e];
        lb = fmax(lb, pos_root_d(u * a[e], tw * u * u));
      }
    lb = seg_max_d<G>(lb);
    s = lb > 0.0 ? lb : 1.0;  // 1.0: ragged slot without entries
  }

  double L = 0.0, U = INFINITY;
  double sfin = s;
  bool done = !rv;
  rounds = 0;
  if (MODE == 0) {
    // Bracketing search with active-set trial points.  At trial s:
    //   g(s) = A + B/s on the active set at s, A = sum u a, B = tw sum u^2;
    //   [min(s, g), max(s, g)] brackets s* (Sec. 2.2);
    //   the positive root of s^2 - A s - B (the quadratic of the active set
    //   at s) is a lower bound on s*, and it is s* itself once the active
    //   set at that root equals the one at s.
    for (int it = 0; it < max_rounds; ++it) {
      if (!__any(!done)) break;
      const double inv = fast_rcp(s);
      const double ti = tw * inv;
      double A = 0.0, Q = 0.0;
      bool on_s[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double u = (double)uh[e];
        on_s[e] = ok[e] && fma(u, ti, a[e]) > 0.0;
        const double fu = (on_s[e] ? 1.0 : 0.0) * u;  // u on the active set, else 0
        A = fma(fu, a[e], A);
        Q = fma(fu, u, Q);
      }
      A = seg_sum_d<G>(A);
      Q = seg_sum_d<G>(Q);
      const double B = tw * Q;
      const double g = fma(B, inv, A);
      const double sA = pos_root_d(A, B);
      const double tA = tw * fast_rcp(sA > 0.0 ? sA : 1.0);
      bool diff = false;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool on_a = ok[e] && fma((double)uh[e], tA, a[e]) > 0.0;
        diff |= (on_s[e] != on_a);
      }
      const bool same = sA > 0.0 && !seg_any<G>(diff);
      if (!done) {
        ++rounds;
        U = fmin(U, fmax(s, g));
        L = fmax(L, fmin(s, g));
        if (sA > 0.0) L = fmax(L, sA);
        if (same || sA == s) {
          sfin = sA;
          done = true;
        } else if (U - L <= rtol * U) {
          sfin = 0.5 * (L + U);
          done = true;
        } else {
          // next trial: the best lower bound, or the bracket midpoint while
          // no positive lower bound is known
          s = (L > 0.0) ? L : 0.5 * U;
          sfin = s;
        }
      }
    }
    if (!done) sfin = (U < INFINITY) ? 0.5 * (L + U) : s;
  } else {
    // k-section search (Sec. 2.2.1): bracket from the trial s = u^T x^k
    // (Alg. 3), then rounds of K candidates s_l = L + l (U - L)/(K + 1),
    // U = min(U, min_l max(s_l, g_l)), L = max(L, max_l min(s_l, g_l)).
    {
      const double ti = tw * fast_rcp(s);
      double g = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double u = (double)uh[e];
        g = fma(u, fmax(fma(u, ti, a[e]), 0.0), g);
      }
      g = seg_sum_d<G>(g);
      U = fmax(s, g);
      L = fmin(s, g);
    }
    for (int it = 0; it < max_rounds; ++it) {
      const bool need = !done && (U - L > rtol * U);
      if (!__any(need)) break;
      const double step = (U - L) / (double)(K + 1);
      double nU = U, nL = L;
      for (int l = 1; l <= K; ++l) {
        const double sl = fma((double)l, step, L);
        const double ti = tw * fast_rcp(sl);
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double u = (double)uh[e];
          acc = fma(u, fmax(fma(u, ti, a[e]), 0.0), acc);
        }
        const double gl = seg_sum_d<G>(acc);
        nU = fmin(nU, fmax(sl, gl));
        nL = fmax(nL, fmin(sl, gl));
      }
      if (need) {
        ++rounds;
        U = nU;
        L = nL;
      }
    }
    sfin = 0.5 * (L + U);
  }
  return sfin;
}

// prox_solve on a row read here: lane r of the segment loads entries r,
// r+G, ... of the row starting at beg (d entries); pget(j) returns the
// price of good j.  The loaded values stay in uh/xk/cj and a for the caller.
template <int G, int E, int MODE, class PGet>
__device__ __forceinline__ double prox_row(bool rv, int beg, int d, int r, double tau, double tw,
                                           const float *__restrict__ uhp,
                                           const int32_t *__restrict__ colp,
                                           const float *__restrict__ xin, PGet pget,
                                           int max_rounds, double rtol, int K, double (&a)[E],
                                           float (&uh)[E], float (&xk)[E], int (&cj)[E],
                                           int &rounds) {
  bool ok[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = r + G * e;
    const bool v = idx < d;
    const int k = beg + idx;
    float u = 0.0f, x = 0.0f;
    double pj = 0.0;
    int c = 0;
    if (v) {
      u = uhp[k];
      x = xin[k];
      c = colp[k];
      pj = pget(c);
    }
    uh[e] = u;
    xk[e] = x;
    cj[e] = c;
    a[e] = fma(-tau, pj, (double)x);  // x^k - tau p
    ok[e] = v;
  }
  return prox_solve<G, E, MODE>(rv, tw, max_rounds, rtol, K, ok, a, uh, xk, rounds);
}

// Entries of a long row in chunks of kWave * U: lane l takes entries
// l, l + kWave, ..., l + (U-1) kWave of the chunk.  Every load of a chunk is
// issued before any is used (indices past the row end are clamped to its
// last entry and flagged invalid), so a pass over the row waits for memory
// once per chunk rather than once per entry.  body(valid, k, u, a, x, c)
// gets u = 0 for invalid entries; a = x^k - tau p.
constexpr int kLongUnroll = 8;
template <class PGet, class Body>
__device__ __forceinline__ void long_row_chunks(int beg, int d, double tau, const float *uh,
                                                const int32_t *col, const float *xin, PGet pget,
                                                Body body) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int base = 0; base < d; base += kWave * kLongUnroll) {
    float u[kLongUnroll], x[kLongUnroll];
    int c[kLongUnroll];
    double pj[kLongUnroll];
#pragma unroll
    for (int e = 0; e < kLongUnroll; ++e) {
      const int k = beg + min(base + lane + kWave * e, d - 1);
      u[e] = uh[k];
      c[e] = col[k];
      x[e] = xin[k];
    }
#pragma unroll
    for (int e = 0; e < kLongUnroll; ++e) pj[e] = pget(c[e]);
#pragma unroll
    for (int e = 0; e < kLongUnroll; ++e) {
      const int k = base + lane + kWave * e;
      const bool v = k < d;
      body(v, beg + k, v ? (double)u[e] : 0.0, fma(-tau, pj[e], (double)x[e]), x[e], c[e]);
    }
  }
}

// Row root for rows longer than a wave holds in registers: one wave per
// row, every search round re-reads the row (it stays in cache).  Same
// search as prox_row (active-set trial points inside the Alg. 3 bracket).
template <class PGet>
__device__ __forceinline__ double prox_row_long(int beg, int d, double tau, double tw, const float *uh,
                                const int32_t *col, const float *xin, PGet pget, int max_rounds,
                                double rtol, int &rounds) {
  double s0 = 0.0;
  long_row_chunks(beg, d, tau, uh, col, xin, pget,
                  [&](bool, int, double u, double, float x, int) { s0 = fma(u, (double)x, s0); });
  s0 = seg_sum_d<kWave>(s0);
  double s = s0;
  if (!(s > 0.0)) {
    double lb = 0.0;
    long_row_chunks(beg, d, tau, uh, col, xin, pget, [&](bool, int, double u, double a, float, int) {
      if (u > 0.0) lb = fmax(lb, pos_root_d(u * a, tw * u * u));
    });
    lb = seg_max_d<kWave>(lb);
    s = lb > 0.0 ? lb : 1.0;
  }
  double L = 0.0, U = INFINITY, sfin = s;
  rounds = 0;
  for (int it = 0; it < max_rounds; ++it) {
    const double inv = fast_rcp(s), ti = tw * inv;
    double A = 0.0, Q = 0.0;
    long_row_chunks(beg, d, tau, uh, col, xin, pget, [&](bool, int, double u, double a, float, int) {
      const double on = fma(u, ti, a) > 0.0 ? u : 0.0;
      A = fma(on, a, A);
      Q = fma(on, u, Q);
    });
    A = seg_sum_d<kWave>(A);
    Q = seg_sum_d<kWave>(Q);
    const double B = tw * Q, g = fma(B, inv, A), sA = pos_root_d(A, B);
    bool same = false;
    if (sA > 0.0) {
      const double tA = tw * fast_rcp(sA);
      bool diff = false;
      long_row_chunks(beg, d, tau, uh, col, xin, pget,
                      [&](bool, int, double u, double a, float, int) {
                        diff |= ((fma(u, ti, a) > 0.0) != (fma(u, tA, a) > 0.0));
                      });
      same = !seg_any<kWave>(diff);
    }
    ++rounds;
    U = fmin(U, fmax(s, g));
    L = fmax(L, fmin(s, g));
    if (sA > 0.0) L = fmax(L, sA);
    if (same || sA == s) return sA;
    if (U - L <= rtol * U) return 0.5 * (L + U);
    s = (L > 0.0) ? L : 0.5 * U;
    sfin = s;
  }
  return (U < INFINITY) ? 0.5 * (L + U) : sfin;
}

}  // namespace pdhcg
