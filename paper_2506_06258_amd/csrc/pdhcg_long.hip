// Rows longer than the register-resident shapes hold (more than 512
// entries): one wave per row, every pass over the row re-reads it (from
// L2 while it stays there).  Same steps as the register-resident kernels:
//   k_row_long   row prox (Sec. 2.2) with the active-set search, lagged fold
//                of the kept allocation into its average (Alg. 2), |dx|^2
//                and column sums; solver passes start each row's search at
//                its previous root, and the first verification pass also
//                writes the allocation at its trial root (no final pass
//                when that root is accepted);
//   k_eval_long  the row part of the relative KKT error (Sec. 5 Criteria);
//   k_adj_long   the reverse of the row prox (see pdhcg_adjoint.hip).
// The LDS conventions (bit 1: float64 column partials, bit 2: float64
// prices, bit 4: only the goods below hot in LDS; workgroup partials
// written to their slot of the partial arrays) are those of the
// register-resident kernels, so a market may mix both.
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pdhcg {

// The solver's long-row kernel runs 12 waves per workgroup (it needs 125
// VGPRs, so 3 waves per SIMD fit): where the LDS holds one workgroup per CU,
// a bin of up to 12 x (CUs) rows then gives every row a wave of its own in
// one round.
constexpr int kLongBlock = 768;
int long_row_threads() { return kLongBlock; }

template <int LDS_MODE>
__global__ __launch_bounds__(kLongBlock) void k_row_long(MarketDev md, BinDev bin, RowIO io) {
  extern __shared__ double lds_d[];
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
  // goods [0, hot) in LDS (all of them unless LDS_MODE & 4)
  const int hot = (LDS_MODE & 4) ? md.hot : ((LDS_MODE & 3) ? m : 0);
  double *lp = lds_d;
  double *lc = (LDS_MODE & 2) ? lds_d + hot : lds_d;
  if (LDS_MODE != 0) {
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      if (LDS_MODE & 2) lp[j] = pp[j];
      if (LDS_MODE & 1) lc[j] = 0.0;
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  constexpr int kWaves = kLongBlock / kWave;
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  // price of good c: LDS for the goods below hot, global memory above (both
  // loads issued, so that a chunk's gathers are not split by a branch)
  auto pget = [&](int c) {
    if (!(LDS_MODE & 2)) return pp[c];
    if (!(LDS_MODE & 4)) return lp[c];
    const bool h = c < hot;
    const double vl = lp[h ? c : 0];
    const double vg = pp[h ? 0 : c];
    return h ? vl : vg;
  };
  const bool fold = wfold != 0.0f;
  const bool fold_read = fold && wfold != 1.0f;  // weight 1 replaces the average
  double dx2 = 0.0;
  uint32_t rmax = 0, rsum = 0, rcount = 0;
  for (int slot = row_lo + wave; slot < row_hi; slot += kWaves) {
    const int i = bin.rows ? bin.rows[slot] : slot;
    const int beg = md.row_ptr[i];
    const int d = md.row_ptr[i + 1] - beg;
    const double tw = tau * (double)md.w[i];
    int rounds = 0;
    // One pass writing the allocation at tf = tw / s: x^{k+1} = [a + u tf]_+,
    // the fold of x^k into the average (unless an earlier pass of this row
    // did it), |dx|^2 and the column sums; with undo, the contributions of a
    // pass already written at tf_undo are taken back.  With check, the pass
    // also compares the active sets at ti and tf (the search's verification).
    auto sweep = [&](double tf, bool do_fold, bool undo, double tf_undo, bool check, double ti,
                     bool &diff) {
      for (int base = 0; base < d; base += kWave * kLongUnroll) {
        float u[kLongUnroll], xk[kLongUnroll], y[kLongUnroll];
        int c[kLongUnroll];
        double pj[kLongUnroll];
#pragma unroll
        for (int e = 0; e < kLongUnroll; ++e) {
          const int q = beg + min(base + lane + kWave * e, d - 1);
          u[e] = md.uh[q];
          c[e] = md.col[q];
          xk[e] = xin[q];
          y[e] = (do_fold && fold_read) ? xavg[q] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < kLongUnroll; ++e) pj[e] = pget(c[e]);
#pragma unroll
        for (int e = 0; e < kLongUnroll; ++e) {
          const int k = base + lane + kWave * e;
          if (k < d) {
            const int q = beg + k;
            const double uu = (double)u[e];
            const double a = fma(-tau, pj[e], (double)xk[e]);
            if (check) diff |= ((fma(uu, ti, a) > 0.0) != (fma(uu, tf, a) > 0.0));
            const float xn = (float)fmax(fma(uu, tf, a), 0.0);
            xout[q] = xn;
            if (do_fold) xavg[q] = fold_read ? fmaf(xk[e] - y[e], wfold, y[e]) : xk[e];
            const double df = (double)xn - (double)xk[e];
            dx2 = fma(df, df, dx2);
            double add = (double)xn;
            if (undo) {
              const float xs = (float)fmax(fma(uu, tf_undo, a), 0.0);
              const double ds = (double)xs - (double)xk[e];
              dx2 = fma(-ds, ds, dx2);
              add -= (double)xs;
            }
            // with LDS_MODE & 4 the goods from hot on go to their panel
            // slot (a later sweep of the row overwrites it) or are gathered
            // by k_cold_sums
            if (io.colsum && (!(LDS_MODE & 4) || c[e] < hot))
              atomicAdd(((LDS_MODE & 1) && c[e] < hot) ? &lc[c[e]] : &cglob[c[e]], add);
            else if ((LDS_MODE & 4) && io.colsum && md.cslot) {
              const int sl = md.cslot[q];
              if (sl >= 0) md.pval[sl] = xn;
            }
          }
        }
      }
    };
    // Root search (prox_row_long's rounds, started at the row's previous root
    // in solver passes) whose first verification pass also writes the
    // allocation at its trial root: when that root is accepted (the common
    // case near convergence) the row needs no separate final pass.
    double s = (io.use_state && md.srow) ? (double)md.srow[i] : 0.0;
    if (!(s > 0.0)) {
      double s0 = 0.0;
      long_row_chunks(beg, d, tau, md.uh, md.col, xin, pget,
                      [&](bool, int, double uu, double, float x, int) { s0 = fma(uu, (double)x, s0); });
      s = seg_sum_d<kWave>(s0);
    }
    if (!(s > 0.0)) {
      double lb = 0.0;
      long_row_chunks(beg, d, tau, md.uh, md.col, xin, pget, [&](bool, int, double uu, double a, float, int) {
        if (uu > 0.0) lb = fmax(lb, pos_root_d(uu * a, tw * uu * uu));
      });
      lb = seg_max_d<kWave>(lb);
      s = lb > 0.0 ? lb : 1.0;
    }
    double L = 0.0, U = INFINITY, sfin = s, tf_spec = 0.0, s_spec = 0.0;
    bool spec = false, found = false;
    for (int it = 0; it < io.max_rounds; ++it) {
      const double inv = fast_rcp(s), ti = tw * inv;
      double A = 0.0, Q = 0.0;
      long_row_chunks(beg, d, tau, md.uh, md.col, xin, pget,
                      [&](bool, int, double uu, double a, float, int) {
                        const double on = fma(uu, ti, a) > 0.0 ? uu : 0.0;
                        A = fma(on, a, A);
                        Q = fma(on, uu, Q);
                      });
      A = seg_sum_d<kWave>(A);
      Q = seg_sum_d<kWave>(Q);
      const double B = tw * Q, g = fma(B, inv, A), sA = pos_root_d(A, B);
      bool same = false;
      if (sA > 0.0) {
        const double tA = tw * fast_rcp(sA);
        bool diff = false;
        if (!spec) {
          sweep(tA, fold, false, 0.0, true, ti, diff);
          spec = true;
          tf_spec = tA;
          s_spec = sA;
        } else {
          long_row_chunks(beg, d, tau, md.uh, md.col, xin, pget,
                          [&](bool, int, double uu, double a, float, int) {
                            diff |= ((fma(uu, ti, a) > 0.0) != (fma(uu, tA, a) > 0.0));
                          });
        }
        same = !seg_any<kWave>(diff);
      }
      ++rounds;
      U = fmin(U, fmax(s, g));
      L = fmax(L, fmin(s, g));
      if (sA > 0.0) L = fmax(L, sA);
      if (same || sA == s) {
        sfin = sA;
        found = true;
        break;
      }
      if (U - L <= io.rtol * U) {
        sfin = 0.5 * (L + U);
        found = true;
        break;
      }
      s = (L > 0.0) ? L : 0.5 * U;
      sfin = s;
    }
    if (!found && U < INFINITY) sfin = 0.5 * (L + U);
    if (io.use_state && md.srow && lane == 0) md.srow[i] = (float)sfin;
    // the allocation at the root, unless the verification pass wrote it
    if (!(spec && sfin == s_spec)) {
      bool unused = false;
      sweep(tw * fast_rcp(sfin), fold && !spec, spec, tf_spec, false, 0.0, unused);
    }
    if (lane == 0) {
      if (io.s_out) io.s_out[i] = (float)sfin;
      rmax = max(rmax, (uint32_t)rounds);
      rsum += (uint32_t)rounds;
      rcount += 1;
    }
  }
  __shared__ double red[kWaves];
  __shared__ uint32_t red_rmax, red_rsum, red_rcnt;
  if (threadIdx.x == 0) {
    red_rmax = 0;
    red_rsum = 0;
    red_rcnt = 0;
  }
  const double dsum = wave_sum_d(dx2);
  __syncthreads();
  if (lane == 0) {
    red[wave] = dsum;
    if (rcount) {
      atomicMax(&red_rmax, rmax);
      atomicAdd(&red_rsum, rsum);
      atomicAdd(&red_rcnt, rcount);
    }
  }
  __syncthreads();
  const int slotw = bin.wg_offset + wg;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[q];
    if (md.rowpart) md.rowpart[(size_t)slotw * kRowStats + 0] = t;
    if (io.use_state) {
      atomicMax(&md.S->rounds_max, red_rmax);
      atomicAdd((unsigned long long *)&md.S->rounds_sum, (unsigned long long)red_rsum);
      atomicAdd((unsigned long long *)&md.S->rows_searched, (unsigned long long)red_rcnt);
    }
  }
  if ((LDS_MODE & 1) && io.colsum) {
    double *dst = md.colpart + (size_t)slotw * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) dst[j] = lc[j];
  }
}

// Row part of the KKT error for long rows; same outputs and partial layout
// as k_eval_row (statistics 0..9, column maxima, column sums).
template <int LDS_MODE>
__global__ __launch_bounds__(kRowBlock) void k_eval_long(MarketDev md, BinDev bin, EvalIO io,
                                                         int total_wg) {
  extern __shared__ double lds_e[];
  const int m = md.m;
  const bool has_avg = io.xa != nullptr;
  const bool sum_avg = has_avg && !io.want_cc;
  const int hot = (LDS_MODE == 1) ? md.hot : 0;
  const bool cg = (LDS_MODE == 1) && md.ecold_ptr != nullptr;  // goods from hot on: k_eval_cold
  double *lcs = lds_e;
  unsigned int *lMc = reinterpret_cast<unsigned int *>(lds_e + hot);
  unsigned int *lMa = lMc + hot;
  if (LDS_MODE == 1) {
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      lcs[j] = 0.0;
      lMc[j] = 0u;
      lMa[j] = 0u;
    }
    __syncthreads();
  }
  const size_t TW = (LDS_MODE == 1) ? (size_t)total_wg * hot : (size_t)m;
  unsigned int *gMc = reinterpret_cast<unsigned int *>(io.evalpart);
  unsigned int *gMa = reinterpret_cast<unsigned int *>(io.evalpart + TW);
  unsigned int *xMc = (LDS_MODE == 1) ? io.gmax : gMc;
  unsigned int *xMa = (LDS_MODE == 1) ? io.gmax + m : gMa;
  double *xcs = (LDS_MODE == 1) ? io.gsum : io.cacc;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  constexpr int kWaves = kRowBlock / kWave;
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  const float wf = io.wfold;
  double st[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) st[q] = 0.0;
  for (int slot = row_lo + wave; slot < row_hi; slot += kWaves) {
    const int i = bin.rows ? bin.rows[slot] : slot;
    const int beg = md.row_ptr[i];
    const int d = md.row_ptr[i + 1] - beg;
    const double wi = (double)md.w[i];
    // pass 1: t = u^T x of both points (folding the average first); chunks
    // of kWave * kLongUnroll entries, every load of a chunk issued first
    double tc = 0.0, ta = 0.0;
    for (int base = 0; base < d; base += kWave * kLongUnroll) {
      float u[kLongUnroll], x[kLongUnroll], y[kLongUnroll], z[kLongUnroll];
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int q = beg + min(base + lane + kWave * e, d - 1);
        u[e] = md.uh[q];
        x[e] = io.xc[q];
        y[e] = has_avg ? io.xa[q] : 0.0f;
        z[e] = io.xanc ? io.xanc[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int k = base + lane + kWave * e;
        if (k < d) {
          tc = fma((double)u[e], (double)x[e], tc);
          if (has_avg) {
            float yy = y[e];
            if (wf != 0.0f) {
              yy = (wf == 1.0f) ? x[e] : fmaf(x[e] - yy, wf, yy);
              io.xa[beg + k] = yy;
            }
            ta = fma((double)u[e], (double)yy, ta);
          }
          if (io.xanc) st[8] += (double)(x[e] - z[e]) * (double)(x[e] - z[e]);
        }
      }
    }
    tc = wave_sum_d(tc);
    ta = wave_sum_d(ta);
    const double yc = wi / tc;
    const double ya = has_avg ? wi / ta : 0.0;
    if (lane == 0) {
      if (io.tc) io.tc[i] = (float)(tc * (double)io.rowscale[i]);
      if (io.ta && has_avg) io.ta[i] = (float)(ta * (double)io.rowscale[i]);
      if (cg) {
        md.yrow[i] = yc;
        md.yrow[(size_t)md.n + i] = ya;
      }
      st[0] = fmax(st[0], yc);
      st[4] = fmax(st[4], ya);
    }
    // pass 2: residual terms, column maxima and sums (the average is folded)
    for (int base = 0; base < d; base += kWave * kLongUnroll) {
      float u[kLongUnroll], xcv[kLongUnroll], xav[kLongUnroll], z[kLongUnroll];
      int cv[kLongUnroll];
      double pcv[kLongUnroll], pav[kLongUnroll];
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int q = beg + min(base + lane + kWave * e, d - 1);
        cv[e] = md.col[q];
        u[e] = md.uh[q];
        xcv[e] = io.xc[q];
        xav[e] = has_avg ? io.xa[q] : 0.0f;
        z[e] = (has_avg && io.xanc) ? io.xanc[q] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        pcv[e] = io.pc[cv[e]];
        pav[e] = has_avg ? io.pa[cv[e]] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < kLongUnroll; ++e) {
        const int k = base + lane + kWave * e;
        if (k < d) {
          const int c = cv[e];
          const double uu = (double)u[e];
          const float xc = xcv[e];
          const double p = pcv[e];
          const double vc = uu * yc;
          const double rc = p - vc;
          if (rc > 0.0) {
            st[2] = fmax(st[2], rc);
            st[1] = fmax(st[1], (double)xc * rc);
          }
          st[3] = fmax(st[3], (double)xc);
          const unsigned int bc = ord_key((float)(vc - p));
          if (c < hot) atomicMax(&lMc[c], bc);
          else if (!cg) atomicMax(&xMc[c], bc);
          const float xa = xav[e];
          if (has_avg) {
            double pa = pav[e];
            if (wf != 0.0f) pa = (wf == 1.0f) ? p : pa + (p - pa) * (double)wf;
            const double va = uu * ya;
            const double ra = pa - va;
            if (ra > 0.0) {
              st[6] = fmax(st[6], ra);
              st[5] = fmax(st[5], (double)xa * ra);
            }
            st[7] = fmax(st[7], (double)xa);
            const unsigned int ba = ord_key((float)(va - pa));
            if (c < hot) atomicMax(&lMa[c], ba);
            else if (!cg) atomicMax(&xMa[c], ba);
            if (io.xanc) st[9] += (double)(xa - z[e]) * (double)(xa - z[e]);
          }
          if ((sum_avg || io.want_cc) && (c < hot || !cg)) {
            const double add = io.want_cc ? xc : xa;
            atomicAdd(c < hot ? &lcs[c] : &xcs[c], add);
          }
        }
      }
    }
  }
  __shared__ double red[kWaves][10];
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const double v = (q >= 8) ? wave_sum_d(st[q]) : wave_max_d(st[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  const int slotw = bin.wg_offset + wg;
  if (threadIdx.x < 10) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int w = 1; w < kWaves; ++w) v = (q >= 8) ? v + red[w][q] : fmax(v, red[w][q]);
    md.rowpart[(size_t)slotw * kEvalRowStats + q] = v;
  }
  if (LDS_MODE == 1) {
    unsigned int *dMc = gMc + (size_t)slotw * hot;
    unsigned int *dMa = gMa + (size_t)slotw * hot;
    double *dcs = io.evalcs + (size_t)slotw * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      dMc[j] = lMc[j];
      dMa[j] = lMa[j];
      dcs[j] = lcs[j];
    }
  }
}

// Reverse of the row prox for long rows (same as k_adj_row).
template <int LDS_MODE>
__global__ __launch_bounds__(kRowBlock) void k_adj_long(MarketDev md, BinDev bin, AdjIO io) {
  extern __shared__ double lcs[];
  const int hot = LDS_MODE ? md.hot : 0;
  if (LDS_MODE) {
    for (int j = threadIdx.x; j < hot; j += blockDim.x) lcs[j] = 0.0;
    __syncthreads();
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  constexpr int kWaves = kRowBlock / kWave;
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  const double tau = io.tau;
  for (int slot = row_lo + wave; slot < row_hi; slot += kWaves) {
    const int i = bin.rows ? bin.rows[slot] : slot;
    const int beg = md.row_ptr[i];
    const int d = md.row_ptr[i + 1] - beg;
    const double tw = tau * (double)md.w[i];
    // entries in chunks of kWave * kLongUnroll, every load of a chunk issued
    // before any is used or any store of the chunk
    constexpr int U = kLongUnroll;
    double s = 0.0, Q = 0.0, Gu = 0.0;
    for (int base = 0; base < d; base += kWave * U) {
      float xn[U], uu[U], rin[U];
      int c[U];
      double bj[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int q = beg + min(base + lane + kWave * e, d - 1);
        xn[e] = io.xn[q];
        uu[e] = md.uh[q];
        rin[e] = io.r_in[q];
        c[e] = md.col[q];
      }
#pragma unroll
      for (int e = 0; e < U; ++e) bj[e] = io.b[c[e]];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        if (base + lane + kWave * e < d && xn[e] > 0.0f) {
          const double u = (double)uu[e];
          const double g = (double)rin[e] + bj[e];
          s = fma(u, (double)xn[e], s);
          Q = fma(u, u, Q);
          Gu = fma(u, g, Gu);
        }
      }
    }
    s = wave_sum_d(s);
    Q = wave_sum_d(Q);
    Gu = wave_sum_d(Gu);
    const bool live = s > 0.0;
    const double is = live ? fast_rcp(s) : 0.0;
    const double tws2 = tw * is * is;
    const double h = live ? tws2 * Gu / (1.0 + tws2 * Q) : 0.0;
    double ru = 0.0;
    for (int base = 0; base < d; base += kWave * U) {
      float xn[U], uu[U], rin[U], du[U];
      int c[U];
      double bj[U];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int q = beg + min(base + lane + kWave * e, d - 1);
        xn[e] = io.xn[q];
        uu[e] = md.uh[q];
        rin[e] = io.r_in[q];
        c[e] = md.col[q];
        du[e] = io.duh[q];
      }
#pragma unroll
      for (int e = 0; e < U; ++e) bj[e] = io.b[c[e]];
#pragma unroll
      for (int e = 0; e < U; ++e) {
        const int k = base + lane + kWave * e;
        if (k < d) {
          const int q = beg + k;
          const double u = (double)uu[e];
          const bool act = live && xn[e] > 0.0f;
          const double rr = act ? (double)rin[e] + bj[e] - h * u : 0.0;
          io.r_out[q] = (float)rr;
          if (act) io.duh[q] = du[e] + (float)(rr * tw * is - h * (double)xn[e]);
          ru = fma(rr, u, ru);
          atomicAdd(c[e] < hot ? &lcs[c[e]] : &io.csum[c[e]], rr);
        }
      }
    }
    ru = wave_sum_d(ru);
    if (live && lane == 0) io.dw[i] += (float)(tau * is * ru);
  }
  if (LDS_MODE) {
    __syncthreads();
    double *dst = md.colpart + (size_t)(bin.wg_offset + wg) * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) dst[j] = lcs[j];
  }
}

// ------------------------------------------------------------- launchers --

hipError_t launch_row_long(const MarketDev &md, const BinDev &bin, int lds_mode, const RowIO &io,
                           int nwg, hipStream_t st) {
  const size_t lh = (lds_mode & 4) ? (size_t)md.hot : (size_t)md.m;
  const size_t shm = lh * (((lds_mode & 2) ? sizeof(double) : 0) +
                           ((lds_mode & 1) ? sizeof(double) : 0));
  switch (lds_mode) {
    case 0: hipLaunchKernelGGL(k_row_long<0>, dim3(nwg), dim3(kLongBlock), shm, st, md, bin, io); break;
    case 1: hipLaunchKernelGGL(k_row_long<1>, dim3(nwg), dim3(kLongBlock), shm, st, md, bin, io); break;
    case 3: hipLaunchKernelGGL(k_row_long<3>, dim3(nwg), dim3(kLongBlock), shm, st, md, bin, io); break;
    case 7: hipLaunchKernelGGL(k_row_long<7>, dim3(nwg), dim3(kLongBlock), shm, st, md, bin, io); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_eval_long(const MarketDev &md, const BinDev &bin, int lds_mode,
                            const EvalIO &io, int nwg, int total_wg, hipStream_t st) {
  const size_t shm = lds_mode ? (size_t)md.hot * (sizeof(double) + 2 * sizeof(uint32_t)) : 0;
  if (lds_mode)
    hipLaunchKernelGGL(k_eval_long<1>, dim3(nwg), dim3(kRowBlock), shm, st, md, bin, io, total_wg);
  else
    hipLaunchKernelGGL(k_eval_long<0>, dim3(nwg), dim3(kRowBlock), shm, st, md, bin, io, total_wg);
  return hipGetLastError();
}

hipError_t launch_adj_long(const MarketDev &md, const BinDev &bin, int lds, const AdjIO &io,
                           int nwg, hipStream_t st) {
  const size_t shm = lds ? (size_t)md.hot * sizeof(double) : 0;
  if (lds)
    hipLaunchKernelGGL(k_adj_long<1>, dim3(nwg), dim3(kRowBlock), shm, st, md, bin, io);
  else
    hipLaunchKernelGGL(k_adj_long<0>, dim3(nwg), dim3(kRowBlock), shm, st, md, bin, io);
  return hipGetLastError();
}

}  // namespace pdhcg
