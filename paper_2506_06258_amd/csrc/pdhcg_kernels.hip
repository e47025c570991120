// HIP kernels (gfx950) of restarted PDHCG for linear Fisher markets.
//
// One iteration of Alg. 2 is a few launches that read the device-resident
// solver state (DevState):
//   k_pstep      price step p_try = p + sigma (2 c - c_prev - 1)  (eq. update:py)
//                and the lagged fold of the kept price into its average;
//   k_row_pass   every buyer's prox subproblem (Sec. 2.2) on its CSR row,
//                the lagged fold of the kept allocation into its average,
//                |x_try - x|^2 and per-workgroup column sums of x_try (one
//                launch per row-shape bin; rows above 512 entries in
//                pdhcg_long.hip);
//   k_cold_sums  column sums of the goods beyond the LDS (relabelled markets);
//   k_col_chunks, k_col_decide
//                float64 column sums from the workgroup partials, dp^T K dx
//                and |dp|^2 per column tile;
//   k_step_rule  the step-size rule (Sec. 5): keep or reject the trial,
//                rotate buffer roles, next eta.
// Every eval_every iterations k_eval_row / k_eval_chunks / k_eval_col /
// k_eval_final compute the relative KKT error (Sec. 5 Criteria) of the
// current and averaged points in float64.
//
// Memory layout: CSR row_ptr/col int32, values float32 aligned with col.
// A row is owned by a segment of G lanes of one wave (G in 4..64); lane r of
// the segment holds the row entries r, r+G, ..., r+(E-1)G in registers for
// the whole search, so the row is read from HBM once per iteration.  Loads
// of a segment are contiguous.  Column sums are privatised per workgroup in
// LDS and reduced in float64 by the column kernels.
#include "pdhcg_internal.h"
#include "pdhcg_device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>

namespace pdhcg {

// Bounds of the row in one slot of a bin, as loaded.  Three loads for every
// bin kind (the row id is a dummy load without an index list), so that the
// number of memory instructions a wave issues never depends on data: the
// vector memory counters of CDNA retire in issue order, and a wait for an
// older load after a branch that may skip newer ones has to wait for all of
// them.  Slots past the end read the last slot of the range.
struct RowBounds {
  int id, lo, hi;
};

__device__ __forceinline__ RowBounds fetch_bounds(const BinDev &bin, const int32_t *ids,
                                                  int slot, int slot_last) {
  const int sl = min(slot, slot_last);
  RowBounds rb;
  rb.id = ids[sl];
  rb.lo = bin.rlo[sl];
  rb.hi = bin.rhi[sl];
  return rb;
}

// Per-edge arrays are addressed through buffer resources with 32-bit byte
// offsets: one offset register per lane and row, the entry index folded into
// the instruction's immediate offset.  An access at or beyond the resource's
// size is dropped (store) or returns zero (load), so idle lanes store to
// kOutOfRange instead of branching, and a resource of size zero turns every
// access into a no-op.  Market creation keeps nnz <= kMaxBufferEntries.
constexpr uint32_t kOutOfRange = 0x80000000u;
constexpr uint32_t kBufWord3 = 0x00020000u;  // raw 32-bit buffer (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                           (int)kBufWord3);
}
__device__ __forceinline__ float bload_f(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __uint_as_float(
      __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ int bload_i(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
__device__ __forceinline__ int bload_u16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (int)__builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
}
__device__ __forceinline__ void bstore_f(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}

// The E entries lane r of a segment holds, as loaded: slots past the row end
// hold whatever follows the row (or zero past the array); the consumer
// masks them.
template <int E>
struct RowRegs {
  float u[E], x[E];
  int c[E];
};

// off: byte offset of the lane's first entry in the 4-byte arrays; with C16
// the good ids are 2-byte (offset off / 2).
template <int G, int E, bool C16>
__device__ __forceinline__ void row_fetch(uint32_t off, __amdgpu_buffer_rsrc_t ru,
                                          __amdgpu_buffer_rsrc_t rc,
                                          __amdgpu_buffer_rsrc_t rx, RowRegs<E> &R) {
#pragma unroll
  for (int e = 0; e < E; ++e) {
    R.u[e] = bload_f(ru, off + 4u * G * e);
    R.x[e] = bload_f(rx, off + 4u * G * e);
    R.c[e] = C16 ? bload_u16(rc, (off >> 1) + 2u * G * e) : bload_i(rc, off + 4u * G * e);
  }
}

// Software pipeline per wave, two passes deep: while the rows of pass t are
// searched, the entries of pass t+1 and the bounds of pass t+2 are loading,
// so each wave keeps a pass of HBM reads in flight through its compute
// phase.  Loads are issued in the order they are consumed (prices and
// averaged allocation of pass t, then the prefetch), the two register sets
// swap roles between the two halves of the loop body (no copies of loaded
// registers, which would wait for them), and no memory instruction sits
// behind a data-dependent branch.
template <int G, int E, int MODE, int LDS_MODE>
__global__ __launch_bounds__(kRowBlock) void k_row_pass(MarketDev md, BinDev bin,
                                                        RowIO io) {
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
  // LDS holds lh goods: all of them, or with LDS_MODE & 4 the goods [0, hot)
  // plus one idle slot (the goods from hot on use global memory)
  constexpr bool kHybrid = (LDS_MODE & 4) != 0;
  const int hot = kHybrid ? md.hot : m;
  const int lh = kHybrid ? hot + 1 : m;
  double *lp = lds_d;  // [lh] prices (LDS_MODE & 2)
  double *lc = (LDS_MODE & 2) ? lds_d + lh : lds_d;  // [lh] column partials
  if (LDS_MODE != 0) {
    for (int j = threadIdx.x; j < lh; j += blockDim.x) {
      if (LDS_MODE & 2) lp[j] = j < hot ? pp[j] : 0.0;
      if (LDS_MODE & 1) lc[j] = 0.0;
    }
    __syncthreads();
  }

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int r = lane & (G - 1);         // lane inside the segment
  const int seg = lane / G;             // segment inside the wave
  constexpr int kSeg = kWave / G;       // rows per wave pass
  constexpr int kWaves = kRowBlock / kWave;
  constexpr int kStep = kWaves * kSeg;  // rows per workgroup pass
  const int wg = blockIdx.x;
  // passes of kStep consecutive rows, workgroup w taking passes w, w + grid,
  // w + 2 grid, ...: the workgroups sweep the arrays together, which keeps
  // the HBM traffic of the chip in a narrow window (measured 4% faster than
  // a block of consecutive rows per workgroup on the 1e8-edge market)
  const int row_lo = wg * kStep;
  const int row_hi = bin.nrows;
  const int stride = (int)gridDim.x * kStep;
  const int last = row_hi - 1;
  const double rtol = io.rtol;
  const bool fold = wfold != 0.0f;
  const bool fold_read = fold && wfold != 1.0f;  // weight 1 replaces the average
  const int32_t *ids = bin.rows ? bin.rows : bin.rlo;
  const uint32_t ebytes = (uint32_t)md.nnz * 4u;
  const __amdgpu_buffer_rsrc_t ru = make_rsrc(md.uh, ebytes);
  // 2-byte good ids when every good sits in LDS (LDS modes 1 and 3)
  constexpr bool kC16 = (LDS_MODE == 1 || LDS_MODE == 3);
  const __amdgpu_buffer_rsrc_t rc =
      kC16 ? make_rsrc(md.col16, (uint32_t)md.nnz * 2u) : make_rsrc(md.col, ebytes);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(xin, ebytes);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(xout, ebytes);
  // the average is read only when folded with a weight below one, and
  // written only when folded
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(xavg, fold_read ? ebytes : 0u);
  const __amdgpu_buffer_rsrc_t ryw = make_rsrc(xavg, fold ? ebytes : 0u);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(io.s_out, io.s_out ? (uint32_t)md.n * 4u : 0u);
  // entries of the goods beyond LDS: their fixed slots in the panel buffer
  const bool slots = kHybrid && io.colsum && md.cslot != nullptr;
  const __amdgpu_buffer_rsrc_t rcs = make_rsrc(md.cslot, slots ? ebytes : 0u);
  const __amdgpu_buffer_rsrc_t rpv = make_rsrc(md.pval, slots ? ebytes : 0u);  // slots < nnz

  double dx2 = 0.0;  // |x_try - x|^2 of the lane's entries (float64, like the global sum)
  uint32_t rmax = 0;
  uint32_t rsum = 0, rcount = 0;

  int base = row_lo + wave * kSeg;
  auto row_id = [&](const RowBounds &rb, int slot) { return bin.rows ? rb.id : min(slot, last); };
  auto row_len = [&](const RowBounds &rb, int slot) { return slot < row_hi ? rb.hi - rb.lo : 0; };
  auto lane_off = [&](const RowBounds &rb) { return 4u * (uint32_t)(rb.lo + r); };

  // prologue: bounds of passes 0 and 1, entries and budget of pass 0, all
  // complete before the loop: the loop header is then entered with nothing
  // in flight from the prologue, and its wait counts are those of the back
  // edge alone.
  RowBounds bA = fetch_bounds(bin, ids, base + seg, last);
  RowBounds bB = fetch_bounds(bin, ids, base + stride + seg, last);
  RowRegs<E> RA, RB;
  int dA = row_len(bA, base + seg), dB = 0;
  row_fetch<G, E, kC16>(lane_off(bA), ru, rc, rx, RA);
  float wA = md.w[row_id(bA, base + seg)], wB = 0.0f;
  __builtin_amdgcn_s_waitcnt(0);

  // Head of a pass: gather the prices of its goods into a and load the
  // averaged allocation into y.
  double a[E];
  float y[E];
  int cs[E];
  auto head = [&](const RowRegs<E> &Rc, const RowBounds &bc) {
    if (kHybrid) {
      // both loads for every entry (no branch around a memory instruction):
      // LDS for the hot goods, global for the others (hot entries read the
      // price of good 0, one cached line)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int c = Rc.c[e];
        const bool hc = c < hot;
        const double vg = pp[hc ? 0 : c];
        const double vl = lp[hc ? c : hot];
        a[e] = hc ? vl : vg;
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) a[e] = (LDS_MODE & 2) ? lp[Rc.c[e]] : pp[Rc.c[e]];
    }
    const uint32_t off = lane_off(bc);
#pragma unroll
    for (int e = 0; e < E; ++e) y[e] = bload_f(ry, off + 4u * G * e);
    if (kHybrid) {
#pragma unroll
      for (int e = 0; e < E; ++e) cs[e] = slots ? bload_i(rcs, off + 4u * G * e) : -1;
    }
  };
  // Body of a pass: entries Rc (dc entries, budget wc, bounds bc) and its
  // prices are in flight or resident; bn holds the bounds of the next pass.
  // Loads the next pass into Rn, dn, wn and the bounds of the pass after
  // into bc, then solves and stores this pass.
  auto body = [&](const RowRegs<E> &Rc, RowBounds &bc, int dc, float wc, RowRegs<E> &Rn,
                  const RowBounds &bn, int &dn, float &wn) {
    const int slot = base + seg;
    const bool rv = slot < row_hi;
    const uint32_t off = lane_off(bc);
    const int rid = row_id(bc, slot);
    const int d = dc;
    dn = row_len(bn, slot + stride);
    row_fetch<G, E, kC16>(lane_off(bn), ru, rc, rx, Rn);
    wn = md.w[row_id(bn, slot + stride)];
    bc = fetch_bounds(bin, ids, slot + 2 * stride, last);

    const double tw = rv ? tau * (double)wc : 0.0;
    bool ok[E];
    float uh[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      ok[e] = r + G * e < d;
      uh[e] = ok[e] ? Rc.u[e] : 0.0f;
      a[e] = fma(-tau, a[e], (double)Rc.x[e]);  // x^k - tau p
    }
    int rounds = 0;
    const double sfin = prox_solve<G, E, MODE>(rv, tw, io.max_rounds, rtol, io.sections, ok, a,
                                               uh, Rc.x, rounds);
    // x^{k+1} = [a + b/s]_+ (eq. bisection), |x^{k+1} - x^k|^2, column sums,
    // and the lagged fold of the kept iterate into the running average
    // (Alg. 2).
    const double tf = tw * fast_rcp(sfin);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t o = (ok[e] ? off : kOutOfRange) + 4u * G * e;
      const float xk = Rc.x[e];
      const float xn = (float)fmax(fma((double)uh[e], tf, a[e]), 0.0);
      bstore_f(ro, o, xn);
      bstore_f(ryw, o, fold_read ? fmaf(xk - y[e], wfold, y[e]) : xk);
      const double df = ok[e] ? (double)xn - (double)xk : 0.0;
      dx2 = fma(df, df, dx2);
      if (io.colsum) {
        if (kHybrid) {
          // goods from hot on: to their panel slot (summed afterwards by
          // the panel kernels), or gathered by k_cold_sums
          const int c = Rc.c[e];
          const bool hc = c < hot;
          atomicAdd(&lc[hc ? c : hot], (ok[e] && hc) ? (double)xn : 0.0);
          bstore_f(rpv, (ok[e] && cs[e] >= 0) ? 4u * (uint32_t)cs[e] : kOutOfRange, xn);
        } else {
          atomicAdd((LDS_MODE & 1) ? &lc[Rc.c[e]] : &cglob[Rc.c[e]], ok[e] ? (double)xn : 0.0);
        }
      }
    }
    bstore_f(rs, (rv && r == 0) ? 4u * (uint32_t)rid : kOutOfRange, (float)sfin);
    if (rv && r == 0) {
      rmax = max(rmax, (uint32_t)rounds);
      rsum += (uint32_t)rounds;
      rcount += 1;
    }
    base += stride;
  };

  while (base < row_hi) {
    head(RA, bA);
    body(RA, bA, dA, wA, RB, bB, dB, wB);
    if (base >= row_hi) break;
    head(RB, bB);
    body(RB, bB, dB, wB, RA, bA, dA, wA);
  }

  // Workgroup partials.
  __shared__ double red[kWaves];
  __shared__ uint32_t red_rmax, red_rsum, red_rcnt;
  if (threadIdx.x == 0) {
    red_rmax = 0;
    red_rsum = 0;
    red_rcnt = 0;
  }
  double dsum = wave_sum_d(dx2);
  __syncthreads();
  if (lane == 0) red[wave] = dsum;
  if (rcount) {
    atomicMax(&red_rmax, rmax);
    atomicAdd(&red_rsum, rsum);
    atomicAdd(&red_rcnt, rcount);
  }
  __syncthreads();
  const int slot = bin.wg_offset + wg;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[q];
    if (md.rowpart) {
      md.rowpart[(size_t)slot * kRowStats + 0] = t;
    }
    if (io.use_state) {
      atomicMax(&md.S->rounds_max, red_rmax);
      atomicAdd((unsigned long long *)&md.S->rounds_sum, (unsigned long long)red_rsum);
      atomicAdd((unsigned long long *)&md.S->rows_searched, (unsigned long long)red_rcnt);
    }
  }
  if ((LDS_MODE & 1) && io.colsum) {
    double *dst = md.colpart + (size_t)slot * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) dst[j] = lc[j];
  }
}

// ------------------------------------------------------------ price step ---

__global__ __launch_bounds__(kColBlock) void k_pstep(MarketDev md, int zero_ctry) {
  const DevState *S = md.S;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= md.m) return;
  const double *pc = pick3<double *>(md.P0, md.P1, md.P2, S->ip[0]);
  double *pt = pick3<double *>(md.P0, md.P1, md.P2, S->ip[1]);
  double *pa = pick3<double *>(md.P0, md.P1, md.P2, S->ip[2]);
  const double *cprev = pick3<double *>(md.C0, md.C1, md.C2, S->ic[0]);
  const double *ccur = pick3<double *>(md.C0, md.C1, md.C2, S->ic[1]);
  double *ctry = pick3<double *>(md.C0, md.C1, md.C2, S->ic[2]);
  const double p = pc[j];
  pt[j] = p + S->sigma * (2.0 * ccur[j] - cprev[j] - 1.0);
  if (S->fold) {
    const double q = pa[j];
    pa[j] = (S->k_in == 1) ? p : q + (p - q) / (double)S->k_in;
  }
  if (zero_ctry) ctry[j] = 0.0;
}

// ---------------------------------------------- column sums + step rule ----

// Column sums (deterministic float64: partial rows in chunks, chunks in a
// fixed order), the tiles' dp^T (c_try - c) and |dp|^2, and the step rule,
// in kernels of their own so that results pass through kernel boundaries.
// Column sums of the goods from hot on: a segment of GC lanes per good
// (GC picked from the goods' mean degree), its entries (in row order)
// gathered from the allocation in chunks of 4 per lane and added in float64
// in a fixed order.  Replaces device atomics for these goods, whose
// scattered read-modify-writes ran at about 22 G/s.
template <int GC>
__global__ __launch_bounds__(256) void k_cold_sums(MarketDev md, int use_state, const float *x,
                                                   double *out) {
  if (use_state) {
    const DevState *S = md.S;
    x = pick3<float *>(md.X0, md.X1, md.X2, S->ix[1]);
    out = pick3<double *>(md.C0, md.C1, md.C2, S->ic[2]);
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane & (GC - 1);
  const int ncold = md.m - md.hot;
  const int segs = (int)(gridDim.x * (blockDim.x / GC));
  // goods of a wave's segments are consecutive, so every segment of a wave
  // runs the same number of trips as long as degrees are alike; the trip
  // count is the wave's maximum (segments past their good add nothing)
  for (int g0 = (blockIdx.x * blockDim.x + threadIdx.x - r) / GC; g0 - (lane / GC) < ncold;
       g0 += segs) {
    const int g = g0;
    const bool gv = g < ncold;
    const int b = gv ? md.cold_ptr[g] : 0, e = gv ? md.cold_ptr[g + 1] : 0;
    double acc = 0.0;
    int trips = (e - b + 4 * GC - 1) / (4 * GC);
    for (int o = 1; o < kWave / GC; o <<= 1) trips = max(trips, __shfl_xor(trips, o * GC));
    for (int t0 = 0; t0 < trips; ++t0) {
      const int k0 = b + r + t0 * 4 * GC;
      int q[4];
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) q[t] = (k0 + t * GC < e) ? md.cold_idx[k0 + t * GC] : -1;
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = q[t] >= 0 ? x[q[t]] : 0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) acc += (double)v[t];
    }
    acc = seg_sum_d<GC>(acc);
    if (gv && r == 0) out[md.hot + g] = acc;
  }
}

// KKT column quantities of the goods from hot on (relabelled markets) from
// their entry lists: a segment of GC lanes per good runs over the good's
// entries (in row order, 4 loads in flight per lane), forms the same keys
// ord_key(u_ij y_i - p_j) as the KKT row kernels (y_i from yrow, prices
// folded the same way) and the float64 sum of the entries of the averaged
// point (or of the current one when want_cc), and writes the good's maxima
// and sum to io.gmax / io.gsum.  The row kernels leave these goods to it.
template <int GC>
__global__ __launch_bounds__(256) void k_eval_cold(MarketDev md, EvalIO io) {
  const int lane = threadIdx.x & (kWave - 1);
  const int r = lane & (GC - 1);
  const int m = md.m, hot = md.hot, ncold = m - hot;
  const size_t n = (size_t)md.n;
  const bool has_avg = io.xa != nullptr;
  const bool want_sum = (has_avg && !io.want_cc) || io.want_cc;
  const float wf = io.wfold;
  const int segs = (int)(gridDim.x * (blockDim.x / GC));
  // as in k_cold_sums: the segments of a wave run the wave's largest trip count
  for (int g0 = (blockIdx.x * blockDim.x + threadIdx.x - r) / GC; g0 - (lane / GC) < ncold;
       g0 += segs) {
    const int g = g0;
    const bool gv = g < ncold;
    const int j = hot + (gv ? g : 0);
    const int b = gv ? md.ecold_ptr[g] : 0, e = gv ? md.ecold_ptr[g + 1] : 0;
    const double p = io.pc[j];
    double pa = has_avg ? io.pa[j] : 0.0;
    if (has_avg && wf != 0.0f) pa = (wf == 1.0f) ? p : pa + (p - pa) * (double)wf;
    unsigned int kc = 0u, ka = 0u;
    double acc = 0.0;
    int trips = (e - b + 4 * GC - 1) / (4 * GC);
    for (int o = 1; o < kWave / GC; o <<= 1) trips = max(trips, __shfl_xor(trips, o * GC));
    for (int t0 = 0; t0 < trips; ++t0) {
      const int k0 = b + r + t0 * 4 * GC;
      int q[4], row[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool ok = k0 + t * GC < e;
        q[t] = ok ? md.ecold_idx[k0 + t * GC] : -1;
        row[t] = ok ? md.ecold_row[k0 + t * GC] : 0;
      }
      float u[4], xc[4], xa[4];
      double yc[4], ya[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = q[t] >= 0 ? q[t] : 0;
        u[t] = md.uh[k];
        xc[t] = io.xc[k];
        xa[t] = has_avg ? io.xa[k] : 0.0f;
        yc[t] = md.yrow[row[t]];
        ya[t] = has_avg ? md.yrow[n + row[t]] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (q[t] < 0) continue;
        const double vc = (double)u[t] * yc[t];
        kc = max(kc, ord_key((float)(vc - p)));
        if (has_avg) {
          const double va = (double)u[t] * ya[t];
          ka = max(ka, ord_key((float)(va - pa)));
        }
        if (want_sum) acc += (double)(io.want_cc ? xc[t] : xa[t]);
      }
    }
    for (int o = 1; o < GC; o <<= 1) {
      kc = max(kc, (unsigned int)__shfl_xor((int)kc, o));
      ka = max(ka, (unsigned int)__shfl_xor((int)ka, o));
    }
    acc = seg_sum_d<GC>(acc);
    if (gv && r == 0) {
      io.gmax[j] = kc;
      if (has_avg) io.gmax[(size_t)m + j] = ka;
      if (want_sum) io.gsum[j] = acc;
    }
  }
}

// Chunk sums of the per-workgroup column partials: block (t, q) adds the
// partial rows of chunk q for tile t's goods (partial rows cover the goods
// [0, hot): all goods unless the market is hybrid, where the others are
// summed by device atomics in c_try).  A kernel of its own, so that the sums
// reach k_col_decide through the kernel boundary rather than a device-scope
// fence per block (on gfx950 a fence writes back and invalidates the L2).
__global__ __launch_bounds__(kColBlock) void k_col_chunks(MarketDev md, int total_wg) {
  const int hot = md.hot;
  const int q = blockIdx.y, nq = gridDim.y;
  const int j = blockIdx.x * kColBlock + threadIdx.x;
  if (j >= hot) return;
  const int per = (total_wg + nq - 1) / nq;
  const int b0 = q * per, b1 = min(total_wg, b0 + per);
  double c = 0.0;
  const double *src = md.colpart + j;
  int b = b0;
  for (; b + 8 <= b1; b += 8) {  // eight loads in flight per thread
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = src[(size_t)(b + t) * hot];
    c += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  for (; b < b1; ++b) c += src[(size_t)b * hot];
  md.colchunk[(size_t)q * md.m + j] = c;
}

// c_try from the chunk sums (nq chunks, fixed order), dp^T (c_try - c) and
// |dp|^2 per block (the step rule follows in k_step_rule).  With ppart the
// goods from hot on also take their panel partial sums (pchunks chunks per
// panel, in chunk order), added to what k_cold_sums wrote when pacc, so the
// panels need no summing kernel of their own.
__global__ __launch_bounds__(kColBlock) void k_col_decide(MarketDev md, int total_wg, int nq,
                                                          const double *ppart, int pchunks,
                                                          int pacc) {
  DevState *S = md.S;
  const int m = md.m;
  const int tile = blockIdx.x;
  const int j = tile * kColBlock + threadIdx.x;
  const double *pc = pick3<double *>(md.P0, md.P1, md.P2, S->ip[0]);
  const double *pt = pick3<double *>(md.P0, md.P1, md.P2, S->ip[1]);
  const double *ccur = pick3<double *>(md.C0, md.C1, md.C2, S->ic[1]);
  double *ctry = pick3<double *>(md.C0, md.C1, md.C2, S->ic[2]);
  // every load issued before the sums (which keep the chunk order)
  if (nq > 0 && j < md.hot) {
    double v[kColChunks];
#pragma unroll
    for (int k = 0; k < kColChunks; ++k) v[k] = k < nq ? md.colchunk[(size_t)k * m + j] : 0.0;
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kColChunks; ++k) c += v[k];
    ctry[j] = c;
  }
  if (ppart && j >= md.hot && j < m) {
    const int g = j - md.hot;
    const double *src = ppart + (size_t)(g >> kPanelShift) * pchunks * kPanelW + (g & (kPanelW - 1));
    double s = 0.0;
    for (int r0 = 0; r0 < pchunks; r0 += 8) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = r0 + t < pchunks ? src[(size_t)(r0 + t) * kPanelW] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) s += v[t];
    }
    ctry[j] = pacc ? ctry[j] + s : s;
  }
  double inter = 0.0, dp2 = 0.0;
  if (j < m) {
    const double c = ctry[j];
    const double dp = pt[j] - pc[j];
    inter = dp * (c - ccur[j]);
    dp2 = dp * dp;
  }
  __shared__ double sh[2][kColBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  inter = wave_sum_d(inter);
  dp2 = wave_sum_d(dp2);
  if (lane == 0) {
    sh[0][wave] = inter;
    sh[1][wave] = dp2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, qq = 0.0;
    for (int w = 0; w < kColBlock / kWave; ++w) {
      a += sh[0][w];
      qq += sh[1][w];
    }
    md.colblk[(size_t)tile * kColStats + 0] = a;
    md.colblk[(size_t)tile * kColStats + 1] = qq;
  }
}

// Global sums and the step-size rule, in one block after k_col_decide (the
// block statistics arrive through the kernel boundary).
// With pdhg = 1 (restarted PDHG, Alg. 1) the workgroup partials also hold
// |dy|^2 (slot 1) and dy^T (dt - U dx) (slot 2), and slot 0 includes |dt|^2:
// the primal norm is over (x, t), the dual norm over (p, y), and the
// interaction is (dp, dy)^T K (dx, dt) with K = [1^T 0; -U I].
__global__ __launch_bounds__(kColBlock) void k_step_rule(MarketDev md, int total_wg, int tiles,
                                                         int pdhg) {
  DevState *S = md.S;
  __shared__ double sh[2][kColBlock / kWave];
  __shared__ double shx[kColBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  double a = 0.0, qq = 0.0, x2 = 0.0;
  for (int b = threadIdx.x; b < tiles; b += blockDim.x) {
    a += md.colblk[(size_t)b * kColStats + 0];
    qq += md.colblk[(size_t)b * kColStats + 1];
  }
  for (int b = threadIdx.x; b < total_wg; b += blockDim.x) {
    x2 += md.rowpart[(size_t)b * kRowStats];
    if (pdhg) {
      qq += md.rowpart[(size_t)b * kRowStats + 1];
      a += md.rowpart[(size_t)b * kRowStats + 2];
    }
  }
  a = wave_sum_d(a);
  qq = wave_sum_d(qq);
  x2 = wave_sum_d(x2);
  __syncthreads();
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = qq;
    shx[wave] = x2;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = qq = x2 = 0.0;
  for (int w = 0; w < kColBlock / kWave; ++w) {
    a += sh[0][w];
    qq += sh[1][w];
    x2 += shx[w];
  }
  S->total += 1;
  S->since += 1;
  bool accept = true;
  if (S->step_mode == 1) {
    // Adaptive step (Sec. 5): keep the trial when
    // eta <= (omega |dx|^2 + |dp|^2 / omega) / (2 |dp^T K dx|).
    const double om = S->omega, eta = S->eta;
    const double emax = fabs(a) > 0.0 ? (om * x2 + qq / om) / (2.0 * fabs(a)) : INFINITY;
    const double kk = (double)(S->total + 1);
    double enew = fmin((1.0 - pow(kk, -0.3)) * emax, (1.0 + pow(kk, -0.6)) * eta);
    enew = fmin(fmax(enew, S->eta_lo), S->eta_hi);
    accept = (eta <= emax) || (eta <= S->eta_lo);
    S->emax_last = emax;
    S->eta = enew;
    S->tau = enew / om;
    S->sigma = enew * om;
  }
  if (accept) {
    int t = S->ix[0]; S->ix[0] = S->ix[1]; S->ix[1] = t;
    t = S->ip[0]; S->ip[0] = S->ip[1]; S->ip[1] = t;
    const int cp = S->ic[0], cc = S->ic[1], ct = S->ic[2];
    S->ic[0] = cc; S->ic[1] = ct; S->ic[2] = cp;
    S->k_in += 1;
    S->accepted += 1;
    S->fold = 1;
  } else {
    S->fold = 0;
  }
  S->accept_last = accept ? 1 : 0;
}

// ---------------------------------------------------------- KKT row pass ---

// Per workgroup row statistics (float64):
//  0 max y_c, 1 max gap_c, 2 max (p - u y)_+ c, 3 max x_c,
//  4 max y_a, 5 max gap_a, 6 max (p - u y)_+ a, 7 max x_a,
//  8 |x_c - anchor|^2, 9 |x_a - anchor|^2
// Column quantities: the column maxima of u_ij y_i - p_j for both points
// (as ord_key keys, max-reduced as unsigned) and the column sums of the
// averaged point (or of the current point when want_cc).
// LDS_MODE 1: per-workgroup partials in LDS (float64 sums: float32 LDS
// atomic adds are slow on gfx950), written to evalpart [2][total_wg][m]
// (maxima) and evalcs [total_wg][m] (sums).  LDS_MODE 0: device-wide atomics
// into evalpart [2][m] (maxima) and io.cacc [m] (float64 sums), all zeroed by
// the caller.
template <int G, int E, int LDS_MODE>
__global__ __launch_bounds__(kRowBlock) void k_eval_row(MarketDev md, BinDev bin,
                                                        EvalIO io, int total_wg) {
  extern __shared__ double lds_e[];
  const int m = md.m;
  const bool has_avg = io.xa != nullptr;
  const bool sum_avg = has_avg && !io.want_cc;
  // LDS mode: goods [0, hot) in LDS, the others in the device-wide
  // accumulators io.gmax / io.gsum, or (with the lists ecold_*) left to
  // k_eval_cold, which takes the rows' y from yrow
  const int hot = (LDS_MODE == 1) ? md.hot : 0;
  const bool cg = (LDS_MODE == 1) && md.ecold_ptr != nullptr;
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
  const int r = lane & (G - 1);
  const int seg = lane / G;
  constexpr int kSeg = kWave / G;
  constexpr int kWaves = kRowBlock / kWave;
  const int wg = blockIdx.x;
  const int row_lo = wg * bin.rows_per_wg;
  const int row_hi = min(row_lo + bin.rows_per_wg, bin.nrows);
  const float wf = io.wfold;

  double st[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) st[q] = 0.0;

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
    double tc = 0.0, ta = 0.0;
    // every load of the pass first (indices clamped to the row start, slots
    // past the row end masked), then the price gathers, then the fold and
    // its stores: a store between loads would order every later load after
    // it
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
#pragma unroll
    for (int e = 0; e < E; ++e) {
      pcj[e] = io.pc[cj[e]];
      paj[e] = has_avg ? io.pa[cj[e]] : 0.0;
    }
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
        q = (wf == 1.0f) ? pcj[e] : q + (pcj[e] - q) * (double)wf;
      }
      xa[e] = y;
      paj[e] = q;
      if (io.xanc) {
        const float z = xz[e];
        st[8] += (double)(x - z) * (double)(x - z);
        if (has_avg) st[9] += (double)(y - z) * (double)(y - z);
      }
      tc += (double)uh[e] * (double)x;
      ta += (double)uh[e] * (double)y;
    }
    tc = seg_sum_d<G>(tc);
    ta = seg_sum_d<G>(ta);
    const double yc = rv ? wi / tc : 0.0;
    const double ya = (rv && has_avg) ? wi / ta : 0.0;
    if (rv && r == 0) {
      if (io.tc) io.tc[i] = (float)(tc * (double)io.rowscale[i]);
      if (io.ta && has_avg) io.ta[i] = (float)(ta * (double)io.rowscale[i]);
      if (cg) {
        md.yrow[i] = yc;
        md.yrow[(size_t)md.n + i] = ya;
      }
      st[0] = fmax(st[0], yc);
      st[4] = fmax(st[4], ya);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = r + G * e;
      if (idx < d) {
        const int c = cj[e];
        const double vc = (double)uh[e] * yc;
        const double rc = pcj[e] - vc;
        if (rc > 0.0) {
          st[2] = fmax(st[2], rc);
          st[1] = fmax(st[1], (double)xc[e] * rc);
        }
        st[3] = fmax(st[3], (double)xc[e]);
        const unsigned int bc = ord_key((float)(vc - pcj[e]));
        if (c < hot) atomicMax(&lMc[c], bc);
        else if (!cg) atomicMax(&xMc[c], bc);
        if (has_avg) {
          const double va = (double)uh[e] * ya;
          const double ra = paj[e] - va;
          if (ra > 0.0) {
            st[6] = fmax(st[6], ra);
            st[5] = fmax(st[5], (double)xa[e] * ra);
          }
          st[7] = fmax(st[7], (double)xa[e]);
          const unsigned int ba = ord_key((float)(va - paj[e]));
          if (c < hot) atomicMax(&lMa[c], ba);
          else if (!cg) atomicMax(&xMa[c], ba);
        }
        if ((sum_avg || io.want_cc) && (c < hot || !cg)) {
          const double add = io.want_cc ? xc[e] : xa[e];
          atomicAdd(c < hot ? &lcs[c] : &xcs[c], add);
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
  const int slot = bin.wg_offset + wg;
  if (threadIdx.x < 10) {
    const int q = threadIdx.x;
    double v = red[0][q];
    for (int w = 1; w < kWaves; ++w) v = (q >= 8) ? v + red[w][q] : fmax(v, red[w][q]);
    md.rowpart[(size_t)slot * kEvalRowStats + q] = v;
  }
  if (LDS_MODE == 1) {
    unsigned int *dMc = gMc + (size_t)slot * hot;
    unsigned int *dMa = gMa + (size_t)slot * hot;
    double *dcs = io.evalcs + (size_t)slot * hot;
    for (int j = threadIdx.x; j < hot; j += blockDim.x) {
      dMc[j] = lMc[j];
      dMa[j] = lMa[j];
      dcs[j] = lcs[j];
    }
  }
}

// ------------------------------------------------------- KKT column pass ---

// Per-workgroup KKT partials reduced in kColChunks chunks of workgroups:
// block (t, q) covers tile t's columns and workgroups [q per, (q+1) per);
// maxima into evalchunk [2][kColChunks][m], sums (float64, fixed order) into
// cacc [kColChunks][m].
__global__ __launch_bounds__(kColBlock) void k_eval_chunks(MarketDev md, EvalIO io,
                                                           int total_wg) {
  const int m = md.m, hot = md.hot;
  const int j = blockIdx.x * kColBlock + threadIdx.x;
  const int q = blockIdx.y;
  if (j >= hot) return;
  const bool has_avg = io.xa != nullptr;
  const bool want_sum = (has_avg && !io.want_cc) || io.want_cc;
  const size_t TW = (size_t)total_wg * hot;
  const int per = (total_wg + kColChunks - 1) / kColChunks;
  const int b0 = q * per, b1 = min(total_wg, b0 + per);
  const unsigned int *sMc = reinterpret_cast<const unsigned int *>(io.evalpart) + j;
  const unsigned int *sMa = reinterpret_cast<const unsigned int *>(io.evalpart + TW) + j;
  unsigned int bMc = 0u, bMa = 0u;
  double cs = 0.0;
  for (int b = b0; b < b1; ++b) {
    bMc = max(bMc, sMc[(size_t)b * hot]);
    if (has_avg) bMa = max(bMa, sMa[(size_t)b * hot]);
    if (want_sum) cs += io.evalcs[(size_t)b * hot + j];
  }
  io.evalchunk[(size_t)q * m + j] = bMc;
  io.evalchunk[(size_t)(kColChunks + q) * m + j] = bMa;
  io.cacc[(size_t)q * m + j] = cs;
}

// Column statistics per block (float64):
//  0 max |c_c - 1|, 1 max |c_c|, 2 max (M_c - p_c)_+, 3 max (p_c - M_c),
//  4 max |c_a - 1|, 5 max |c_a|, 6 max (M_a - p_a)_+, 7 max (p_a - M_a),
//  8 |p_c - p_anchor|^2, 9 |p_a - p_anchor|^2
// The last block combines them with the row statistics into the relative
// KKT error of Sec. 5 and writes it, with the anchor distances, to DevState.
__global__ __launch_bounds__(kColBlock) void k_eval_col(MarketDev md, EvalIO io, int total_wg,
                                                        int partials) {
  const int m = md.m;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const bool has_avg = io.xa != nullptr;
  const bool sum_avg = has_avg && !io.want_cc;
  const size_t TW = partials ? (size_t)total_wg * m : (size_t)m;
  double st[10];
  for (int q = 0; q < 10; ++q) st[q] = 0.0;
  st[3] = -INFINITY;
  st[7] = -INFINITY;
  if (j < m) {
    unsigned int bMc = 0u, bMa = 0u;
    double cs = 0.0;
    const unsigned int *sMc = reinterpret_cast<const unsigned int *>(io.evalpart) + j;
    const unsigned int *sMa = reinterpret_cast<const unsigned int *>(io.evalpart + TW) + j;
    if (partials && j < md.hot) {
      // chunk results of k_eval_chunks, combined in a fixed order
      for (int q = 0; q < kColChunks; ++q) {
        bMc = max(bMc, io.evalchunk[(size_t)q * m + j]);
        if (has_avg) bMa = max(bMa, io.evalchunk[(size_t)(kColChunks + q) * m + j]);
        if (sum_avg || io.want_cc) cs += io.cacc[(size_t)q * m + j];
      }
    } else if (partials) {
      // goods from hot on: device-wide accumulators
      bMc = io.gmax[j];
      if (has_avg) bMa = io.gmax[m + j];
      if (sum_avg || io.want_cc) cs = io.gsum[j];
    } else {
      bMc = sMc[0];
      if (has_avg) bMa = sMa[0];
      if (sum_avg || io.want_cc) cs = io.cacc[j];
    }
    // column maxima of u y - p (keys of ord_key)
    const double Dc = (double)ord_dec(bMc);
    const double Da = (double)ord_dec(bMa);
    const double cc = io.want_cc ? cs : io.ccur[j];
    const double pc = io.pc[j];
    st[0] = fabs(cc - 1.0);
    st[1] = fabs(cc);
    st[2] = fmax(0.0, Dc);
    st[3] = -Dc;
    if (io.panc) st[8] = (pc - io.panc[j]) * (pc - io.panc[j]);
    if ((sum_avg || io.want_cc) && io.cavg_out) io.cavg_out[j] = cs;
    if (has_avg) {
      double q = io.pa[j];
      if (io.wfold != 0.0f) q = (io.wfold == 1.0f) ? pc : q + (pc - q) * (double)io.wfold;
      if (io.pa_out) io.pa_out[j] = q;
      const double pa = q;
      st[4] = fabs(cs - 1.0);
      st[5] = fabs(cs);
      st[6] = fmax(0.0, Da);
      st[7] = -Da;
      if (io.panc) st[9] = (pa - io.panc[j]) * (pa - io.panc[j]);
    }
  }
  __shared__ double red[kColBlock / kWave][10];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  for (int q = 0; q < 10; ++q) {
    const double v = (q >= 8) ? wave_sum_d(st[q]) : wave_max_d(st[q]);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 0; q < 10; ++q) {
      double v = red[0][q];
      for (int w = 1; w < kColBlock / kWave; ++w)
        v = (q >= 8) ? v + red[w][q] : fmax(v, red[w][q]);
      md.colblk[(size_t)blockIdx.x * kEvalColStats + q] = v;
    }
  }
}

// The relative KKT errors from the block statistics of k_eval_col and the
// workgroup statistics of the row kernels, in one block (both arrive
// through the kernel boundary).  Every thread combines a strided share,
// then a fixed-order block reduction.
__global__ __launch_bounds__(kColBlock) void k_eval_final(MarketDev md, int total_wg, int tiles) {
  DevState *S = md.S;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  double c[10], rw[10];
  for (int q = 0; q < 10; ++q) {
    c[q] = (q == 3 || q == 7) ? -INFINITY : 0.0;
    rw[q] = 0.0;
  }
  for (int b = threadIdx.x; b < tiles; b += blockDim.x)
    for (int q = 0; q < 10; ++q) {
      const double v = md.colblk[(size_t)b * kEvalColStats + q];
      c[q] = (q >= 8) ? c[q] + v : fmax(c[q], v);
    }
  for (int b = threadIdx.x; b < total_wg; b += blockDim.x)
    for (int q = 0; q < 10; ++q) {
      const double v = md.rowpart[(size_t)b * kEvalRowStats + q];
      rw[q] = (q >= 8) ? rw[q] + v : fmax(rw[q], v);
    }
  __shared__ double fin[2][kColBlock / kWave][10];
  for (int q = 0; q < 10; ++q) {
    const double cv = (q >= 8) ? wave_sum_d(c[q]) : wave_max_d(c[q]);
    const double rv = (q >= 8) ? wave_sum_d(rw[q]) : wave_max_d(rw[q]);
    if (lane == 0) {
      fin[0][wave][q] = cv;
      fin[1][wave][q] = rv;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 0; q < 10; ++q) {
    c[q] = fin[0][0][q];
    rw[q] = fin[1][0][q];
    for (int w = 1; w < kColBlock / kWave; ++w) {
      c[q] = (q >= 8) ? c[q] + fin[0][w][q] : fmax(c[q], fin[0][w][q]);
      rw[q] = (q >= 8) ? rw[q] + fin[1][w][q] : fmax(rw[q], fin[1][w][q]);
    }
  }
  // Relative KKT error (Sec. 5 Criteria) with t = Ux, y = w / t:
  //   r_primal = max|c - 1| / (1 + max(max|c|, 1))
  //   r_dual   = max (M - p)_+ / (1 + max(max y, max (p - M)))
  //   r_gap    = max x (p - u y)_+ / (1 + max(max x, max (p - u y)_+))
  for (int z = 0; z < 2; ++z) {
    const int o = 4 * z;
    S->kkt[z][0] = c[o + 0] / (1.0 + fmax(c[o + 1], 1.0));
    S->kkt[z][1] = c[o + 2] / (1.0 + fmax(rw[o + 0], c[o + 3]));
    S->kkt[z][2] = rw[o + 1] / (1.0 + fmax(rw[o + 3], rw[o + 2]));
  }
  S->dxa2[0] = rw[8];
  S->dxa2[1] = rw[9];
  S->dpa2[0] = c[8];
  S->dpa2[1] = c[9];
}

// ------------------------------------------------------------ utilities ----

__global__ void k_normalize(const int32_t *row_ptr, const float *u, float *uh, float *rowmax,
                            int n) {
  // one wave per row
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= n) return;
  const int b = row_ptr[i], e = row_ptr[i + 1];
  float mx = 0.0f;
  for (int k = b + lane; k < e; k += kWave) mx = fmaxf(mx, u[k]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  for (int k = b + lane; k < e; k += kWave) uh[k] = u[k] / mx;
  if (lane == 0) rowmax[i] = mx;
}

__global__ void k_degrees(const int32_t *col, int64_t nnz, int32_t *deg) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&deg[col[k]], 1);
}

__global__ void k_init_point(const int32_t *col, const int32_t *deg, int64_t nnz, float *x,
                             double *p, int m, double p0) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = g; k < nnz; k += stride) x[k] = 1.0f / (float)deg[col[k]];
  for (int64_t j = g; j < m; j += stride) p[j] = p0;
}

__global__ void k_copy_f32(const float *src, float *dst, int64_t len) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

__global__ void k_copy_f64(const double *src, double *dst, int64_t len) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

__global__ void k_f32_to_f64(const float *src, double *dst, int64_t len) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = (double)src[k];
}

__global__ void k_gather_f32_to_f64(const float *src, const int32_t *map, double *dst, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = (double)src[map ? map[i] : i];
}

__global__ void k_gather_f64_to_f32(const double *src, const int32_t *map, float *dst, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = (float)src[map ? map[i] : i];
}

__global__ void k_f64_to_f32(const double *src, float *dst, int64_t len) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = (float)src[k];
}

__global__ void k_fill_f64(double *dst, double v, int64_t len) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < len;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = v;
}

__global__ void k_scale_rows(const float *t, const float *s, float *out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = t[i] * s[i];
}

// w_i = sum_j e_ij p_j (Alg. 4), one wave per agent.
__global__ void k_budget_spmv(const int32_t *rp, const int32_t *col, const float *val,
                              const float *p, float *w, int n) {
  const int lane = threadIdx.x & (kWave - 1);
  const int i = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i] + lane; k < rp[i + 1]; k += kWave) s += (double)val[k] * (double)p[col[k]];
  s = wave_sum_d(s);
  if (lane == 0) w[i] = (float)s;
}

// -------------------------------------------------------------- launchers --

static int grid_for(int64_t len, int block) {
  int64_t g = (len + block - 1) / block;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}


bool row_variant_exists(int G, int E) {
#define PDHCG_EXISTS(g, e) \
  if (G == g && E == e) return true;
  PDHCG_ROW_VARIANTS(PDHCG_EXISTS)
#undef PDHCG_EXISTS
  return false;
}

template <int G, int E, int MODE, int LDSM>
static hipError_t row_launch_t(const MarketDev &md, const BinDev &bin, const RowIO &io, int nwg,
                               hipStream_t st) {
  const size_t lh = (LDSM & 4) ? (size_t)md.hot + 1 : (size_t)md.m;
  const size_t shm = lh * (((LDSM & 2) ? sizeof(double) : 0) + ((LDSM & 1) ? sizeof(double) : 0));
  hipLaunchKernelGGL((k_row_pass<G, E, MODE, LDSM>), dim3(nwg), dim3(kRowBlock), shm, st, md,
                     bin, io);
  return hipGetLastError();
}

hipError_t launch_row_pass(const MarketDev &md, const BinDev &bin, int G, int E, int lds_mode,
                           const RowIO &io, int nwg, hipStream_t st) {
  if (G == 0)
    return E > 0 ? launch_row_team(md, bin, E, lds_mode, io, nwg, st)
                 : launch_row_long(md, bin, lds_mode, io, nwg, st);
  const int mode = io.search;
#define PDHCG_ROW_LDS(g, e, md_)                                                  \
  switch (lds_mode) {                                                             \
    case 7: return row_launch_t<g, e, md_, 7>(md, bin, io, nwg, st);              \
    case 3: return row_launch_t<g, e, md_, 3>(md, bin, io, nwg, st);              \
    case 1: return row_launch_t<g, e, md_, 1>(md, bin, io, nwg, st);              \
    case 0: return row_launch_t<g, e, md_, 0>(md, bin, io, nwg, st);              \
    default: return hipErrorInvalidValue;                                         \
  }
#define PDHCG_ROW_DISPATCH(g, e)                                                   \
  if (G == g && E == e) {                                                          \
    if (mode == 0) { PDHCG_ROW_LDS(g, e, 0) }                                     \
    PDHCG_ROW_LDS(g, e, 1)                                                         \
  }
  PDHCG_ROW_VARIANTS(PDHCG_ROW_DISPATCH)
#undef PDHCG_ROW_DISPATCH
#undef PDHCG_ROW_LDS
  return hipErrorInvalidValue;
}

template <int G, int E, int LDSM>
static hipError_t eval_launch_t(const MarketDev &md, const BinDev &bin, const EvalIO &io,
                                int nwg, int total_wg, hipStream_t st) {
  const size_t shm = LDSM == 1 ? (size_t)md.hot * (sizeof(double) + 2 * sizeof(uint32_t)) : 0;
  hipLaunchKernelGGL((k_eval_row<G, E, LDSM>), dim3(nwg), dim3(kRowBlock), shm, st, md, bin,
                     io, total_wg);
  return hipGetLastError();
}

hipError_t launch_eval_row(const MarketDev &md, const BinDev &bin, int G, int E, int lds_mode,
                           const EvalIO &io, int nwg, int total_wg, hipStream_t st) {
  if (G == 0) return launch_eval_long(md, bin, lds_mode, io, nwg, total_wg, st);
#define PDHCG_EVAL_DISPATCH(g, e)                                                    \
  if (G == g && E == e)                                                              \
    return lds_mode ? eval_launch_t<g, e, 1>(md, bin, io, nwg, total_wg, st)        \
                    : eval_launch_t<g, e, 0>(md, bin, io, nwg, total_wg, st);
  PDHCG_ROW_VARIANTS(PDHCG_EVAL_DISPATCH)
#undef PDHCG_EVAL_DISPATCH
  return hipErrorInvalidValue;
}

hipError_t launch_pstep(const MarketDev &md, int zero_ctry, hipStream_t st) {
  hipLaunchKernelGGL(k_pstep, dim3((md.m + kColBlock - 1) / kColBlock), dim3(kColBlock), 0, st,
                     md, zero_ctry);
  return hipGetLastError();
}

hipError_t launch_cold_sums(const MarketDev &md, int use_state, const float *x, double *out,
                            int mean_degree, hipStream_t st) {
  const int ncold = md.m - md.hot;
  if (ncold <= 0 || !md.cold_ptr) return hipSuccess;
  // lanes per good: about a quarter of the mean degree (4 loads in flight per lane)
  const int gc = mean_degree >= 192 ? 64 : mean_degree >= 96 ? 32 : mean_degree >= 48 ? 16 : 8;
  const int per_block = 256 / gc;
  const int blocks = (int)std::min<int64_t>(((int64_t)ncold + per_block - 1) / per_block, 4096);
  switch (gc) {
    case 8: hipLaunchKernelGGL(k_cold_sums<8>, dim3(blocks), dim3(256), 0, st, md, use_state, x, out); break;
    case 16: hipLaunchKernelGGL(k_cold_sums<16>, dim3(blocks), dim3(256), 0, st, md, use_state, x, out); break;
    case 32: hipLaunchKernelGGL(k_cold_sums<32>, dim3(blocks), dim3(256), 0, st, md, use_state, x, out); break;
    default: hipLaunchKernelGGL(k_cold_sums<64>, dim3(blocks), dim3(256), 0, st, md, use_state, x, out); break;
  }
  return hipGetLastError();
}

hipError_t launch_eval_cold(const MarketDev &md, const EvalIO &io, int mean_degree,
                            hipStream_t st) {
  const int ncold = md.m - md.hot;
  if (ncold <= 0 || !md.ecold_ptr) return hipSuccess;
  // lanes per good: about a quarter of the mean degree (4 loads in flight per lane)
  const int gc = mean_degree >= 192 ? 64 : mean_degree >= 96 ? 32 : mean_degree >= 48 ? 16 : 8;
  const int per_block = 256 / gc;
  const int blocks = (int)std::min<int64_t>(((int64_t)ncold + per_block - 1) / per_block, 4096);
  switch (gc) {
    case 8: hipLaunchKernelGGL(k_eval_cold<8>, dim3(blocks), dim3(256), 0, st, md, io); break;
    case 16: hipLaunchKernelGGL(k_eval_cold<16>, dim3(blocks), dim3(256), 0, st, md, io); break;
    case 32: hipLaunchKernelGGL(k_eval_cold<32>, dim3(blocks), dim3(256), 0, st, md, io); break;
    default: hipLaunchKernelGGL(k_eval_cold<64>, dim3(blocks), dim3(256), 0, st, md, io); break;
  }
  return hipGetLastError();
}

hipError_t launch_col_decide(const MarketDev &md, int total_wg, int from_partials,
                             const double *ppart, int pchunks, int pacc, hipStream_t st) {
  const int tiles = (md.m + kColBlock - 1) / kColBlock;
  const int chunks = from_partials ? (total_wg < kColChunks ? total_wg : kColChunks) : 0;
  if (chunks > 0 && md.hot > 0) {
    hipLaunchKernelGGL(k_col_chunks, dim3((md.hot + kColBlock - 1) / kColBlock, chunks),
                       dim3(kColBlock), 0, st, md, total_wg);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_col_decide, dim3(tiles), dim3(kColBlock), 0, st, md, total_wg,
                     md.hot > 0 ? chunks : 0, ppart, pchunks, pacc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_rule, dim3(1), dim3(kColBlock), 0, st, md, total_wg, tiles, 0);
  return hipGetLastError();
}

hipError_t launch_col_decide_pdhg(const MarketDev &md, int total_wg, hipStream_t st) {
  const int tiles = (md.m + kColBlock - 1) / kColBlock;
  const int chunks = total_wg < kColChunks ? total_wg : kColChunks;
  hipLaunchKernelGGL(k_col_chunks, dim3((md.hot + kColBlock - 1) / kColBlock, chunks),
                     dim3(kColBlock), 0, st, md, total_wg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_col_decide, dim3(tiles), dim3(kColBlock), 0, st, md, total_wg, chunks,
                     nullptr, 0, 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_rule, dim3(1), dim3(kColBlock), 0, st, md, total_wg, tiles, 1);
  return hipGetLastError();
}

hipError_t launch_eval_col_stats(const MarketDev &md, const EvalIO &io, int total_wg, int partials,
                                 hipStream_t st) {
  const int tiles = (md.m + kColBlock - 1) / kColBlock;
  hipLaunchKernelGGL(k_eval_col, dim3(tiles), dim3(kColBlock), 0, st, md, io, total_wg, partials);
  return hipGetLastError();
}

hipError_t launch_eval_chunks(const MarketDev &md, const EvalIO &io, int total_wg,
                              hipStream_t st) {
  if (md.hot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_chunks, dim3((md.hot + kColBlock - 1) / kColBlock, kColChunks),
                     dim3(kColBlock), 0, st, md, io, total_wg);
  return hipGetLastError();
}

hipError_t launch_eval_col(const MarketDev &md, const EvalIO &io, int total_wg,
                           int partials, hipStream_t st) {
  const int tiles = (md.m + kColBlock - 1) / kColBlock;
  hipLaunchKernelGGL(k_eval_col, dim3(tiles), dim3(kColBlock), 0, st, md, io, total_wg, partials);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_eval_final, dim3(1), dim3(kColBlock), 0, st, md, total_wg, tiles);
  return hipGetLastError();
}

hipError_t launch_normalize(const int32_t *row_ptr, const float *u, float *uh, float *rowmax,
                            int n, hipStream_t st) {
  const int rows_per_block = 256 / kWave;
  hipLaunchKernelGGL(k_normalize, dim3((n + rows_per_block - 1) / rows_per_block), dim3(256), 0,
                     st, row_ptr, u, uh, rowmax, n);
  return hipGetLastError();
}

hipError_t launch_degrees(const int32_t *col, int64_t nnz, int32_t *deg, hipStream_t st) {
  hipLaunchKernelGGL(k_degrees, dim3(grid_for(nnz, 256)), dim3(256), 0, st, col, nnz, deg);
  return hipGetLastError();
}

hipError_t launch_init_point(const int32_t *col, const int32_t *deg, int64_t nnz, float *x,
                             double *p, int m, double p0, hipStream_t st) {
  hipLaunchKernelGGL(k_init_point, dim3(grid_for(nnz > m ? nnz : m, 256)), dim3(256), 0, st, col,
                     deg, nnz, x, p, m, p0);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float *src, float *dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(len, 256)), dim3(256), 0, st, src, dst, len);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double *src, double *dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(len, 256)), dim3(256), 0, st, src, dst, len);
  return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(len, 256)), dim3(256), 0, st, src, dst, len);
  return hipGetLastError();
}

hipError_t launch_gather_f32_to_f64(const float *src, const int32_t *map, double *dst, int m,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_gather_f32_to_f64, dim3(grid_for(m, 256)), dim3(256), 0, st, src, map, dst,
                     m);
  return hipGetLastError();
}

hipError_t launch_gather_f64_to_f32(const double *src, const int32_t *map, float *dst, int m,
                                    hipStream_t st) {
  hipLaunchKernelGGL(k_gather_f64_to_f32, dim3(grid_for(m, 256)), dim3(256), 0, st, src, map, dst,
                     m);
  return hipGetLastError();
}

hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(len, 256)), dim3(256), 0, st, src, dst, len);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *dst, double v, int64_t len, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(len, 256)), dim3(256), 0, st, dst, v, len);
  return hipGetLastError();
}

hipError_t launch_scale_rows(const float *t, const float *rowscale, float *out, int n,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_scale_rows, dim3((n + 255) / 256), dim3(256), 0, st, t, rowscale, out, n);
  return hipGetLastError();
}

hipError_t launch_budget_spmv(const int32_t *e_row_ptr, const int32_t *e_col, const float *e_val,
                              const float *p, float *w, int n, hipStream_t st) {
  const int rows_per_block = 256 / kWave;
  hipLaunchKernelGGL(k_budget_spmv, dim3((n + rows_per_block - 1) / rows_per_block), dim3(256),
                     0, st, e_row_ptr, e_col, e_val, p, w, n);
  return hipGetLastError();
}

}  // namespace pdhcg
