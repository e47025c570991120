// Internal declarations of the gfx950 PDHCG library (kernels <-> host side).
// Not part of the public ABI (include/pdhcg.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdhcg {

constexpr int kWave = 64;        // CDNA wavefront
constexpr int kRowBlock = 512;   // threads per row-kernel workgroup (8 waves)
constexpr int kColBlock = 256;   // threads per column-kernel block
constexpr int kMaxSections = 32; // largest k of the k-section search with G lanes per row
constexpr int kMaxWaveSections = 64;  // largest k with one lane per candidate (wave64)
constexpr int kKwaveMaxRow = 512;     // longest row of the one-wave-per-row k-section kernel
constexpr int kRowStats = 4;     // per-workgroup partials of the row kernel
constexpr int kEvalRowStats = 12;
constexpr int kColStats = 2;
constexpr int kEvalColStats = 12;
constexpr int kColChunks = 16;   // partial-row chunks per column tile
// Long rows held in registers by teams of waves (pdhcg_team.hip).
constexpr int kTeamBlock = 512;     // threads per workgroup of the team kernel
constexpr int kTeamMaxRow = 16384;  // longest row it holds (512 threads x 32)
// Goods beyond the LDS: panels of kPanelW goods, at most kMaxPanels.
constexpr int kPanelShift = 13;
constexpr int kPanelW = 1 << kPanelShift;
constexpr int kMaxPanels = 32;
// Per-edge arrays are addressed with 32-bit byte offsets, and offsets from
// 2^31 up mark idle lanes: markets have at most 2^29 stored entries.
constexpr int64_t kMaxBufferEntries = int64_t(1) << 29;

// Device-resident solver state.  The step kernels read it at launch and the
// last block of the column kernel updates it (step-size rule, role swaps);
// the host reads and rewrites it only while the stream is idle.
struct DevState {
  int32_t ix[3];  // allocation buffers: [0] current, [1] trial, [2] average
  int32_t ip[3];  // price buffers, same roles
  int32_t ic[3];  // column-sum buffers: [0] previous, [1] current, [2] trial
  int32_t fold;   // 1: the current iterate is not yet in the averages
  int32_t step_mode;
  int32_t accept_last;
  int32_t pad0;
  int64_t total;     // iterations (trial steps) so far
  int64_t since;     // iterations since the last restart
  int64_t k_in;      // kept steps since the last restart
  int64_t accepted;  // kept steps overall
  double eta, omega, eta0, eta_lo, eta_hi, tau, sigma;
  double emax_last;
  uint32_t rounds_max;
  uint32_t pad1;
  uint64_t rounds_sum;
  uint64_t rows_searched;
  // results of the last KKT evaluation: [0] current, [1] average
  double kkt[2][3];     // r_primal, r_dual, r_gap
  double dxa2[2];       // |x - x_anchor|^2
  double dpa2[2];       // |p - p_anchor|^2
};

// Device view of one market (passed by value to kernels).
struct MarketDev {
  int32_t n, m;
  int64_t nnz;
  int32_t hot;       // goods [0, hot) have prices and column partials in LDS;
                     // goods from hot on (the less bought ones after the
                     // relabelling by degree) use global memory and atomics
  int32_t pad_hot;
  // goods from hot on, column by column (relabelled markets): entries of
  // good hot + g are cold_idx[cold_ptr[g] .. cold_ptr[g + 1]) in row order
  const int32_t *cold_ptr;
  const int32_t *cold_idx;
  float *srow;       // [n] root of each long row at the last solver pass (0: none)
  // panel buffers of the goods from hot on (rows of the team kernel): the
  // entries' values and their good's index inside its panel; row r of the
  // team bins owns the run starting at proff[r * npanel + panel]
  float *pval;
  uint16_t *pid;
  const int32_t *proff;
  // the other rows' entries of those goods have fixed slots: cslot[q] (-1
  // for the entries of the goods in LDS and of team-kernel rows)
  const int32_t *cslot;
  int32_t npanel, pad_panel;
  // every entry of the goods from hot on, column by column in row order,
  // with its row (KKT pass of relabelled markets, k_eval_cold; null when
  // their maxima and sums are taken with device atomics), and the rows'
  // dual values y = w / u^T x of the current and averaged points [2][n]
  // written by the KKT row kernels for it
  const int32_t *ecold_ptr;
  const int32_t *ecold_idx;
  const int32_t *ecold_row;
  double *yrow;
  const int32_t *row_ptr;
  const int32_t *col;
  const uint16_t *col16;  // the same good ids in 16 bits, for markets whose
                          // goods all sit in LDS (m < 65536); else null
  const float *uh;   // row-normalised utilities
  const float *w;    // budgets
  float *X0, *X1, *X2;
  double *P0, *P1, *P2;  // prices (float64: O(m), updates fall below float32 resolution)
  double *C0, *C1, *C2;
  float *XA;         // restart anchor x^{n,0}
  double *PA;        // restart anchor p^{n,0}
  double *colpart;   // [total_wg][hot] per-workgroup column partials of the LDS goods
  double *rowpart;   // [total_wg][kRowStats]
  double *colblk;    // [col blocks][kColStats or kEvalColStats]
  double *colchunk;  // [kColChunks][m] chunk sums of the column partials
  DevState *S;
};

// Per-buyer state of restarted PDHG (Alg. 1) on the reformulated program:
// utilities t and their duals y (normalised units, float64), and the
// residuals g = t - U x of the utility constraint.  t and the primal anchor
// follow the allocation's roles (DevState::ix), y the prices' (ip), g the
// column sums' (ic: previous / current / trial).
struct PdhgDev {
  double *T0, *T1, *T2;
  double *Y0, *Y1, *Y2;
  double *G0, *G1, *G2;
  double *TA, *YA;   // restart anchors of t and y
};
constexpr int kPdhgEvalStats = 20;  // per-workgroup statistics of the PDHG KKT pass

// Row kernel shapes (G lanes per row, E entries per lane) that are built.
#define PDHCG_ROW_VARIANTS(X) \
  X(4, 1) X(4, 2) X(4, 4) X(4, 8) \
  X(8, 1) X(8, 2) X(8, 4) X(8, 8) \
  X(16, 1) X(16, 2) X(16, 4) X(16, 6) X(16, 7) X(16, 8) \
  X(32, 1) X(32, 2) X(32, 4) X(32, 8) \
  X(64, 1) X(64, 2) X(64, 4) X(64, 8)

// Rows handled by one kernel variant.
struct BinDev {
  const int32_t *rows;  // row ids of this bin (null: slot s is row s)
  const int32_t *rlo;   // per slot: first entry of its row (row_ptr without rows)
  const int32_t *rhi;   // per slot: one past its last entry (row_ptr + 1 without rows)
  int32_t nrows;
  int32_t wg_offset;    // first partial slot of this bin
  int32_t rows_per_wg;  // rows per workgroup (the row kernel interleaves passes instead)
  int32_t team_off;     // team kernel: index of the bin's first row in the panel offsets
};

// Inputs/outputs of a row pass.  With use_state = 1 the kernel takes the
// buffers and tau from DevState roles; otherwise from the fields below.
struct RowIO {
  const float *xin;
  const double *p;
  float *xout;
  float *xavg;      // averaged allocation to fold xin into (nullable)
  float *s_out;     // per-row root (nullable)
  double tau;
  float wfold;      // fold weight 1/k (0: no fold)
  int32_t use_state;
  int32_t colsum;   // accumulate column sums of xout
  int32_t search;   // 0 active-set, 1 k-section (G lanes per row), 2 k-section
                    // (one wave per row, one lane per candidate)
  int32_t sections;
  int32_t max_rounds;
  double rtol;
  double *csum;     // float64 column sums of xout by device atomics (explicit
                    // mode without LDS partials), zeroed by the caller
};

// Reverse step of the row prox (pdhcg_adjoint.hip).
struct AdjIO {
  const float *xn;    // x^{k+1}, the prox output of the step being reversed
  const float *r_in;  // adjoint of x^{k+1}: r_in + b[col]
  const double *b;
  float *r_out;       // r, the adjoint of x^k - tau p^{k+1}
  float *duh;         // += dL/d uh (row-normalised utilities)
  float *dw;          // += dL/dw
  double *csum;       // column sums of r by device atomics (no LDS partials)
  double tau;
};

// Inputs/outputs of a KKT pass over one or two points.
struct EvalIO {
  const float *xc;   // current allocation
  const double *pc;  // current prices
  float *xa;         // averaged allocation (nullable), folded in place
  const double *pa;  // averaged prices (before the fold)
  float wfold;       // fold weight for the averaged point (0: none)
  const float *xanc; // restart anchor (nullable)
  float *tc;         // per-row utility of the current point (nullable)
  float *ta;         // per-row utility of the averaged point (nullable)
  const float *rowscale; // multiply t by this (original units)
  float *evalpart;   // column maxima (ord_key keys): [2][total_wg][hot] (LDS mode) or [2][m]
  double *evalcs;    // [total_wg][hot] float64 column-sum partials (LDS mode)
  uint32_t *evalchunk; // [2][kColChunks][m] chunk maxima (LDS mode)
  uint32_t *gmax;    // [2][m] device-wide maxima of the goods from hot on (LDS mode)
  double *gsum;      // [m] device-wide sums of the goods from hot on (LDS mode)
  double *cacc;      // [m] float64 column sums: accumulator (non-LDS mode), else
                     // [kColChunks][m] chunk sums
  int32_t want_cc;   // sum the columns of xc (no average; ccur unused)
  const double *ccur;// column sums of xc (float64) when !want_cc
  double *cavg_out;  // receives the float64 column sums this pass computed
                     // (of the averaged point, or of xc when want_cc)
  double *pa_out;    // receives the folded averaged prices
  const double *panc;// price anchor (nullable)
};

// Launchers (pdhcg_kernels.hip).
hipError_t launch_row_pass(const MarketDev &md, const BinDev &bin, int G, int E,
                           int lds_mode, const RowIO &io, int nwg, hipStream_t st);
hipError_t launch_pstep(const MarketDev &md, int zero_ctry, hipStream_t st);
// Column sums of the goods from hot on (relabelled markets), gathered from
// the new allocation in a fixed order: with use_state the trial allocation
// and trial column sums of DevState, else x / out.
hipError_t launch_cold_sums(const MarketDev &md, int use_state, const float *x, double *out,
                            int mean_degree, hipStream_t st);
// ppart (or null): panel partials of the goods from hot on, summed into
// c_try by k_col_decide (added to c_try when pacc).
// KKT column maxima and sums of the goods from hot on from the lists
// ecold_* (one segment of lanes per good, no atomics), into io.gmax / io.gsum.
hipError_t launch_eval_cold(const MarketDev &md, const EvalIO &io, int mean_degree, hipStream_t st);
hipError_t launch_col_decide(const MarketDev &md, int total_wg, int from_partials,
                             const double *ppart, int pchunks, int pacc, hipStream_t st);
hipError_t launch_eval_row(const MarketDev &md, const BinDev &bin, int G, int E,
                           int lds_mode, const EvalIO &io, int nwg, int total_wg,
                           hipStream_t st);
hipError_t launch_eval_col(const MarketDev &md, const EvalIO &io, int total_wg,
                           int partials, hipStream_t st);
hipError_t launch_eval_chunks(const MarketDev &md, const EvalIO &io, int total_wg,
                              hipStream_t st);
hipError_t launch_normalize(const int32_t *row_ptr, const float *u, float *uh,
                            float *rowmax, int n, hipStream_t st);
hipError_t launch_degrees(const int32_t *col, int64_t nnz, int32_t *deg, hipStream_t st);
hipError_t launch_init_point(const int32_t *col, const int32_t *deg, int64_t nnz,
                             float *x, double *p, int m, double p0, hipStream_t st);
hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t len, hipStream_t st);
// dst[i] = src[map[i]] (map may be null: dst[i] = src[i]); goods vectors
// between the caller's order and the relabelled one.
hipError_t launch_gather_f32_to_f64(const float *src, const int32_t *map, double *dst, int m,
                                    hipStream_t st);
hipError_t launch_gather_f64_to_f32(const double *src, const int32_t *map, float *dst, int m,
                                    hipStream_t st);
hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t len, hipStream_t st);
hipError_t launch_copy_f32(const float *src, float *dst, int64_t len, hipStream_t st);
hipError_t launch_copy_f64(const double *src, double *dst, int64_t len, hipStream_t st);
hipError_t launch_fill_f64(double *dst, double v, int64_t len, hipStream_t st);
hipError_t launch_scale_rows(const float *t, const float *rowscale, float *out, int n,
                             hipStream_t st);
hipError_t launch_budget_spmv(const int32_t *e_row_ptr, const int32_t *e_col,
                              const float *e_val, const float *p, float *w, int n,
                              hipStream_t st);
bool row_variant_exists(int G, int E);
// Rows longer than kLongRow entries: one wave per row (pdhcg_long.hip); a
// bin of them has G = E = 0.
constexpr int kLongRow = 512;
hipError_t launch_row_long(const MarketDev &md, const BinDev &bin, int lds_mode, const RowIO &io,
                           int nwg, hipStream_t st);
hipError_t launch_eval_long(const MarketDev &md, const BinDev &bin, int lds_mode,
                            const EvalIO &io, int nwg, int total_wg, hipStream_t st);
hipError_t launch_adj_long(const MarketDev &md, const BinDev &bin, int lds, const AdjIO &io,
                           int nwg, hipStream_t st);
// Rows of 513 .. kTeamMaxRow entries in registers of teams of waves: a bin
// of them has G = 0 and E = its team shape code (team_code of its rows);
// its cold entries go to the panel buffers, summed by launch_panel_sums.
int team_code(int d);
hipError_t launch_row_team(const MarketDev &md, const BinDev &bin, int code, int lds_mode,
                           const RowIO &io, int nwg, hipStream_t st);
// With sum = 0 only the partials are written (the caller sums them, as
// launch_col_decide does).
hipError_t launch_panel_sums(const MarketDev &md, int use_state, double *out, const float *pval,
                             const uint16_t *pid, const int64_t *pbeg, double *part, int nchunk,
                             int accumulate, int sum, hipStream_t st);
// k-section search with one wave per row and one lane per candidate
// (pdhcg_ksec.hip); rows of at most kKwaveMaxRow entries, column partials
// of every good in LDS.
size_t kwave_lds_bytes(int m);
hipError_t launch_row_kwave(const MarketDev &md, const RowIO &io, int nwg, hipStream_t st);

// Restarted PDHG (pdhcg_pdhg.hip); markets whose goods all sit in LDS
// (LDS mode 3) and rows of at most 512 entries.
hipError_t launch_pdhg_row(const MarketDev &md, const PdhgDev &pd, const BinDev &bin, int G, int E,
                           int nwg, hipStream_t st);
hipError_t launch_pdhg_eval(const MarketDev &md, const PdhgDev &pd, const BinDev &bin, int G,
                            int E, const EvalIO &io, const double *tc, const double *yc,
                            double *ta, double *ya, double *g_avg, int nwg, int total_wg,
                            hipStream_t st);
hipError_t launch_pdhg_eval_final(const MarketDev &md, int total_wg, hipStream_t st);
hipError_t launch_pdhg_rows_init(const MarketDev &md, const float *x, const float *t_in,
                                 const float *y_in, const float *rowmax, double *t, double *y,
                                 double *g0, double *g1, hipStream_t st);
hipError_t launch_pdhg_rows_out(const double *t, const double *y, const float *rowmax, float *t_out,
                                float *y_out, int n, hipStream_t st);
// KKT column statistics only (k_eval_col), without the PDHCG combination.
hipError_t launch_eval_col_stats(const MarketDev &md, const EvalIO &io, int total_wg, int partials,
                                 hipStream_t st);
// Column kernels of a PDHG step: the step-size rule with the buyers' terms.
hipError_t launch_col_decide_pdhg(const MarketDev &md, int total_wg, hipStream_t st);

// Reverse mode (pdhcg_adjoint.hip).
// Largest number of buyers with x_ij > 0 over the goods (cnt: [m] work
// array; out: one int, device).
hipError_t launch_active_colmax(const int32_t *col, const float *x, int64_t nnz, int32_t *cnt,
                               int m, int32_t *out, hipStream_t st);
hipError_t launch_adj_pstep(double *p, const double *c, const double *cprev, double sigma, int m,
                            hipStream_t st);
hipError_t launch_sum_partials(const double *part, int rows, int hot, int m, double *chunk,
                               hipStream_t st);
hipError_t launch_finish_colsum(const double *chunk, const double *cold, int hot, int m,
                                double *out, hipStream_t st);
hipError_t launch_colsum_atomic(const int32_t *col, const float *x, int64_t nnz, double *out,
                                int m, hipStream_t st);
hipError_t launch_zero_f64(double *a, int64_t len, hipStream_t st);
hipError_t launch_zero_f32(float *a, int64_t len, hipStream_t st);
hipError_t launch_adj_row(const MarketDev &md, const BinDev &bin, int G, int E, int lds,
                          const AdjIO &io, int nwg, hipStream_t st);
hipError_t launch_adj_col(const double *chunk, const double *cold, int hot, double *P, double *B,
                          double *Cn, double tau, double sigma, int m, hipStream_t st);
hipError_t launch_adj_unnormalize(const int32_t *row_ptr, const float *uh, const float *rowmax,
                                  const float *duh, int n, float *du, hipStream_t st);

}  // namespace pdhcg
