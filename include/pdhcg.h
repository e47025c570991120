/*
 * pdhcg.h -- C ABI of the MI355X (gfx950) PDHCG solver for linear Fisher
 * markets and the Arrow-Debreu fixed point built on it.
 *
 * Method: Liu, Huang, Li, Ge, Ye, "PDHCG: A Scalable First-Order Method for
 * Large-Scale Competitive Market Equilibrium Computation" (arXiv 2506.06258).
 *
 * Problem (Sec. 1, Eisenberg-Gale program): n buyers with budgets w_i > 0,
 * m goods of unit supply, linear utilities u_ij >= 0 on a sparse pattern:
 *     max_x  sum_i w_i log(sum_j u_ij x_ij)  s.t.  sum_i x_ij = 1, x >= 0.
 * The optimal duals p of the supply constraints are the unique equilibrium
 * prices (Sec. 3, Fact 1); x is an equilibrium allocation.
 *
 * Conventions shared by every call:
 *  - Pointers named "device" are HIP device pointers; the caller owns them.
 *    Calls only read inputs; outputs are written in place.
 *  - CSR: row_ptr[n+1] (int32, row_ptr[0] = 0, non-decreasing), col[nnz]
 *    (int32, strictly increasing inside every row, values in [0, m)).  All
 *    per-edge arrays (u, x) are aligned with col.
 *  - Values are float32.  Internal global reductions (column sums, KKT and
 *    restart norms) accumulate in float64.
 *  - Every call returns a pdhcg_status (int).  Nothing throws across the
 *    ABI.  pdhcg_last_error() returns a description of the last failure on
 *    the calling thread.
 *  - A market handle owns its device copies and workspace and is bound to
 *    the device and stream given at creation.  Handles are not thread-safe;
 *    different handles may be used from different threads.
 *  - Synchronisation: pdhcg_market_create, pdhcg_solve, pdhcg_kkt and
 *    pdhcg_arrow_debreu return after their device work on the handle's
 *    stream has finished.  pdhcg_row_prox only enqueues.
 *  - Environment overrides, read at pdhcg_market_create (for tests and
 *    parameter sweeps; results stay those of the method):
 *      PDHCG_ROW_G, PDHCG_ROW_E   force the row shape (lanes, entries per
 *                                 lane) of every bin that it can hold;
 *      PDHCG_MERGE_BINS=0         keep one bin per row shape (default: the
 *                                 register-resident bins of equal lane
 *                                 count merge into the one with the most
 *                                 entries per lane);
 *      PDHCG_HOT=k                relabel the goods by degree and keep only
 *                                 the first k in LDS (as for large m);
 *      PDHCG_SLOT_SHARE=f         on relabelled markets, give the short
 *                                 rows' entries of goods beyond LDS fixed
 *                                 panel slots when they are at least this
 *                                 share of those rows' entries (default 0.1;
 *                                 else they are gathered by column);
 *      PDHCG_P_LDS=0              prices from global memory, partials in LDS;
 *      PDHCG_NO_LDS=1             no LDS: device atomics for column sums;
 *      PDHCG_TEAM=0 / 2           rows above 512 entries all on the
 *                                 one-wave-per-row kernel / all (up to
 *                                 16384 entries) in registers of teams of
 *                                 waves (default: teams for the rows of
 *                                 relabelled markets);
 *    and at pdhcg_batch_solve: PDHCG_BATCH_EAGER=1 launches the batch's
 *    kernels directly instead of replaying its graph; at pdhcg_batch_create:
 *    PDHCG_BATCH_GANG=0 keeps every market on one workgroup,
 *    PDHCG_BATCH_GANG=k (k >= 2) splits every market of at least k rows over
 *    k workgroups (as far as the resident workgroups allow).
 */
#ifndef PDHCG_H
#define PDHCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PDHCG_ABI_VERSION 1

typedef struct pdhcg_market_s *pdhcg_market;

typedef enum {
  PDHCG_OK = 0,
  PDHCG_MAX_ITER = 1,         /* not fatal: outputs hold the last candidate */
  PDHCG_ERR_ARG = -1,         /* bad size, pointer, CSR shape or value */
  PDHCG_ERR_ASSUMPTION = -2,  /* a buyer or good with no positive utility
                                 (Assumption 1, Sec. 2) */
  PDHCG_ERR_NUMERIC = -3,     /* non-finite iterate or no positive row root */
  PDHCG_ERR_OOM = -4,         /* device or host allocation failed */
  PDHCG_ERR_HIP = -5,         /* a HIP runtime call failed */
  PDHCG_ERR_UNSUPPORTED = -6  /* shape outside the built kernel variants */
} pdhcg_status;

/* Root search for the row subproblem (Sec. 2.2). */
enum {
  /* Bracketing search of Alg. 3 whose trial points are the roots of the
   * quadratic that holds on the active set of the previous trial; each
   * such root is a lower bound on s* and is exact once the active set
   * settles.  Default on gfx950. */
  PDHCG_SEARCH_ACTIVESET = 0,
  /* k-section search of Sec. 2.2.1 (sections = k <= 32, 32 in the paper)
   * on the row shapes of the active-set search: the G lanes that hold a
   * row evaluate the k candidates one after the other.
   * pdhcg_solve and pdhcg_row_prox return PDHCG_ERR_UNSUPPORTED for it on
   * markets with rows of more than 512 entries. */
  PDHCG_SEARCH_KSECTION = 1,
  /* The same k-section search mapped as Sec. 2.2.1 maps it: one wave per
   * row with the row staged in LDS and one lane per candidate
   * (sections = k <= 64 on wave64).  pdhcg_solve and pdhcg_row_prox return
   * PDHCG_ERR_UNSUPPORTED for it on markets with rows of more than 512
   * entries or whose column partials do not fit LDS beside the staging
   * (m > 14000 on gfx950). */
  PDHCG_SEARCH_KSECTION_WAVE = 2
};

enum { PDHCG_STEP_FIXED = 0, PDHCG_STEP_ADAPTIVE = 1 };
enum { PDHCG_RESTART_NONE = 0, PDHCG_RESTART_ADAPTIVE = 1 };
enum { PDHCG_OUTPUT_CANDIDATE = 0, PDHCG_OUTPUT_CURRENT = 1, PDHCG_OUTPUT_AVERAGE = 2 };

/* Solver parameters.  pdhcg_default_params() fills the values given in
 * Sec. 5 ("Algorithmic Enhancements", "Criteria") and the readings of the
 * passages the paper leaves open (documented with the defaults). */
typedef struct pdhcg_params {
  double tol;                /* stop when the candidate's relative KKT <= tol
                                (Sec. 5 Criteria; default 1e-4) */
  int64_t max_iter;          /* cap on iterations (every prox sweep counts) */
  int32_t eval_every;        /* iterations between KKT / restart checks (64) */
  int32_t search;            /* PDHCG_SEARCH_* */
  int32_t sections;          /* k of the k-section search (32, Sec. 2.2.1) */
  int32_t max_search_rounds; /* cap on search rounds per row (16) */
  double search_rtol;        /* a row search stops when U - L <= rtol * U */
  int32_t step_mode;         /* PDHCG_STEP_* (adaptive, Sec. 5) */
  int32_t restart;           /* PDHCG_RESTART_* (adaptive, Sec. 5) */
  double beta_sufficient;    /* 0.2 (Sec. 5) */
  double beta_necessary;     /* 0.8 (Sec. 5) */
  double beta_artificial;    /* 0.2 (Sec. 5) */
  double theta;              /* primal-weight smoothing, 0.2 (Sec. 5) */
  int32_t omega_check_every; /* restarts between primal-weight checks (3) */
  int32_t output;            /* PDHCG_OUTPUT_* */
  double omega_bound;        /* reset omega to omega0 when outside
                                [omega0/bound, omega0*bound] */
  double eta0;               /* <= 0: 1 in adaptive mode, 0.9/||K|| fixed */
  double omega0;             /* <= 0: sum(w) / (20 m), a twentieth of the
                                mean equilibrium price */
  int32_t normalize_rows;    /* divide each buyer's utilities by their
                                maximum (Sec. 5 Preprocessing; 1) */
  int32_t verbose;           /* print one line per check to stderr */
  int32_t timing;            /* 1: time every row-kernel launch with HIP
                                events on the handle's stream (fills the
                                row_pass_* fields of pdhcg_info) */
} pdhcg_params;

/* Result of a solve or a KKT evaluation (host struct). */
typedef struct pdhcg_info {
  double rel_kkt;            /* max of the three relative residuals */
  double rel_primal;
  double rel_dual;
  double rel_gap;
  double eta;                /* final step size */
  double omega;              /* final primal weight */
  double seconds;            /* wall time of the solve */
  int64_t iters;             /* iterations (prox sweeps) */
  int64_t accepted;          /* iterations kept by the step-size rule */
  int32_t restarts;
  int32_t status;
  int32_t evals;             /* KKT checks performed */
  int32_t search_rounds_max; /* largest number of search rounds of any row */
  double search_rounds_mean; /* mean search rounds per row and iteration */
  double row_pass_seconds;   /* summed device time of the row-kernel launches
                                (params.timing = 1), else 0 */
  int64_t row_pass_launches; /* number of timed row-kernel launch groups */
} pdhcg_info;

int32_t pdhcg_abi_version(void);
const char *pdhcg_status_string(int32_t status);
/* Description of the last error raised on the calling thread ("" if none). */
const char *pdhcg_last_error(void);
void pdhcg_default_params(pdhcg_params *params);

/* Host-side validation of a market given in host memory (all pointers
 * host).  Checks sizes, CSR shape, strictly increasing in-range columns,
 * finite u >= 0, finite w > 0 (PDHCG_ERR_ARG), then Assumption 1 of Sec. 2
 * on the positive entries (PDHCG_ERR_ASSUMPTION).  Needs no GPU. */
int32_t pdhcg_validate_host(int32_t n, int32_t m, int64_t nnz,
                            const int32_t *row_ptr, const int32_t *col,
                            const float *u, const float *w);

/* Create a market handle from device arrays (Sec. 1 problem data: U on its
 * CSR pattern, budgets w).  The inputs are validated (as
 * pdhcg_validate_host), copied, and preprocessed on the device: each row of
 * U is divided by its maximum (Sec. 5), column degrees and ||K|| are
 * computed, and the row kernels are chosen from the degree profile.  The
 * caller may free its inputs afterwards.  stream: a hipStream_t (NULL =
 * default stream).  On failure *out is NULL. */
int32_t pdhcg_market_create(int32_t n, int32_t m, int64_t nnz,
                            const int32_t *row_ptr, const int32_t *col,
                            const float *u, const float *w, void *stream,
                            pdhcg_market *out);

/* Replace the budgets (device pointer, n floats, all > 0).  Used by the
 * Arrow-Debreu outer loop (Sec. 4, Alg. 4). */
int32_t pdhcg_set_budgets(pdhcg_market market, const float *w);

/* Solve the Fisher market by restarted PDHCG (Alg. 2 with the Sec. 5
 * enhancements).
 *   p [m]   device.  warm != 0: starting prices on entry.  Out: prices.
 *   x [nnz] device.  warm != 0: starting allocation on entry (CSR order).
 *           Out: allocation.
 *   t [n]   device, may be NULL.  Out: utilities sum_j u_ij x_ij in the
 *           caller's (unnormalised) units.
 *   info    host, may be NULL.
 * Returns PDHCG_OK when the candidate's relative KKT reached tol,
 * PDHCG_MAX_ITER when max_iter ran out (outputs hold the last candidate). */
int32_t pdhcg_solve(pdhcg_market market, const pdhcg_params *params,
                    int32_t warm, float *p, float *x, float *t,
                    pdhcg_info *info);

/* Alg. 2 in the setting of its analysis (Sec. 3: Lemma 1, Lemma 2,
 * Theorem 1): fixed step sizes sigma = tau = eta, a fixed restart length K,
 * and every restart to the average of the K iterates of its inner loop, with
 * none of the Sec. 5 enhancements except the row normalisation.  Runs
 * `restarts` inner loops from the default initial point (x0_ij = 1/deg_j,
 * p0_j = sum(w)/m).
 *   eta   <= 0: 1/(2||K||) with ||K|| = sqrt(max_j deg_j) (the norm of the
 *         column-sum operator on the stored pattern); else the step.
 *   p_ref [m] device, may be NULL: reference prices (normally p*).
 *   dist  [restarts + 1] host, may be NULL: ||p^{n,0} - p_ref||_2 of the
 *         restart points n = 0 (the start) .. restarts (0 without p_ref).
 *   kkt   [restarts + 1] host, may be NULL: relative KKT error (Sec. 5
 *         Criteria) of each restart point.
 *   p [m], x [nnz] device outputs: the last restart point.
 *   info  host, may be NULL (iters = K * restarts).
 * ERR_ARG on null p/x, K < 1, restarts < 0 or a non-finite eta. */
int32_t pdhcg_solve_fixed_restart(pdhcg_market market, int32_t K,
                                  int32_t restarts, double eta,
                                  const float *p_ref, double *dist,
                                  double *kkt, float *p, float *x,
                                  pdhcg_info *info);

/* Solve the Fisher market by restarted PDHG (Alg. 1, Sec. 2.1), the
 * method PDHCG is compared with in Sec. 5: primal (x, t), dual (p, y) of
 * the reformulated program (eq. primal-dual-formulation), iterations of
 * eqs. update:py, update:t and update:x, with the same Sec. 5 enhancements
 * as pdhcg_solve (row normalisation, adaptive restarts, primal weight,
 * adaptive step size) and the Sec. 5 Criteria KKT error of (x, t, p, y).
 * params: as pdhcg_solve (the search fields are unused).  Fixed step mode
 * uses eta = 0.9 / (sqrt(max_j deg_j) + 1 + sqrt(max_j deg_j max_i deg_i)),
 * a bound below 1/||K||; adaptive mode starts at eta = 1.  Initial point:
 * x0_ij = 1/deg_j, p0_j = sum(w)/m, t0 = U x0, y0 = w / t0.
 *   p [m], x [nnz] device: as pdhcg_solve (warm != 0 reads them).
 *   t [n], y [n]   device, may be NULL: utilities and their duals in the
 *                  caller's units (t_i in units of u_i, y_i in 1/u_i); with
 *                  warm != 0 a non-NULL t or y is also the starting value
 *                  (else t = U x, y = w / t).
 * Built for markets whose goods all keep their prices in LDS (m <= 10000
 * on gfx950) and rows of at most 512 entries: PDHCG_ERR_UNSUPPORTED
 * otherwise.  Returns as pdhcg_solve. */
int32_t pdhcg_pdhg_solve(pdhcg_market market, const pdhcg_params *params,
                         int32_t warm, float *p, float *x, float *t, float *y,
                         pdhcg_info *info);

/* Relative KKT error (Sec. 5 Criteria, with t_i = u_i^T x_i, y = w/t) of a
 * given point (device p[m], x[nnz]) on the normalised market; float64
 * reductions.  Fills rel_kkt / rel_primal / rel_dual / rel_gap of info. */
int32_t pdhcg_kkt(pdhcg_market market, const float *p, const float *x,
                  pdhcg_info *info);

/* One parallel row update of Alg. 2 on its own: for every buyer i, the
 * minimiser of  -w_i log(u_i^T x_i) + p^T x_i + |x_i - x_in_i|^2/(2 tau)
 * over x_i >= 0 (Sec. 2.2), using the market's normalised utilities and
 * the search selected in params (NULL: defaults).  All arrays device:
 * x_in, x_out [nnz], p [m], s_out [n] (may be NULL; receives u_i^T x_i of
 * the normalised row).  Enqueued on the handle's stream; no
 * synchronisation. */
int32_t pdhcg_row_prox(pdhcg_market market, const float *x_in,
                       const float *p, double tau,
                       const pdhcg_params *params, float *x_out,
                       float *s_out);

/* Arrow-Debreu exchange market by the fixed-point iteration w <- E p(w)
 * (Sec. 4, Alg. 4).  E: device CSR (e_row_ptr[n+1], e_col[e_nnz],
 * e_val[e_nnz]) with column sums one (Sec. 4).  Each Fisher solve uses
 * `inner` and is warm-started from the previous prices and allocation.
 * Stops when ||p^k - p^{k-1}||_inf / ||p^{k-1}||_inf <= outer_tol; returns
 * PDHCG_OK then if the inner solve that produced p^k reached inner->tol,
 * else PDHCG_MAX_ITER (the small change may only reflect a solve cut off by
 * inner->max_iter), and PDHCG_MAX_ITER when outer_max ran out.
 *   w  [n] device: initial budgets on entry, final budgets E p on exit.
 *   p  [m], x [nnz] device: outputs.
 *   outer_iters, inner_iters: host, may be NULL. */
int32_t pdhcg_arrow_debreu(pdhcg_market market, const int32_t *e_row_ptr,
                           const int32_t *e_col, const float *e_val,
                           int64_t e_nnz, const pdhcg_params *inner,
                           double outer_tol, int32_t outer_max, float *w,
                           float *p, float *x, int32_t *outer_iters,
                           int64_t *inner_iters, pdhcg_info *info);

/* Gradient of a loss L(p) of the prices with respect to the utilities u
 * and budgets w, by reverse mode through `unroll` fixed-step PDHCG
 * iterations (the price step of eq. update:py and the row prox of Sec. 2.2,
 * tau = eta/omega, sigma = eta*omega, eta = 0.9/||K_x|| with K_x the
 * column-sum operator on the support of x: ||K_x|| = sqrt(the largest
 * number of buyers with x_ij > 0 of a good), Lemma 1's step condition for
 * the entries that move near the start point) started from
 * (x, p), normally the solution pdhcg_solve returned; the start point is
 * held constant, so at an equilibrium the result tends, as unroll grows, to
 * the derivative of the equilibrium prices (implicit function theorem on
 * the equilibrium conditions, Sec. 3).  The forward states are kept every
 * `ckpt_every` iterations and recomputed in between (memory
 * (unroll/ckpt_every + ckpt_every) nnz floats, allocated by the call).
 * Loss: L(p^unroll) with dL/dp given.
 *   x [nnz], p [m], dL_dp [m]: device inputs (float32);
 *   omega: the primal weight (pdhcg_info.omega of the solve), > 0;
 *   dL_du [nnz] (CSR order, the caller's unnormalised u), dL_dw [n]:
 *   device outputs.
 * Synchronises the handle's stream before returning.  ERR_ARG on null
 * pointers, omega <= 0, unroll < 1 or ckpt_every < 1; ERR_HIP / ERR_OOM on
 * device failures. */
int32_t pdhcg_backward(pdhcg_market market, const float *x, const float *p,
                       double omega, int32_t unroll, int32_t ckpt_every,
                       const float *dL_dp, float *dL_du, float *dL_dw);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as pdhcg_backward, with its workspace taken from
 * a fixed 64 MiB array that the library holds in each GPU's memory until the
 * process ends, instead of buffers allocated per call.  Calls no hipMalloc,
 * hipFree or allocating library routine.  The workspace needed is
 *   4 nnz (ceil(unroll/c) + c + 5) + 4 n + 8 m (3 ceil(unroll/c) + 23) + 4 (m + 1)
 * bytes (c = min(ckpt_every, unroll); each piece rounded up to 256 bytes);
 * above 64 MiB the call returns PDHCG_ERR_UNSUPPORTED before any device work.
 * Every call on one GPU uses that GPU's single array and leaves it dirty
 * (each call initialises what it reads): calls that overlap in time on one
 * GPU (other threads, other streams) race and must be serialised by the
 * caller.  Arguments, errors and synchronisation as pdhcg_backward. */
int32_t pdhcg_backward_noalloc(pdhcg_market market, const float *x,
                               const float *p, double omega, int32_t unroll,
                               int32_t ckpt_every, const float *dL_dp,
                               float *dL_du, float *dL_dw);

/* Number of market rows in each kernel bin and the bin shapes chosen at
 * creation (host arrays of length cap; returns the number of bins).  Rows of
 * up to 512 entries take G lanes x E entries per lane, the bins of equal G
 * merged into the largest E (unless PDHCG_MERGE_BINS=0).  Rows
 * above 512 entries have 0 lanes per row and, as entries per lane, the team
 * shape code: 1..5 for rows held in registers of teams of waves (up to
 * 1024, 2048, 4096, 8192 and 16384 entries), 0 for the one-wave-per-row
 * kernel. */
int32_t pdhcg_market_bins(pdhcg_market market, int32_t cap,
                          int32_t *lanes_per_row, int32_t *entries_per_lane,
                          int32_t *rows);

/* Number of goods whose prices and column partial sums the row kernels keep
 * in LDS: m when all fit, 0 when none is kept there, and in between when the
 * market's goods were relabelled by degree (most bought first) at creation
 * and only the first ones fit; the others are read from global memory and
 * summed with device atomics.  The relabelling is internal: every entry
 * point takes and returns goods in the caller's order.  Negative status for
 * a null market. */
int32_t pdhcg_market_lds_goods(pdhcg_market market);

void pdhcg_market_destroy(pdhcg_market market);

/* ---- Batched markets -------------------------------------------------- */

typedef struct pdhcg_batch_s *pdhcg_batch;

/* Create a batch of `count` independent Fisher markets (each as in
 * pdhcg_market_create).  n[count], m[count]: host arrays of market sizes
 * (1 <= m[b] <= 2048).  Device arrays, markets concatenated in order:
 *   row_ptr_cat [sum_b (n[b] + 1)]  each market's own CSR row pointer
 *                                   (starting at 0),
 *   col_cat, u_cat [sum_b nnz_b]    local good ids (0..m[b]-1) and
 *                                   utilities,
 *   w_cat [sum_b n[b]]              budgets.
 * Every market is validated (status of the first bad market is returned),
 * copied and row-normalised (Sec. 5).  The caller may free its inputs. */
int32_t pdhcg_batch_create(int32_t count, const int32_t *n, const int32_t *m,
                           const int32_t *row_ptr_cat, const int32_t *col_cat,
                           const float *u_cat, const float *w_cat, void *stream,
                           pdhcg_batch *out);

/* Solve every market of the batch by restarted PDHCG (Alg. 2 with the
 * Sec. 5 enhancements, active-set search) in ONE persistent launch: each
 * workgroup takes work from a queue (largest markets first) and runs a
 * market's whole solve, so markets converge and retire independently.  A
 * market holding more than half of the mean load per resident workgroup is
 * split over a gang of up to 4 workgroups (rows divided by entries) that
 * meet once per iteration to sum their column partials; the gangs' tickets
 * come first and never exceed the resident workgroups.  The launch (queue reset, persistent kernel)
 * is a HIP graph built at the first call and replayed; the parameters and
 * output pointers are read by the kernel from device memory.
 *   p_cat [sum m] and x_cat [sum nnz]: device outputs, concatenated like
 *   the inputs; infos [count]: host, per-market results (may be NULL);
 *   infos[b].seconds is market b's solve time on its workgroup and
 *   infos[b].row_pass_seconds the whole launch.
 * Returns PDHCG_OK when every market reached tol, PDHCG_MAX_ITER when some
 * market ran out of iterations, or the most negative error status. */
int32_t pdhcg_batch_solve(pdhcg_batch batch, const pdhcg_params *params,
                          float *p_cat, float *x_cat, pdhcg_info *infos);

/* Schedule of the batched launch: resident workgroups per CU and the row
 * shape policy (0: fewest lanes per row that hold the market's longest row,
 * 1: one size wider). */
typedef struct {
  int32_t wg_per_cu;
  int32_t shape_policy;
  int32_t trials;             /* configurations timed */
  double best_trial_seconds;  /* time of the chosen one */
} pdhcg_batch_schedule;

/* Pick the batch's schedule by timing it: every (wg_per_cu, shape_policy)
 * candidate solves the whole batch for trial_iters iterations per market
 * (tolerance ignored, outputs discarded; the markets' results are not
 * kept), and the fastest is kept for later pdhcg_batch_solve calls.  It
 * changes the schedule only, not what is computed.  out (host) may be NULL.
 * Errors: PDHCG_ERR_ARG for a null batch or trial_iters < 1; device
 * failures restore the previous schedule. */
int32_t pdhcg_batch_autotune(pdhcg_batch batch, const pdhcg_params *params,
                             int32_t trial_iters, pdhcg_batch_schedule *out);

/* Reverse mode for every market of the batch (as pdhcg_backward, market by
 * market on the batch's stream): from the batch solve's outputs x_cat,
 * p_cat and each market's primal weight omega[count] (host, infos[b].omega
 * of pdhcg_batch_solve), unroll fixed steps with checkpoints every
 * ckpt_every, dL_dp_cat [sum m] -> dL_du_cat [sum nnz], dL_dw_cat [sum n]
 * (device, concatenated like the inputs).  Errors: PDHCG_ERR_ARG for null
 * arguments, unroll or ckpt_every < 1 or a non-positive omega; the status
 * of the first market that fails otherwise. */
int32_t pdhcg_batch_backward(pdhcg_batch batch, const float *x_cat,
                             const float *p_cat, const double *omega,
                             int32_t unroll, int32_t ckpt_every,
                             const float *dL_dp_cat, float *dL_du_cat,
                             float *dL_dw_cat);

/* Offsets of market b's goods and edges in the concatenated arrays (host
 * arrays of count + 1 entries, either may be NULL). */
int32_t pdhcg_batch_layout(pdhcg_batch batch, int64_t *good_off,
                           int64_t *edge_off);

void pdhcg_batch_destroy(pdhcg_batch batch);

#ifdef __cplusplus
}
#endif

#endif /* PDHCG_H */
