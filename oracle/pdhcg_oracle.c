/*
 * pdhcg_oracle.c -- FP64 CPU oracle for restarted PDHCG on the Eisenberg-Gale
 * program of linear Fisher markets, and for the Arrow-Debreu fixed point.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU solver never
 * calls, links or includes anything from here, and this file includes nothing
 * from the GPU solver: the two implementations share no code.
 *
 * Paper: Liu, Huang, Li, Ge, Ye, "PDHCG: A Scalable First-Order Method for
 * Large-Scale Competitive Market Equilibrium Computation" (arXiv 2506.06258).
 *
 * Everything is double precision and written for clarity, not speed:
 *   - the row subproblem of Sec. 2.2 is solved exactly (active-set walk over
 *     sorted breakpoints); Alg. 3 (enhanced bisection) and the 32-section
 *     search of Sec. 2.2.1 are provided for cross-checks;
 *   - Alg. 2 (restarted PDHCG) with the price step of eq. (update:py), the
 *     running averages, and the enhancements listed in Sec. 5 (row
 *     normalisation, adaptive restart, primal weight), using the readings
 *     documented beside each function;
 *   - the relative KKT error of Sec. 5 ("Criteria");
 *   - Alg. 4 (fixed-point iteration for the Arrow-Debreu market).
 *
 * CSR convention: row_ptr has n+1 entries (int64), col has nnz entries
 * (int32, strictly increasing inside a row), values are aligned with col.
 */
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_MAX_ITER 1
#define ORA_ERR_ARG (-1)
#define ORA_ERR_ASSUMPTION (-2)
#define ORA_ERR_NUMERIC (-3)
#define ORA_ERR_OOM (-4)

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Row subproblem (Sec. 2.2).                                                */
/*                                                                          */
/*   min_{x_i >= 0}  -w_i log(u_i^T x_i) + p^T x_i + |x_i - x_i^k|^2/(2 tau)  */
/*                                                                          */
/* Its KKT conditions give x_ij = [x^k_ij - tau p_j + tau w_i u_ij / s]_+     */
/* with s = u_i^T x_i (eq. (bisection); the factor u_ij on the barrier term  */
/* follows from differentiating -w_i log(u_i^T x_i) with respect to x_ij).   */
/* Writing a_j = x^k_ij - tau p_j and b_j = tau w_i u_ij >= 0,               */
/*     g(s)   = sum_j u_ij [a_j + b_j / s]_+                                  */
/*     phi(s) = s - g(s)          (monotone increasing, unique root s* > 0)  */
/* ------------------------------------------------------------------------ */

/* g(s) = sum_j u_j [a_j + b_j/s]_+ */
static double row_g(int d, const double *u, const double *a, const double *b,
                    double s) {
  double g = 0.0;
  for (int j = 0; j < d; ++j) {
    double v = a[j] + b[j] / s;
    if (v > 0.0) g += u[j] * v;
  }
  return g;
}

/* x_j(s) = [a_j + b_j/s]_+   (eq. (bisection)) */
static void row_x(int d, const double *a, const double *b, double s,
                  double *x) {
  for (int j = 0; j < d; ++j) {
    double v = a[j] + b[j] / s;
    x[j] = v > 0.0 ? v : 0.0;
  }
}

/* Positive root of s^2 - A s - B = 0 (B >= 0), in the cancellation-free form. */
static double pos_root(double A, double B) {
  double disc = sqrt(A * A + 4.0 * B);
  if (A >= 0.0) return 0.5 * (A + disc);
  return (disc - A) > 0.0 ? 2.0 * B / (disc - A) : 0.0;
}

typedef struct {
  double c;  /* breakpoint b_j / (-a_j): the entry is active iff s < c */
  double ua; /* u_j a_j */
  double ub; /* u_j b_j */
} brk_t;

static int brk_desc(const void *p, const void *q) {
  double x = ((const brk_t *)p)->c, y = ((const brk_t *)q)->c;
  return (x < y) - (x > y);
}

/* Exact root s* of phi.  Entries with u_j > 0 and a_j >= 0 are active for
 * every s > 0; entries with u_j > 0 and a_j < 0 are active exactly when
 * s < c_j = b_j/(-a_j); entries with u_j = 0 do not enter g.  On a piece of
 * (0, inf) between consecutive breakpoints the active set is fixed, and
 * phi(s) = s - A - B/s there, with A = sum_act u a and B = sum_act u b.
 * Walk the pieces from the right: the root lies on the first piece whose
 * left end has phi <= 0, and on that piece it is the positive root of
 * s^2 - A s - B = 0.  Returns s*, or a negative value if the row has no
 * positive utility (Assumption 1 violated).  work must hold d entries. */
double ora_row_root_exact(int d, const double *u, const double *a,
                          const double *b, void *work) {
  brk_t *br = (brk_t *)work;
  int r = 0;
  double A = 0.0, B = 0.0;
  int any_pos = 0;
  for (int j = 0; j < d; ++j) {
    if (!(u[j] > 0.0)) continue;
    any_pos = 1;
    if (a[j] >= 0.0) {
      A += u[j] * a[j];
      B += u[j] * b[j];
    } else {
      br[r].c = b[j] / (-a[j]);
      br[r].ua = u[j] * a[j];
      br[r].ub = u[j] * b[j];
      ++r;
    }
  }
  if (!any_pos) return -1.0;
  qsort(br, (size_t)r, sizeof(brk_t), brk_desc);
  for (int q = 0; q <= r; ++q) {
    /* piece q: entries 0..q-1 of the sorted list are active, the rest not;
     * it spans [left, c_{q-1}] with left = c_q (or 0 when q == r). */
    double left = (q < r) ? br[q].c : 0.0;
    if (q == r || left - A - B / left <= 0.0) return pos_root(A, B);
    A += br[q].ua;
    B += br[q].ub;
  }
  return pos_root(A, B); /* not reached */
}

/* Row prox by the exact root: x = [a + b/s*]_+.  Returns s*. */
double ora_row_prox_exact(int d, const double *u, const double *xk,
                          const double *pg, double w, double tau, double *x,
                          void *work, double *ab) {
  double *a = ab, *b = ab + d;
  for (int j = 0; j < d; ++j) {
    a[j] = xk[j] - tau * pg[j];
    b[j] = tau * w * u[j];
  }
  double s = ora_row_root_exact(d, u, a, b, work);
  if (s > 0.0) row_x(d, a, b, s, x);
  return s;
}

/* A positive lower bound on s*: for each single good j, the root of
 * s = u_j (a_j + b_j/s) bounds s* from below because g(s) is at least that
 * one term.  Used as the trial value when u^T x^k = 0. */
static double single_good_lower(int d, const double *u, const double *a,
                                const double *b) {
  double L = 0.0;
  for (int j = 0; j < d; ++j) {
    if (!(u[j] > 0.0)) continue;
    double sj = pos_root(u[j] * a[j], u[j] * b[j]);
    if (sj > L) L = sj;
  }
  return L;
}

/* Alg. 3 (bisection search with the (s, s~) bracket of Sec. 2.2).
 * Trial s = u^T x^k; s~ = u^T x~(s); U = max, L = min; then midpoints until
 * U - L <= eps * U.  Output x~ of the last trial.  Returns the last trial s
 * and the number of bracket rounds in *rounds. */
double ora_row_prox_bisect(int d, const double *u, const double *xk,
                           const double *pg, double w, double tau, double eps,
                           int max_rounds, double *x, double *ab, int *rounds) {
  double *a = ab, *b = ab + d;
  double s = 0.0;
  for (int j = 0; j < d; ++j) {
    a[j] = xk[j] - tau * pg[j];
    b[j] = tau * w * u[j];
    s += u[j] * xk[j];
  }
  if (!(s > 0.0)) s = single_good_lower(d, u, a, b);
  double st = row_g(d, u, a, b, s);
  double U = st > s ? st : s, L = st > s ? s : st;
  int it = 0;
  while (U - L > eps * U && it < max_rounds) {
    s = 0.5 * (U + L);
    st = row_g(d, u, a, b, s);
    double hi = st > s ? st : s, lo = st > s ? s : st;
    if (hi < U) U = hi;
    if (lo > L) L = lo;
    ++it;
  }
  row_x(d, a, b, s, x);
  if (rounds) *rounds = it;
  return s;
}

/* k-section search (Sec. 2.2.1): K candidates s_l = (1 - l/(K+1)) L +
 * (l/(K+1)) U, l = 1..K, per round; U = min(U, min_l max(s_l, s~_l)),
 * L = max(L, max_l min(s_l, s~_l)).  The initial bracket is Alg. 3's.  The
 * output is x~ at the midpoint of the final bracket.  Lo and Hi receive the
 * final bracket (for invariant tests) when non-NULL. */
double ora_row_prox_ksection(int d, const double *u, const double *xk,
                             const double *pg, double w, double tau, int K,
                             double eps, int max_rounds, double *x, double *ab,
                             int *rounds, double *Lo, double *Hi) {
  double *a = ab, *b = ab + d;
  double s = 0.0;
  for (int j = 0; j < d; ++j) {
    a[j] = xk[j] - tau * pg[j];
    b[j] = tau * w * u[j];
    s += u[j] * xk[j];
  }
  if (!(s > 0.0)) s = single_good_lower(d, u, a, b);
  double st = row_g(d, u, a, b, s);
  double U = st > s ? st : s, L = st > s ? s : st;
  int it = 0;
  while (U - L > eps * U && it < max_rounds) {
    double newU = U, newL = L;
    for (int l = 1; l <= K; ++l) {
      double sl = (1.0 - (double)l / (K + 1)) * L + ((double)l / (K + 1)) * U;
      double gl = row_g(d, u, a, b, sl);
      double hi = gl > sl ? gl : sl, lo = gl > sl ? sl : gl;
      if (hi < newU) newU = hi;
      if (lo > newL) newL = lo;
    }
    U = newU;
    L = newL;
    ++it;
  }
  if (Lo) *Lo = L;
  if (Hi) *Hi = U;
  s = 0.5 * (L + U);
  row_x(d, a, b, s, x);
  if (rounds) *rounds = it;
  return s;
}

/* ------------------------------------------------------------------------ */
/* Relative KKT error (Sec. 5, "Criteria"), PDHCG form: t_i = u_i^T x_i and   */
/* y = w / t, so the terms |t - u^T x| and |w/t - y| vanish.  Maxima run over */
/* the stored entries of the sparse utility matrix.                          */
/*   r_primal = ||1^T x - 1||_inf / (1 + max(||1^T x||_inf, 1))             */
/*   r_dual   = max_j (p_j - M_j)_- / (1 + max(||y||_inf, max_j (p_j - M_j)))*/
/*              with M_j = max_i u_ij y_i                                    */
/*   r_gap    = max_ij x_ij (p_j - u_ij y_i)_+                               */
/*              / (1 + max(||x||_inf, max_ij (p_j - u_ij y_i)_+))           */
/* out[0..2] = r_primal, r_dual, r_gap; returns max of the three.           */
/* ------------------------------------------------------------------------ */
double ora_kkt(int n, int m, const int64_t *row_ptr, const int32_t *col,
               const double *u, const double *w, const double *x,
               const double *p, double *out) {
  double *c = (double *)calloc((size_t)m, sizeof(double));
  double *M = (double *)calloc((size_t)m, sizeof(double));
  double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  if (!c || !M || !y) {
    free(c); free(M); free(y);
    return NAN;
  }
  double ymax = 0.0, xmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double t = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) t += u[k] * x[k];
    y[i] = w[i] / t;
    if (y[i] > ymax) ymax = y[i];
  }
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int j = col[k];
      c[j] += x[k];
      double v = u[k] * y[i];
      if (v > M[j]) M[j] = v;
      if (x[k] > xmax) xmax = x[k];
    }
  double pr_num = 0.0, cmax = 0.0;
  double du_num = 0.0, du_pm = -INFINITY;
  for (int j = 0; j < m; ++j) {
    double e = fabs(c[j] - 1.0);
    if (e > pr_num) pr_num = e;
    if (fabs(c[j]) > cmax) cmax = fabs(c[j]);
    double dpm = p[j] - M[j];
    if (-dpm > du_num) du_num = -dpm;
    if (dpm > du_pm) du_pm = dpm;
  }
  double gap_num = 0.0, gap_pos = 0.0;
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      double r = p[col[k]] - u[k] * y[i];
      if (r > 0.0) {
        if (r > gap_pos) gap_pos = r;
        if (x[k] * r > gap_num) gap_num = x[k] * r;
      }
    }
  double rp = pr_num / (1.0 + (cmax > 1.0 ? cmax : 1.0));
  double dd = ymax > du_pm ? ymax : du_pm;
  double rd = du_num / (1.0 + dd);
  double gd = xmax > gap_pos ? xmax : gap_pos;
  double rg = gap_num / (1.0 + gd);
  free(c); free(M); free(y);
  if (out) { out[0] = rp; out[1] = rd; out[2] = rg; }
  double r = rp > rd ? rp : rd;
  return r > rg ? r : rg;
}

/* ------------------------------------------------------------------------ */
/* Restarted PDHCG (Alg. 2) with the enhancements of Sec. 5.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  double tol;          /* stop when the candidate's relative KKT <= tol     */
  int64_t max_iter;    /* iteration cap (PDHCG steps)                        */
  int32_t eval_every;  /* KKT / restart check period                         */
  int32_t restart;     /* 0: never restart, 1: adaptive restart              */
  double beta_sufficient, beta_necessary, beta_artificial;
  double theta;        /* primal-weight smoothing                            */
  int32_t omega_check_every; /* restarts between primal-weight bound checks */
  double omega_bound;  /* reset omega to omega0 outside [omega0/b, omega0*b] */
  double eta0;         /* <= 0: 1 (adaptive) or 0.9/||K|| (fixed)          */
  double omega0;       /* <= 0: sum(w) / (20 m)                             */
  int32_t output;      /* 0: restart candidate, 1: current, 2: average       */
  int32_t prox;        /* 0: exact, 1: Alg. 3 bisection, 2: k-section        */
  int32_t sections;    /* K for the k-section search                         */
  double prox_eps;     /* relative bracket width for prox 1/2                */
  int32_t normalize_rows; /* divide each row of u by its maximum            */
  int32_t verbose;
  int32_t step_mode;   /* 0: fixed eta, 1: adaptive eta in [0.01, 3]*eta0   */
} ora_params;

typedef struct {
  double rel_kkt, rel_primal, rel_dual, rel_gap;
  double eta, omega;
  int64_t iters;
  int32_t restarts;
  int32_t status;
  int64_t accepted;    /* steps kept by the adaptive step rule (all when fixed) */
  double emax_last;    /* the step-size bound eta_max of the last adaptive step */
} ora_info;

void ora_default_params(ora_params *prm) {
  memset(prm, 0, sizeof(*prm));
  prm->tol = 1e-4;
  prm->max_iter = 100000;
  prm->eval_every = 64;
  prm->restart = 1;
  prm->beta_sufficient = 0.2;
  prm->beta_necessary = 0.8;
  prm->beta_artificial = 0.2;
  prm->theta = 0.2;
  prm->omega_check_every = 3;
  prm->omega_bound = 1e4;
  prm->eta0 = 0.0;
  prm->omega0 = 0.0;
  prm->output = 0;
  prm->prox = 0;
  prm->sections = 32;
  prm->prox_eps = 1e-13;
  prm->normalize_rows = 1;
  prm->verbose = 0;
  prm->step_mode = 1;
}

/* Column sums c_j = sum_i x_ij. */
static void colsum(int n, int m, const int64_t *row_ptr, const int32_t *col,
                   const double *x, double *c) {
  for (int j = 0; j < m; ++j) c[j] = 0.0;
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) c[col[k]] += x[k];
}

static double dist2(int64_t len, const double *a, const double *b) {
  double s = 0.0;
  for (int64_t k = 0; k < len; ++k) s += (a[k] - b[k]) * (a[k] - b[k]);
  return s;
}

/* Validation: sizes, CSR shape, strictly increasing in-range columns,
 * finite non-negative u, finite positive w; Assumption 1 (Sec. 2) on the
 * positive entries: every buyer and every good has some u_ij > 0. */
int ora_validate(int n, int m, const int64_t *row_ptr, const int32_t *col,
                 const double *u, const double *w) {
  if (n <= 0 || m <= 0 || !row_ptr || !col || !u || !w) return ORA_ERR_ARG;
  if (row_ptr[0] != 0) return ORA_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return ORA_ERR_ARG;
    if (!(w[i] > 0.0) || !isfinite(w[i])) return ORA_ERR_ARG;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= m) return ORA_ERR_ARG;
      if (k > row_ptr[i] && col[k] <= col[k - 1]) return ORA_ERR_ARG;
      if (!(u[k] >= 0.0) || !isfinite(u[k])) return ORA_ERR_ARG;
    }
  }
  char *good = (char *)calloc((size_t)m, 1);
  if (!good) return ORA_ERR_OOM;
  int rc = ORA_OK;
  for (int i = 0; i < n && rc == ORA_OK; ++i) {
    int liked = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (u[k] > 0.0) { liked = 1; good[col[k]] = 1; }
    if (!liked) rc = ORA_ERR_ASSUMPTION;
  }
  for (int j = 0; j < m && rc == ORA_OK; ++j)
    if (!good[j]) rc = ORA_ERR_ASSUMPTION;
  free(good);
  return rc;
}

/* One prox sweep over all rows: x_new_i = prox(x_old_i; p, tau).  Returns
 * ORA_ERR_NUMERIC if a row has no positive root. */
static int prox_sweep(int n, const int64_t *row_ptr, const int32_t *col,
                      const double *uh, const double *w, const double *x_old,
                      const double *p, double tau, const ora_params *prm,
                      int dmax, double *x_new, double *s_out) {
  int bad = 0;
#pragma omp parallel reduction(| : bad) if (n >= 512)
  {
    double *pg = (double *)malloc((size_t)(dmax > 0 ? dmax : 1) * sizeof(double));
    double *ab = (double *)malloc((size_t)(dmax > 0 ? 2 * dmax : 2) * sizeof(double));
    brk_t *work = (brk_t *)malloc((size_t)(dmax > 0 ? dmax : 1) * sizeof(brk_t));
    if (!pg || !ab || !work) bad = 1;
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (bad) continue;
      int64_t b0 = row_ptr[i];
      int d = (int)(row_ptr[i + 1] - b0);
      for (int e = 0; e < d; ++e) pg[e] = p[col[b0 + e]];
      double s;
      if (prm->prox == 1)
        s = ora_row_prox_bisect(d, uh + b0, x_old + b0, pg, w[i], tau,
                                prm->prox_eps, 200, x_new + b0, ab, NULL);
      else if (prm->prox == 2)
        s = ora_row_prox_ksection(d, uh + b0, x_old + b0, pg, w[i], tau,
                                  prm->sections, prm->prox_eps, 200,
                                  x_new + b0, ab, NULL, NULL, NULL);
      else
        s = ora_row_prox_exact(d, uh + b0, x_old + b0, pg, w[i], tau,
                               x_new + b0, work, ab);
      if (!(s > 0.0) || !isfinite(s)) bad = 1;
      if (s_out) s_out[i] = s;
    }
    free(pg); free(ab); free(work);
  }
  return bad ? ORA_ERR_NUMERIC : ORA_OK;
}

/*
 * Solve the Fisher market (n buyers, m goods, utilities u on the CSR pattern,
 * budgets w) by restarted PDHCG.
 *
 * Readings of passages the paper leaves open (the same readings are used by
 * the GPU solver, which implements them independently):
 *  - preprocessing (Sec. 5): each row of u is divided by its maximum;
 *  - operator norm: K maps x to its column sums, K K^T = diag(column degree),
 *    so ||K|| = sqrt(max_j deg_j) (the sparse analogue of L = sqrt(n), Sec. 3);
 *  - initial point: x0_ij = 1/deg_j (column sums one), p0_j = sum(w)/m;
 *  - steps tau = eta/omega, sigma = eta*omega (Sec. 5).  Fixed mode:
 *    eta = 0.9/||K|| (sigma tau ||K||^2 < 1, Lemma 1).  Adaptive mode (the
 *    default): eta starts at 1 = 1/max|K_ij| and follows the rule in the
 *    loop, clamped to [0.01, 3] eta0 (Sec. 5); omega0 = sum(w)/(20 m);
 *  - the price step extrapolates with the column sums:
 *    p^{k+1} = p^k + sigma (2 c^k - c^{k-1} - 1), c = colsum(x) (eq. update:py);
 *    after a restart c^{k-1} := c^k;
 *  - averages: xbar^{k} is the mean of the iterates since the last restart
 *    (Alg. 2), likewise pbar;
 *  - every eval_every iterations the relative KKT error of the current and
 *    of the averaged point are computed; the one with the smaller error is
 *    the restart candidate; restart (to the candidate) when
 *      KKT_c <= beta_sufficient * KKT_0, or
 *      KKT_c <= beta_necessary * KKT_0 and KKT_c > KKT_c(previous check), or
 *      iterations since restart >= beta_artificial * total iterations,
 *    where KKT_0 is the error at the last restart point;
 *  - at each restart the primal weight is smoothed towards
 *    ||p^{n+1,0}-p^{n,0}|| / ||x^{n+1,0}-x^{n,0}||:
 *    omega = exp(theta log(dp/dx) + (1-theta) log omega); every
 *    omega_check_every restarts omega is reset to omega0 when it left
 *    [omega0/omega_bound, omega0*omega_bound];
 *  - stop when the candidate's error <= tol; the output is the candidate.
 *    When max_iter runs out, the last check's candidate is the output, with
 *    no restart decision at that check (Sec. 5 gives no rule there; a run
 *    cut at k iterations is then the first k iterations of a longer run).
 *
 * p[m], x[nnz]: if warm != 0 they hold the starting point on entry.  On exit
 * they hold the solution; t[n] (if non-NULL) receives u_i^T x_i in the
 * original (unnormalised) units.
 */
int ora_solve(int n, int m, const int64_t *row_ptr, const int32_t *col,
              const double *u, const double *w, const ora_params *prm,
              int warm, double *p, double *x, double *t, ora_info *info) {
  int rc = ora_validate(n, m, row_ptr, col, u, w);
  if (rc != ORA_OK) {
    if (info) info->status = rc;
    return rc;
  }
  int64_t nnz = row_ptr[n];
  int dmax = 0;
  for (int i = 0; i < n; ++i) {
    int d = (int)(row_ptr[i + 1] - row_ptr[i]);
    if (d > dmax) dmax = d;
  }
  double *uh = (double *)malloc((size_t)nnz * sizeof(double));
  double *xb = (double *)malloc((size_t)nnz * sizeof(double));
  double *xa = (double *)malloc((size_t)nnz * sizeof(double));
  double *xn = (double *)malloc((size_t)nnz * sizeof(double));
  double *rs = (double *)malloc((size_t)n * sizeof(double));
  double *deg = (double *)calloc((size_t)m, sizeof(double));
  double *c = (double *)malloc((size_t)m * sizeof(double));
  double *cp = (double *)malloc((size_t)m * sizeof(double));
  double *pb = (double *)malloc((size_t)m * sizeof(double));
  double *pa = (double *)malloc((size_t)m * sizeof(double));
  double *pn = (double *)malloc((size_t)m * sizeof(double));
  double *cn = (double *)malloc((size_t)m * sizeof(double));
  if (!uh || !xb || !xa || !xn || !rs || !deg || !c || !cp || !pb || !pa || !pn || !cn) {
    rc = ORA_ERR_OOM;
    goto done;
  }

  /* Preprocessing: u_hat = u / max_j u_ij (Sec. 5). */
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (u[k] > mx) mx = u[k];
    rs[i] = prm->normalize_rows ? mx : 1.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) uh[k] = u[k] / rs[i];
  }
  for (int64_t k = 0; k < nnz; ++k) deg[col[k]] += 1.0;
  double maxdeg = 0.0;
  for (int j = 0; j < m; ++j)
    if (deg[j] > maxdeg) maxdeg = deg[j];
  double Knorm = sqrt(maxdeg);

  double sumw = 0.0;
  for (int i = 0; i < n; ++i) sumw += w[i];
  if (!warm) {
    for (int i = 0; i < n; ++i)
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) x[k] = 1.0 / deg[col[k]];
    for (int j = 0; j < m; ++j) p[j] = sumw / m;
  }
  /* initial step: fixed mode uses the Chambolle-Pock bound 0.9/||K||; the
   * adaptive mode starts from 1/max_ij |K_ij| = 1 (K is a 0/1 matrix) */
  double eta0 = prm->eta0 > 0.0 ? prm->eta0 : (prm->step_mode == 1 ? 1.0 : 0.9 / Knorm);
  /* initial primal weight: a twentieth of the mean price sum(w)/m */
  double omega0 = prm->omega0 > 0.0 ? prm->omega0 : 0.05 * sumw / (double)m;
  double eta = eta0, omega = omega0;

  colsum(n, m, row_ptr, col, x, c);
  memcpy(cp, c, (size_t)m * sizeof(double));
  memcpy(xa, x, (size_t)nnz * sizeof(double));
  memcpy(pa, p, (size_t)m * sizeof(double));
  memcpy(xb, x, (size_t)nnz * sizeof(double));
  memcpy(pb, p, (size_t)m * sizeof(double));

  double kkt0 = ora_kkt(n, m, row_ptr, col, uh, w, x, p, NULL);
  double kkt_prev = INFINITY;
  int64_t k_in = 0, total = 0, accepted = 0;
  double emax_last = NAN;
  int restarts = 0;
  double kout[3] = {NAN, NAN, NAN}, kbest = INFINITY;
  int status = ORA_MAX_ITER;
  int cand_avg = 0;

  int64_t since = 0; /* iterations since the last restart */
  while (total < prm->max_iter) {
    double tau = eta / omega, sigma = eta * omega;
    /* price step (eq. update:py) */
    for (int j = 0; j < m; ++j) pn[j] = p[j] + sigma * (2.0 * c[j] - cp[j] - 1.0);
    /* primal step: exact prox of every row (Sec. 2.2) */
    rc = prox_sweep(n, row_ptr, col, uh, w, x, pn, tau, prm, dmax, xn, NULL);
    if (rc != ORA_OK) goto done;
    colsum(n, m, row_ptr, col, xn, cn);
    ++total;
    ++since;
    int accept = 1;
    if (prm->step_mode == 1) {
      /* adaptive step (Sec. 5): the step is kept when
       * eta <= eta_max = (omega |dx|^2 + |dp|^2/omega) / (2 |dp^T K dx|),
       * K dx being the change of the column sums; the next eta is
       * min((1-(k+1)^-0.3) eta_max, (1+(k+1)^-0.6) eta), clamped to
       * [0.01, 3] eta0.  A rejected step leaves (x, p) unchanged. */
      double dx2 = dist2(nnz, xn, x), dp2 = dist2(m, pn, p), inter = 0.0;
      for (int j = 0; j < m; ++j) inter += (pn[j] - p[j]) * (cn[j] - c[j]);
      double emax = fabs(inter) > 0.0 ? (omega * dx2 + dp2 / omega) / (2.0 * fabs(inter))
                                      : INFINITY;
      double kk = (double)(total + 1);
      double enew = fmin((1.0 - pow(kk, -0.3)) * emax, (1.0 + pow(kk, -0.6)) * eta);
      if (enew > 3.0 * eta0) enew = 3.0 * eta0;
      if (enew < 0.01 * eta0) enew = 0.01 * eta0;
      accept = (eta <= emax) || (eta <= 0.01 * eta0);
      eta = enew;
      emax_last = emax;
    }
    if (accept) {
      memcpy(x, xn, (size_t)nnz * sizeof(double));
      memcpy(p, pn, (size_t)m * sizeof(double));
      memcpy(cp, c, (size_t)m * sizeof(double));
      memcpy(c, cn, (size_t)m * sizeof(double));
      ++k_in;
      ++accepted;
      /* running averages over the iterates since the last restart (Alg. 2) */
      for (int64_t k = 0; k < nnz; ++k) xb[k] += (x[k] - xb[k]) / (double)k_in;
      for (int j = 0; j < m; ++j) pb[j] += (p[j] - pb[j]) / (double)k_in;
    }

    int eval = (total % prm->eval_every == 0) || total == prm->max_iter;
    if (!eval) continue;
    if (k_in == 0) { /* no step kept since the restart: the average is the start */
      memcpy(xb, x, (size_t)nnz * sizeof(double));
      memcpy(pb, p, (size_t)m * sizeof(double));
    }
    double kc[3], ka[3];
    double ec = ora_kkt(n, m, row_ptr, col, uh, w, x, p, kc);
    double ea = ora_kkt(n, m, row_ptr, col, uh, w, xb, pb, ka);
    if (!isfinite(ec) || !isfinite(ea)) {
      rc = ORA_ERR_NUMERIC;
      goto done;
    }
    cand_avg = ea < ec;
    double kcand = cand_avg ? ea : ec;
    memcpy(kout, cand_avg ? ka : kc, sizeof(kout));
    kbest = kcand;
    if (prm->verbose)
      fprintf(stderr, "[oracle] it=%lld kin=%lld cur=%.3e (%.2e %.2e %.2e) avg=%.3e (%.2e %.2e %.2e) eta=%.3e omega=%.3e\n",
              (long long)total, (long long)k_in, ec, kc[0], kc[1], kc[2], ea, ka[0], ka[1], ka[2], eta, omega);
    if (kcand <= prm->tol) {
      status = ORA_OK;
      break;
    }
    if (total >= prm->max_iter) break;
    if (prm->restart) {
      int do_restart = (kcand <= prm->beta_sufficient * kkt0) ||
                       (kcand <= prm->beta_necessary * kkt0 && kcand > kkt_prev) ||
                       ((double)since >= prm->beta_artificial * (double)total);
      if (do_restart) {
        if (cand_avg) {
          memcpy(x, xb, (size_t)nnz * sizeof(double));
          memcpy(p, pb, (size_t)m * sizeof(double));
          colsum(n, m, row_ptr, col, x, c);
        }
        memcpy(cp, c, (size_t)m * sizeof(double));
        double dx = sqrt(dist2(nnz, x, xa)), dp = sqrt(dist2(m, p, pa));
        if (dx > 1e-10 && dp > 1e-10)
          omega = exp(prm->theta * log(dp / dx) + (1.0 - prm->theta) * log(omega));
        ++restarts;
        if (prm->omega_check_every > 0 && restarts % prm->omega_check_every == 0 &&
            (omega < omega0 / prm->omega_bound || omega > omega0 * prm->omega_bound))
          omega = omega0;
        memcpy(xa, x, (size_t)nnz * sizeof(double));
        memcpy(pa, p, (size_t)m * sizeof(double));
        kkt0 = kcand;
        kkt_prev = INFINITY;
        k_in = 0;
        since = 0;
        cand_avg = 0; /* x, p now hold the candidate */
      } else {
        kkt_prev = kcand;
      }
    }
  }

  /* output */
  if (prm->output == 2 || (prm->output == 0 && cand_avg)) {
    memcpy(x, xb, (size_t)nnz * sizeof(double));
    memcpy(p, pb, (size_t)m * sizeof(double));
  }
  if (prm->output != 0) {
    kbest = ora_kkt(n, m, row_ptr, col, uh, w, x, p, kout);
  }
  if (t)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += u[k] * x[k];
      t[i] = s;
    }
  if (info) {
    info->rel_kkt = kbest;
    info->rel_primal = kout[0];
    info->rel_dual = kout[1];
    info->rel_gap = kout[2];
    info->eta = eta;
    info->omega = omega;
    info->iters = total;
    info->restarts = restarts;
    info->status = status;
    info->accepted = accepted;
    info->emax_last = emax_last;
  }
  rc = status;

done:
  free(uh); free(xb); free(xa); free(xn); free(rs); free(deg);
  free(c); free(cp); free(pb); free(pa); free(pn); free(cn);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Arrow-Debreu exchange market by fixed-point iteration (Sec. 4, Alg. 4).   */
/* T(w) = E p(w): each inner Fisher solve is warm-started from the previous  */
/* (x, p).  E is n x m with column sums one, so sum(T(w)) = sum(w).          */
/* Stop when ||p^{k} - p^{k-1}||_inf / ||p^{k-1}||_inf <= outer_tol.         */
/* w[n] holds w^0 on entry and the last budgets on exit; p[m] the prices.    */
/* ------------------------------------------------------------------------ */
int ora_arrow_debreu(int n, int m, const int64_t *row_ptr, const int32_t *col,
                     const double *u, const int64_t *e_row_ptr,
                     const int32_t *e_col, const double *e_val,
                     const ora_params *inner, double outer_tol, int outer_max,
                     double *w, double *p, double *x, int *outer_iters,
                     int64_t *inner_iters, double *last_change) {
  int64_t nnz = row_ptr[n];
  double *pprev = (double *)malloc((size_t)m * sizeof(double));
  if (!pprev) return ORA_ERR_OOM;
  int rc = ORA_MAX_ITER, warm = 0;
  int64_t tot_inner = 0;
  double change = INFINITY;
  int k;
  (void)nnz;
  for (k = 0; k < outer_max; ++k) {
    ora_info info;
    int r = ora_solve(n, m, row_ptr, col, u, w, inner, warm, p, x, NULL, &info);
    tot_inner += info.iters;
    if (r < 0) { rc = r; break; }
    warm = 1;
    if (k > 0) {
      double num = 0.0, den = 0.0;
      for (int j = 0; j < m; ++j) {
        double dj = fabs(p[j] - pprev[j]);
        if (dj > num) num = dj;
        if (fabs(pprev[j]) > den) den = fabs(pprev[j]);
      }
      change = num / den;
    }
    memcpy(pprev, p, (size_t)m * sizeof(double));
    /* w <- E p */
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int64_t q = e_row_ptr[i]; q < e_row_ptr[i + 1]; ++q) s += e_val[q] * p[e_col[q]];
      w[i] = s;
    }
    /* p^k = p(E p^{k-1}) close to p^{k-1} certifies a fixed point only when
     * the solve that produced p^k reached its tolerance */
    if (k > 0 && change <= outer_tol) { rc = (r == ORA_OK) ? ORA_OK : ORA_MAX_ITER; ++k; break; }
  }
  if (outer_iters) *outer_iters = k;
  if (inner_iters) *inner_iters = tot_inner;
  if (last_change) *last_change = change;
  free(pprev);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Derivatives of the equilibrium prices with respect to u and w, by the    */
/* implicit function theorem on the equilibrium conditions (the KKT system  */
/* of Sec. 3, eq. KKT-system-pdhcg) restricted to the active support        */
/* S = {(i,j) : x_ij > act_tol}.  Unknowns z = (x_S, p, a) with a_i the     */
/* buyer's best utility per unit of money (Fact 1: every bought good        */
/* attains it):                                                             */
/*   F_ij = u_ij - a_i p_j                 for (i,j) in S,                  */
/*   F_i  = sum_{j:(i,j) in S} p_j x_ij - w_i       (budget spent),         */
/*   F_j  = sum_{i:(i,j) in S} x_ij - 1              (market clears).        */
/* J = dF/dz is square (|S| + m + n).  For a loss L(p), J^T lam = dL/dz     */
/* (dL/dp in the p block, zero elsewhere) and dL/dtheta = -(dF/dtheta)^T    */
/* lam; dF_ij/du_ij = 1 and dF_i/dw_i = -1 give                             */
/*   dL/du_ij = -lam_ij on S, 0 off S;   dL/dw_i = lam_i.                   */
/* Off S the derivative is zero because a nondegenerate equilibrium keeps   */
/* its support under small perturbations.  u is the caller's (not row-      */
/* normalised) utility: the conditions are homogeneous in each row.         */
/* Dense Gaussian elimination with partial pivoting: small markets only.    */
/* Returns ORA_ERR_NUMERIC when J is singular (a degenerate support) and    */
/* writes the size of the system to *dim.                                   */
/* ------------------------------------------------------------------------ */
static int dense_solve(int N, double *A, double *b) {
  /* A row-major N x N, overwritten; b overwritten by the solution */
  double amax = 0.0;
  for (int64_t q = 0; q < (int64_t)N * N; ++q) amax = fmax(amax, fabs(A[q]));
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int r = k + 1; r < N; ++r)
      if (fabs(A[(int64_t)r * N + k]) > fabs(A[(int64_t)piv * N + k])) piv = r;
    if (!(fabs(A[(int64_t)piv * N + k]) > 1e-12 * amax)) return ORA_ERR_NUMERIC;
    if (piv != k) {
      for (int c = 0; c < N; ++c) {
        double t = A[(int64_t)k * N + c];
        A[(int64_t)k * N + c] = A[(int64_t)piv * N + c];
        A[(int64_t)piv * N + c] = t;
      }
      double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int r = k + 1; r < N; ++r) {
      double f = A[(int64_t)r * N + k] / A[(int64_t)k * N + k];
      if (f == 0.0) continue;
      for (int c = k; c < N; ++c) A[(int64_t)r * N + c] -= f * A[(int64_t)k * N + c];
      b[r] -= f * b[k];
    }
  }
  for (int k = N - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < N; ++c) s -= A[(int64_t)k * N + c] * b[c];
    b[k] = s / A[(int64_t)k * N + k];
  }
  return ORA_OK;
}

int ora_implicit_grad(int n, int m, const int64_t *row_ptr, const int32_t *col,
                      const double *u, const double *w, const double *x, const double *p,
                      const double *dL_dp, double act_tol, double *dL_du, double *dL_dw,
                      int *dim) {
  (void)w;
  int64_t nnz = row_ptr[n];
  int64_t *sidx = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
  int32_t *srow = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
  double *a = (double *)calloc((size_t)n, sizeof(double));
  if (!sidx || !srow || !a) { free(sidx); free(srow); free(a); return ORA_ERR_OOM; }
  int S = 0;
  for (int i = 0; i < n; ++i) {
    int cnt = 0;
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
      if (x[q] > act_tol) {
        sidx[S] = q;
        srow[S] = i;
        ++S;
        a[i] += u[q] / p[col[q]];
        ++cnt;
      }
    if (cnt == 0) { free(sidx); free(srow); free(a); return ORA_ERR_NUMERIC; }
    a[i] /= cnt;
  }
  const int N = S + m + n;
  if (dim) *dim = N;
  double *J = (double *)calloc((size_t)N * N, sizeof(double));
  double *At = (double *)malloc((size_t)N * N * sizeof(double));
  double *lam = (double *)calloc((size_t)N, sizeof(double));
  if (!J || !At || !lam) {
    free(J); free(At); free(lam); free(sidx); free(srow); free(a);
    return ORA_ERR_OOM;
  }
  /* unknown columns: x_S -> [0, S), p -> [S, S+m), a -> [S+m, N)           */
  /* equation rows:   F_ij -> [0, S), F_i -> [S, S+n), F_j -> [S+n, N)      */
#define JX(r, c) J[(int64_t)(r) * N + (c)]
  for (int s = 0; s < S; ++s) {
    const int i = srow[s];
    const int j = col[sidx[s]];
    JX(s, S + m + i) = -p[j];         /* dF_ij/da_i */
    JX(s, S + j) = -a[i];             /* dF_ij/dp_j */
    JX(S + i, s) = p[j];              /* dF_i/dx_ij */
    JX(S + i, S + j) += x[sidx[s]];   /* dF_i/dp_j  */
    JX(S + n + j, s) = 1.0;           /* dF_j/dx_ij */
  }
#undef JX
  for (int r = 0; r < N; ++r)
    for (int c = 0; c < N; ++c) At[(int64_t)r * N + c] = J[(int64_t)c * N + r];
  for (int j = 0; j < m; ++j) lam[S + j] = dL_dp[j];
  int rc = dense_solve(N, At, lam);
  if (rc == ORA_OK) {
    for (int64_t q = 0; q < nnz; ++q) dL_du[q] = 0.0;
    for (int s = 0; s < S; ++s) dL_du[sidx[s]] = -lam[s];
    for (int i = 0; i < n; ++i) dL_dw[i] = lam[S + i];
  }
  free(J); free(At); free(lam); free(sidx); free(srow); free(a);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Reverse mode through K fixed-step PDHCG iterations (the price step of    */
/* eq. update:py and the exact row prox of Sec. 2.2) started from a given   */
/* point (x0, p0), for a loss L(p_K) of the final prices.  The start point  */
/* is held constant, so as K grows the result tends to the derivative of    */
/* the fixed point, i.e. to ora_implicit_grad at an equilibrium.            */
/*                                                                          */
/* Forward, k = 0..K-1 (c^{-1} = colsum(x0)):                               */
/*   c^k = colsum(x^k);  p^{k+1} = p^k + sigma (2 c^k - c^{k-1} - 1);       */
/*   x^{k+1}_i = prox_i(x^k_i - tau p^{k+1}; w_i, uh_i).                    */
/* Row prox derivative: on the active set A (x^{k+1}_ij > 0) with           */
/* s = sum_A uh_j x^{k+1}_j, x_j = a_j + tau w uh_j / s, so for an incoming */
/* adjoint g_j = dL/dx^{k+1}_ij:                                            */
/*   D = 1 + tau w sum_A uh_j^2 / s^2,                                      */
/*   h = (tau w / s^2) sum_A g_j uh_j / D,  r_j = g_j - h uh_j on A, 0 off; */
/*   dL/da_j = r_j,  dL/dw_i += (tau/s) sum_A r_j uh_j,                     */
/*   dL/duh_j += r_j tau w / s - h x^{k+1}_j  (on A).                       */
/* With a = x^k - tau p^{k+1} and the linear price step:                    */
/*   Pt = dL/dp^{k+1} - tau colsum(r);  dL/dp^k = Pt;                       */
/*   dL/dx^k_ij = r_ij + 2 sigma Pt_j + Cn_j,  Cn_j = dL/dc^k from step k+1;*/
/*   dL/dc^{k-1} = -sigma Pt.                                               */
/* Finally through uh = u / max_j u_ij (first maximum):                     */
/*   dL/du_ij = g_ij / r_i - [j = argmax] sum_k uh_ik g_ik / r_i.           */
/* p_out (nullable) receives p^K.  Stores all K+1 iterates: small markets.  */
/* ------------------------------------------------------------------------ */
int ora_unrolled_grad(int n, int m, const int64_t *row_ptr, const int32_t *col,
                      const double *u, const double *w, const double *x0, const double *p0,
                      double tau, double sigma, int K, const double *dL_dp, double *dL_du,
                      double *dL_dw, double *p_out) {
  int rc = ora_validate(n, m, row_ptr, col, u, w);
  if (rc != ORA_OK) return rc;
  if (K < 0 || !(tau > 0.0) || !(sigma > 0.0)) return ORA_ERR_ARG;
  const int64_t nnz = row_ptr[n];
  int dmax = 0;
  for (int i = 0; i < n; ++i) {
    int d = (int)(row_ptr[i + 1] - row_ptr[i]);
    if (d > dmax) dmax = d;
  }
  double *uh = (double *)malloc((size_t)nnz * sizeof(double));
  double *rs = (double *)malloc((size_t)n * sizeof(double));
  double *xs = (double *)malloc((size_t)(K + 1) * (size_t)nnz * sizeof(double));
  double *p = (double *)malloc((size_t)m * sizeof(double));
  double *c = (double *)malloc((size_t)m * sizeof(double));
  double *cprev = (double *)malloc((size_t)m * sizeof(double));
  double *R = (double *)calloc((size_t)nnz, sizeof(double));
  double *r = (double *)calloc((size_t)nnz, sizeof(double));
  double *duh = (double *)calloc((size_t)nnz, sizeof(double));
  double *B = (double *)calloc((size_t)m, sizeof(double));
  double *P = (double *)malloc((size_t)m * sizeof(double));
  double *Cn = (double *)calloc((size_t)m, sizeof(double));
  double *rc_col = (double *)malloc((size_t)m * sizeof(double));
  if (!uh || !rs || !xs || !p || !c || !cprev || !R || !r || !duh || !B || !P || !Cn || !rc_col) {
    rc = ORA_ERR_OOM;
    goto done;
  }
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (u[k] > mx) mx = u[k];
    rs[i] = mx;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) uh[k] = u[k] / mx;
  }
  /* forward */
  ora_params prm;
  ora_default_params(&prm);
  prm.prox = 0;
  memcpy(xs, x0, (size_t)nnz * sizeof(double));
  memcpy(p, p0, (size_t)m * sizeof(double));
  colsum(n, m, row_ptr, col, x0, cprev);
  for (int k = 0; k < K; ++k) {
    const double *xk = xs + (size_t)k * nnz;
    colsum(n, m, row_ptr, col, xk, c);
    for (int j = 0; j < m; ++j) p[j] += sigma * (2.0 * c[j] - cprev[j] - 1.0);
    rc = prox_sweep(n, row_ptr, col, uh, w, xk, p, tau, &prm, dmax, xs + (size_t)(k + 1) * nnz,
                    NULL);
    if (rc != ORA_OK) goto done;
    memcpy(cprev, c, (size_t)m * sizeof(double));
  }
  if (p_out) memcpy(p_out, p, (size_t)m * sizeof(double));
  /* reverse: dL/dx^{k+1} = R + B[col], dL/dp^{k+1} = P, dL/dc^k = Cn */
  memcpy(P, dL_dp, (size_t)m * sizeof(double));
  for (int i = 0; i < n; ++i) dL_dw[i] = 0.0;
  for (int k = K - 1; k >= 0; --k) {
    const double *xn = xs + (size_t)(k + 1) * nnz;
    for (int i = 0; i < n; ++i) {
      double s = 0.0, Q = 0.0, Gu = 0.0;
      for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        if (xn[q] > 0.0) {
          const double g = R[q] + B[col[q]];
          s += uh[q] * xn[q];
          Q += uh[q] * uh[q];
          Gu += g * uh[q];
        }
      }
      const double D = 1.0 + tau * w[i] * Q / (s * s);
      const double h = (tau * w[i] / (s * s)) * Gu / D;
      double ru = 0.0;
      for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        if (xn[q] > 0.0) {
          const double g = R[q] + B[col[q]];
          r[q] = g - h * uh[q];
          ru += r[q] * uh[q];
          duh[q] += r[q] * tau * w[i] / s - h * xn[q];
        } else {
          r[q] = 0.0;
        }
      }
      dL_dw[i] += tau / s * ru;
    }
    colsum(n, m, row_ptr, col, r, rc_col);
    for (int j = 0; j < m; ++j) {
      const double Pt = P[j] - tau * rc_col[j];
      B[j] = 2.0 * sigma * Pt + Cn[j];
      Cn[j] = -sigma * Pt;
      P[j] = Pt;
    }
    memcpy(R, r, (size_t)nnz * sizeof(double));
  }
  /* through the row normalisation */
  for (int i = 0; i < n; ++i) {
    double gs = 0.0;
    int64_t qmax = row_ptr[i];
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
      gs += uh[q] * duh[q];
      if (u[q] > u[qmax]) qmax = q;
    }
    for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) dL_du[q] = duh[q] / rs[i];
    dL_du[qmax] -= gs / rs[i];
  }
  rc = ORA_OK;
done:
  free(uh); free(rs); free(xs); free(p); free(c); free(cprev); free(R); free(r); free(duh);
  free(B); free(P); free(Cn); free(rc_col);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Restarted PDHG on the reformulated program (Sec. 2.1, Alg. 1) with the    */
/* enhancements of Sec. 5.  Primal (x, t), dual (p, y) of                    */
/*   L = -sum_i w_i log t_i + p^T (1^T x - 1) + y^T (t - U x)               */
/* (eq. primal-dual-formulation), u normalised per row as in ora_solve.      */
/* ------------------------------------------------------------------------ */

/* Relative KKT error (Sec. 5, "Criteria") of a point (x, t, p, y) of the
 * reformulated program, with r_i = u_i^T x_i and M_j = max_i u_ij y_i over
 * the stored entries:
 *   r_primal = max(||1^T x - 1||_inf, max_i |t_i - r_i|)
 *              / (1 + max(||1^T x||_inf, max_i |t_i - r_i|, 1))
 *   r_dual   = max(||w/t - y||_inf, max_j (p_j - M_j)_-)
 *              / (1 + max(||w/t||_inf, ||y||_inf, max_j (p_j - M_j)))
 *   r_gap    = max_ij x_ij (p_j - u_ij y_i)_+
 *              / (1 + max(||x||_inf, max_ij (p_j - u_ij y_i)_+))
 * out[0..2] = r_primal, r_dual, r_gap; returns the largest. */
double ora_kkt_ty(int n, int m, const int64_t *row_ptr, const int32_t *col,
                  const double *u, const double *w, const double *x, const double *t,
                  const double *p, const double *y, double *out) {
  double *c = (double *)calloc((size_t)m, sizeof(double));
  double *M = (double *)malloc((size_t)m * sizeof(double));
  if (!c || !M) {
    free(c); free(M);
    return NAN;
  }
  for (int j = 0; j < m; ++j) M[j] = -INFINITY;
  double tr = 0.0, wty = 0.0, wt = 0.0, ya = 0.0, xmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double r = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int j = col[k];
      r += u[k] * x[k];
      c[j] += x[k];
      double v = u[k] * y[i];
      if (v > M[j]) M[j] = v;
      if (fabs(x[k]) > xmax) xmax = fabs(x[k]);
    }
    if (fabs(t[i] - r) > tr) tr = fabs(t[i] - r);
    double q = w[i] / t[i];
    if (fabs(q - y[i]) > wty) wty = fabs(q - y[i]);
    if (fabs(q) > wt) wt = fabs(q);
    if (fabs(y[i]) > ya) ya = fabs(y[i]);
  }
  double cres = 0.0, cmax = 0.0, dneg = 0.0, dmax = -INFINITY;
  for (int j = 0; j < m; ++j) {
    if (fabs(c[j] - 1.0) > cres) cres = fabs(c[j] - 1.0);
    if (fabs(c[j]) > cmax) cmax = fabs(c[j]);
    double d = p[j] - M[j];
    if (-d > dneg) dneg = -d;
    if (d > dmax) dmax = d;
  }
  double gnum = 0.0, gpos = 0.0;
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      double r = p[col[k]] - u[k] * y[i];
      if (r > 0.0) {
        if (r > gpos) gpos = r;
        if (x[k] * r > gnum) gnum = x[k] * r;
      }
    }
  double pn = cres > tr ? cres : tr;
  double pd = cmax;
  if (tr > pd) pd = tr;
  if (1.0 > pd) pd = 1.0;
  double rp = pn / (1.0 + pd);
  double dn = wty > dneg ? wty : dneg;
  double dd = wt > ya ? wt : ya;
  if (dmax > dd) dd = dmax;
  double rd = dn / (1.0 + dd);
  double gd = xmax > gpos ? xmax : gpos;
  double rg = gnum / (1.0 + gd);
  free(c); free(M);
  if (out) { out[0] = rp; out[1] = rd; out[2] = rg; }
  double r = rp > rd ? rp : rd;
  return r > rg ? r : rg;
}

/* Row sums r_i = u_i^T x_i. */
static void rowsum(int n, const int64_t *row_ptr, const double *u, const double *x, double *r) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += u[k] * x[k];
    r[i] = s;
  }
}

/* One PDHG iteration (Alg. 1) on the normalised market u:
 *   p' = p + sigma (2 c - c_prev - 1),  c = 1^T x            (eq. update:py)
 *   y' = y + sigma (2 g - g_prev),      g = t - U x          (eq. update:py)
 *   t' = (t - tau y' + sqrt((tau y' - t)^2 + 4 tau w)) / 2   (eq. update:t)
 *   x' = max(0, x - tau (p'_j - u_ij y'_i))                  (eq. update:x)
 * c_prev, g_prev are the column sums and utility residuals of the previous
 * iterate.  Outputs x2[nnz], t2[n], p2[m], y2[n]. */
void ora_pdhg_step(int n, int m, const int64_t *row_ptr, const int32_t *col,
                   const double *u, const double *w, const double *x, const double *t,
                   const double *p, const double *y, const double *c_prev,
                   const double *g_prev, double tau, double sigma, double *x2, double *t2,
                   double *p2, double *y2) {
  double *c = (double *)malloc((size_t)m * sizeof(double));
  double *r = (double *)malloc((size_t)n * sizeof(double));
  colsum(n, m, row_ptr, col, x, c);
  rowsum(n, row_ptr, u, x, r);
  for (int j = 0; j < m; ++j) p2[j] = p[j] + sigma * (2.0 * c[j] - c_prev[j] - 1.0);
  for (int i = 0; i < n; ++i) {
    double g = t[i] - r[i];
    y2[i] = y[i] + sigma * (2.0 * g - g_prev[i]);
    double b = tau * y2[i] - t[i];
    t2[i] = (-b + sqrt(b * b + 4.0 * tau * w[i])) / 2.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      double v = x[k] - tau * (p2[col[k]] - u[k] * y2[i]);
      x2[k] = v > 0.0 ? v : 0.0;
    }
  }
  free(c); free(r);
}

/*
 * Solve the Fisher market by restarted PDHG (Alg. 1) with the Sec. 5
 * enhancements, which the paper applies to both PDHG and PDHCG.  Readings
 * (shared with ora_solve where they apply):
 *  - initial point: x0_ij = 1/deg_j, p0_j = sum(w)/m, t0 = U x0 (the utility
 *    constraint holds), y0 = w / t0 (the dual residual w/t - y is zero);
 *  - steps tau = eta/omega, sigma = eta*omega.  Adaptive mode: eta0 = 1 =
 *    max |K_ij| (|u_ij| <= 1 after normalisation, the t column is 1) and
 *    the rule of ora_solve with primal norm |dx|^2 + |dt|^2, dual norm
 *    |dp|^2 + |dy|^2 and interaction dp^T (1^T dx) + dy^T (dt - U dx).
 *    Fixed mode: eta = 0.9 / B with
 *    B = sqrt(max_j deg_j) + 1 + sqrt(max_j deg_j * max_i deg_i) >= ||K||
 *    (K = [1^T 0; -U I], |u_ij| <= 1), so sigma tau ||K||^2 < 1;
 *  - restarts, primal weight and stop test as in ora_solve, with the KKT
 *    error of ora_kkt_ty and primal/dual distances over (x, t) / (p, y);
 *    after a restart c_prev := c, g_prev := g.
 * p[m], x[nnz], t[n], y[n]: outputs (t, y in the normalised units). */
int ora_pdhg_solve(int n, int m, const int64_t *row_ptr, const int32_t *col,
                   const double *u_in, const double *w, const ora_params *prm,
                   double *p, double *x, double *t, double *y, ora_info *info) {
  int rc = ora_validate(n, m, row_ptr, col, u_in, w);
  if (rc != ORA_OK) {
    if (info) info->status = rc;
    return rc;
  }
  int64_t nnz = row_ptr[n];
  double *u = (double *)malloc((size_t)nnz * sizeof(double));
  double *X[4], *T[4], *P[4], *Y[4];  /* 0 current, 1 trial, 2 average, 3 anchor */
  for (int q = 0; q < 4; ++q) {
    X[q] = (double *)malloc((size_t)nnz * sizeof(double));
    T[q] = (double *)malloc((size_t)n * sizeof(double));
    P[q] = (double *)malloc((size_t)m * sizeof(double));
    Y[q] = (double *)malloc((size_t)n * sizeof(double));
  }
  double *c = (double *)malloc((size_t)m * sizeof(double));
  double *cp = (double *)malloc((size_t)m * sizeof(double));
  double *cn = (double *)malloc((size_t)m * sizeof(double));
  double *g = (double *)malloc((size_t)n * sizeof(double));
  double *gp = (double *)malloc((size_t)n * sizeof(double));
  double *gn = (double *)malloc((size_t)n * sizeof(double));
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *deg = (double *)calloc((size_t)m, sizeof(double));

  /* preprocessing (Sec. 5) */
  int maxrow = 0;
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (u_in[k] > mx) mx = u_in[k];
    if (!prm->normalize_rows) mx = 1.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) u[k] = u_in[k] / mx;
    if ((int)(row_ptr[i + 1] - row_ptr[i]) > maxrow) maxrow = (int)(row_ptr[i + 1] - row_ptr[i]);
  }
  for (int64_t k = 0; k < nnz; ++k) deg[col[k]] += 1.0;
  double maxcol = 0.0, sumw = 0.0;
  for (int j = 0; j < m; ++j)
    if (deg[j] > maxcol) maxcol = deg[j];
  for (int i = 0; i < n; ++i) sumw += w[i];
  double Kbound = sqrt(maxcol) + 1.0 + sqrt(maxcol * (double)maxrow);

  /* initial point */
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) X[0][k] = 1.0 / deg[col[k]];
  for (int j = 0; j < m; ++j) P[0][j] = sumw / m;
  rowsum(n, row_ptr, u, X[0], T[0]);
  for (int i = 0; i < n; ++i) Y[0][i] = w[i] / T[0][i];
  colsum(n, m, row_ptr, col, X[0], c);
  memcpy(cp, c, (size_t)m * sizeof(double));
  for (int i = 0; i < n; ++i) g[i] = 0.0;
  memcpy(gp, g, (size_t)n * sizeof(double));
  memcpy(X[2], X[0], (size_t)nnz * sizeof(double));
  memcpy(T[2], T[0], (size_t)n * sizeof(double));
  memcpy(P[2], P[0], (size_t)m * sizeof(double));
  memcpy(Y[2], Y[0], (size_t)n * sizeof(double));
  memcpy(X[3], X[0], (size_t)nnz * sizeof(double));
  memcpy(T[3], T[0], (size_t)n * sizeof(double));
  memcpy(P[3], P[0], (size_t)m * sizeof(double));
  memcpy(Y[3], Y[0], (size_t)n * sizeof(double));

  double eta0 = prm->eta0 > 0.0 ? prm->eta0 : (prm->step_mode == 1 ? 1.0 : 0.9 / Kbound);
  double omega0 = prm->omega0 > 0.0 ? prm->omega0 : 0.05 * sumw / (double)m;
  double eta = eta0, omega = omega0;
  double kkt0 = ora_kkt_ty(n, m, row_ptr, col, u, w, X[0], T[0], P[0], Y[0], NULL);
  double kkt_prev = INFINITY, kout[3] = {NAN, NAN, NAN}, kbest = INFINITY;
  int64_t k_in = 0, total = 0, since = 0, accepted = 0;
  double emax_last = NAN;
  int restarts = 0, status = ORA_MAX_ITER, cand_avg = 0;

  while (total < prm->max_iter) {
    double tau = eta / omega, sigma = eta * omega;
    ora_pdhg_step(n, m, row_ptr, col, u, w, X[0], T[0], P[0], Y[0], cp, gp, tau, sigma,
                  X[1], T[1], P[1], Y[1]);
    colsum(n, m, row_ptr, col, X[1], cn);
    rowsum(n, row_ptr, u, X[1], r);
    for (int i = 0; i < n; ++i) gn[i] = T[1][i] - r[i];
    ++total;
    ++since;
    int accept = 1;
    if (prm->step_mode == 1) {
      double pz = dist2(nnz, X[1], X[0]) + dist2(n, T[1], T[0]);
      double dz = dist2(m, P[1], P[0]) + dist2(n, Y[1], Y[0]);
      double inter = 0.0;
      for (int j = 0; j < m; ++j) inter += (P[1][j] - P[0][j]) * (cn[j] - c[j]);
      for (int i = 0; i < n; ++i) inter += (Y[1][i] - Y[0][i]) * (gn[i] - g[i]);
      double emax = fabs(inter) > 0.0 ? (omega * pz + dz / omega) / (2.0 * fabs(inter)) : INFINITY;
      double kk = (double)(total + 1);
      double enew = fmin((1.0 - pow(kk, -0.3)) * emax, (1.0 + pow(kk, -0.6)) * eta);
      if (enew > 3.0 * eta0) enew = 3.0 * eta0;
      if (enew < 0.01 * eta0) enew = 0.01 * eta0;
      accept = (eta <= emax) || (eta <= 0.01 * eta0);
      eta = enew;
      emax_last = emax;
    }
    if (accept) {
      memcpy(X[0], X[1], (size_t)nnz * sizeof(double));
      memcpy(T[0], T[1], (size_t)n * sizeof(double));
      memcpy(P[0], P[1], (size_t)m * sizeof(double));
      memcpy(Y[0], Y[1], (size_t)n * sizeof(double));
      memcpy(cp, c, (size_t)m * sizeof(double));
      memcpy(c, cn, (size_t)m * sizeof(double));
      memcpy(gp, g, (size_t)n * sizeof(double));
      memcpy(g, gn, (size_t)n * sizeof(double));
      ++k_in;
      ++accepted;
      /* running averages since the last restart (Alg. 1) */
      for (int64_t k = 0; k < nnz; ++k) X[2][k] += (X[0][k] - X[2][k]) / (double)k_in;
      for (int i = 0; i < n; ++i) T[2][i] += (T[0][i] - T[2][i]) / (double)k_in;
      for (int j = 0; j < m; ++j) P[2][j] += (P[0][j] - P[2][j]) / (double)k_in;
      for (int i = 0; i < n; ++i) Y[2][i] += (Y[0][i] - Y[2][i]) / (double)k_in;
    }
    int eval = (total % prm->eval_every == 0) || total == prm->max_iter;
    if (!eval) continue;
    if (k_in == 0) {
      memcpy(X[2], X[0], (size_t)nnz * sizeof(double));
      memcpy(T[2], T[0], (size_t)n * sizeof(double));
      memcpy(P[2], P[0], (size_t)m * sizeof(double));
      memcpy(Y[2], Y[0], (size_t)n * sizeof(double));
    }
    double kc[3], ka[3];
    double ec = ora_kkt_ty(n, m, row_ptr, col, u, w, X[0], T[0], P[0], Y[0], kc);
    double ea = ora_kkt_ty(n, m, row_ptr, col, u, w, X[2], T[2], P[2], Y[2], ka);
    if (!isfinite(ec) || !isfinite(ea)) {
      rc = ORA_ERR_NUMERIC;
      goto done;
    }
    cand_avg = ea < ec;
    double kcand = cand_avg ? ea : ec;
    memcpy(kout, cand_avg ? ka : kc, sizeof(kout));
    kbest = kcand;
    if (prm->verbose)
      fprintf(stderr, "[oracle-pdhg] it=%lld cur=%.3e avg=%.3e eta=%.3e omega=%.3e\n",
              (long long)total, ec, ea, eta, omega);
    if (kcand <= prm->tol) {
      status = ORA_OK;
      break;
    }
    if (total >= prm->max_iter) break;
    if (prm->restart) {
      int do_restart = (kcand <= prm->beta_sufficient * kkt0) ||
                       (kcand <= prm->beta_necessary * kkt0 && kcand > kkt_prev) ||
                       ((double)since >= prm->beta_artificial * (double)total);
      if (do_restart) {
        if (cand_avg) {
          memcpy(X[0], X[2], (size_t)nnz * sizeof(double));
          memcpy(T[0], T[2], (size_t)n * sizeof(double));
          memcpy(P[0], P[2], (size_t)m * sizeof(double));
          memcpy(Y[0], Y[2], (size_t)n * sizeof(double));
          colsum(n, m, row_ptr, col, X[0], c);
          rowsum(n, row_ptr, u, X[0], r);
          for (int i = 0; i < n; ++i) g[i] = T[0][i] - r[i];
        }
        memcpy(cp, c, (size_t)m * sizeof(double));
        memcpy(gp, g, (size_t)n * sizeof(double));
        double dx = sqrt(dist2(nnz, X[0], X[3]) + dist2(n, T[0], T[3]));
        double dp = sqrt(dist2(m, P[0], P[3]) + dist2(n, Y[0], Y[3]));
        if (dx > 1e-10 && dp > 1e-10)
          omega = exp(prm->theta * log(dp / dx) + (1.0 - prm->theta) * log(omega));
        ++restarts;
        if (prm->omega_check_every > 0 && restarts % prm->omega_check_every == 0 &&
            (omega < omega0 / prm->omega_bound || omega > omega0 * prm->omega_bound))
          omega = omega0;
        memcpy(X[3], X[0], (size_t)nnz * sizeof(double));
        memcpy(T[3], T[0], (size_t)n * sizeof(double));
        memcpy(P[3], P[0], (size_t)m * sizeof(double));
        memcpy(Y[3], Y[0], (size_t)n * sizeof(double));
        kkt0 = kcand;
        kkt_prev = INFINITY;
        k_in = 0;
        since = 0;
        cand_avg = 0;
      } else {
        kkt_prev = kcand;
      }
    }
  }
  {
    int z = (prm->output == 2 || (prm->output == 0 && cand_avg)) ? 2 : 0;
    memcpy(x, X[z], (size_t)nnz * sizeof(double));
    memcpy(p, P[z], (size_t)m * sizeof(double));
    if (t) memcpy(t, T[z], (size_t)n * sizeof(double));
    if (y) memcpy(y, Y[z], (size_t)n * sizeof(double));
    if (prm->output != 0) kbest = ora_kkt_ty(n, m, row_ptr, col, u, w, X[z], T[z], P[z], Y[z], kout);
  }
  if (info) {
    info->rel_kkt = kbest;
    info->rel_primal = kout[0];
    info->rel_dual = kout[1];
    info->rel_gap = kout[2];
    info->eta = eta;
    info->omega = omega;
    info->iters = total;
    info->restarts = restarts;
    info->status = status;
    info->accepted = accepted;
    info->emax_last = emax_last;
  }
  rc = status;
done:
  free(u);
  for (int q = 0; q < 4; ++q) { free(X[q]); free(T[q]); free(P[q]); free(Y[q]); }
  free(c); free(cp); free(cn); free(g); free(gp); free(gn); free(r); free(deg);
  if (rc < 0 && info) info->status = rc;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 as analysed in Sec. 3 (Lemma 1, Lemma 2, Theorem 1): fixed step   */
/* sizes sigma = tau = eta, fixed restart length K, every restart to the    */
/* average of the K iterates of its inner loop; no adaptive enhancement.    */
/* Row normalisation and the initial point as in ora_solve.                 */
/* eta <= 0: 1/(2 ||K||), ||K|| = sqrt(max_j deg_j).                        */
/* p_ref[m] (may be NULL): dist[n] = ||p^{n,0} - p_ref||_2, n = 0..R, and   */
/* kkt[n] (may be NULL) the relative KKT error of (x^{n,0}, p^{n,0}).        */
/* p[m], x[nnz]: the last restart point.                                     */
/* ------------------------------------------------------------------------ */
int ora_fixed_restart(int n, int m, const int64_t *row_ptr, const int32_t *col,
                      const double *u, const double *w, int K, int R, double eta,
                      const double *p_ref, double *dist, double *kkt, double *p, double *x) {
  int rc = ora_validate(n, m, row_ptr, col, u, w);
  if (rc != ORA_OK) return rc;
  if (K < 1 || R < 0) return ORA_ERR_ARG;
  int64_t nnz = row_ptr[n];
  int dmax = 0;
  for (int i = 0; i < n; ++i)
    if ((int)(row_ptr[i + 1] - row_ptr[i]) > dmax) dmax = (int)(row_ptr[i + 1] - row_ptr[i]);
  double *uh = (double *)malloc((size_t)nnz * sizeof(double));
  double *xn = (double *)malloc((size_t)nnz * sizeof(double));
  double *xb = (double *)malloc((size_t)nnz * sizeof(double));
  double *deg = (double *)calloc((size_t)m, sizeof(double));
  double *c = (double *)malloc((size_t)m * sizeof(double));
  double *cp = (double *)malloc((size_t)m * sizeof(double));
  double *pn = (double *)malloc((size_t)m * sizeof(double));
  double *pb = (double *)malloc((size_t)m * sizeof(double));
  ora_params prm;
  ora_default_params(&prm);
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
      if (u[k] > mx) mx = u[k];
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) uh[k] = u[k] / mx;
  }
  for (int64_t k = 0; k < nnz; ++k) deg[col[k]] += 1.0;
  double maxdeg = 0.0, sumw = 0.0;
  for (int j = 0; j < m; ++j)
    if (deg[j] > maxdeg) maxdeg = deg[j];
  for (int i = 0; i < n; ++i) sumw += w[i];
  if (!(eta > 0.0)) eta = 1.0 / (2.0 * sqrt(maxdeg));
  for (int i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) x[k] = 1.0 / deg[col[k]];
  for (int j = 0; j < m; ++j) p[j] = sumw / m;

  for (int r = 0; r <= R; ++r) {
    /* restart point (x^{r,0}, p^{r,0}) */
    if (p_ref && dist) dist[r] = sqrt(dist2(m, p, p_ref));
    if (kkt) kkt[r] = ora_kkt(n, m, row_ptr, col, uh, w, x, p, NULL);
    if (r == R) break;
    /* inner loop of K iterations from the restart point; after a restart
     * the extrapolation has no previous iterate: c^{-1} = c^0 */
    colsum(n, m, row_ptr, col, x, c);
    memcpy(cp, c, (size_t)m * sizeof(double));
    for (int k = 0; k < K; ++k) {
      for (int j = 0; j < m; ++j) pn[j] = p[j] + eta * (2.0 * c[j] - cp[j] - 1.0);
      rc = prox_sweep(n, row_ptr, col, uh, w, x, pn, eta, &prm, dmax, xn, NULL);
      if (rc != ORA_OK) goto done;
      memcpy(x, xn, (size_t)nnz * sizeof(double));
      memcpy(p, pn, (size_t)m * sizeof(double));
      memcpy(cp, c, (size_t)m * sizeof(double));
      colsum(n, m, row_ptr, col, x, c);
      /* running average of the iterates of this inner loop */
      if (k == 0) {
        memcpy(xb, x, (size_t)nnz * sizeof(double));
        memcpy(pb, p, (size_t)m * sizeof(double));
      } else {
        for (int64_t q = 0; q < nnz; ++q) xb[q] += (x[q] - xb[q]) / (double)(k + 1);
        for (int j = 0; j < m; ++j) pb[j] += (p[j] - pb[j]) / (double)(k + 1);
      }
    }
    /* restart to the average */
    memcpy(x, xb, (size_t)nnz * sizeof(double));
    memcpy(p, pb, (size_t)m * sizeof(double));
  }
  rc = ORA_OK;
done:
  free(uh); free(xn); free(xb); free(deg); free(c); free(cp); free(pn); free(pb);
  return rc;
}
