// C ABI of the gfx950 PDHCG library (include/pdhcg.h): validation, market
// creation (copies, row normalisation, degree binning), the host control of
// restarted PDHCG (Alg. 2 with the Sec. 5 enhancements) and the
// Arrow-Debreu fixed point (Alg. 4).  The per-iteration work runs in the
// kernels of pdhcg_kernels.hip; the host only acts every eval_every
// iterations (KKT check, restart, primal weight).
#include "../../include/pdhcg.h"
#include "pdhcg_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <numeric>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace pdhcg;

namespace pdhcg {
int long_row_threads();  // threads per workgroup of the solver's long-row kernel (pdhcg_long.hip)
}

namespace {

thread_local std::string g_err;

int32_t fail(int32_t st, const std::string &msg) {
  g_err = msg;
  return st;
}

}  // namespace

void pdhcg_internal_set_error(const char *msg) { g_err = msg ? msg : ""; }

namespace {

#define HIPC(call)                                                                  \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(PDHCG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Bin {
  int G = 0, E = 0;
  std::vector<int32_t> rows;  // empty = identity (all rows)
  int32_t *d_rows = nullptr;
  int32_t *d_rbeg = nullptr;  // per slot: first entry and end of its row
  int32_t *d_rend = nullptr;
  int32_t nrows = 0;
  int32_t nwg = 0;
  int32_t wg_offset = 0;
  int32_t rows_per_wg = 0;
  int32_t team_off = 0;  // team kernel (G = 0, E > 0): first row index in the panel offsets
  int64_t nnz = 0;
};

template <typename T>
hipError_t dalloc(T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void **)p, count * sizeof(T));
}

}  // namespace

struct pdhcg_market_s {
  int32_t n = 0, m = 0;
  int64_t nnz = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  // problem data (device)
  int32_t *row_ptr = nullptr, *col = nullptr, *deg = nullptr;
  float *uh = nullptr, *rowmax = nullptr, *w = nullptr;
  // workspace (device)
  float *X[3] = {nullptr, nullptr, nullptr};
  double *P[3] = {nullptr, nullptr, nullptr};
  double *C[3] = {nullptr, nullptr, nullptr};
  float *XA = nullptr;
  double *PA = nullptr;
  double *Pk = nullptr;  // float64 copy of caller prices (kkt, row_prox)
  float *T[2] = {nullptr, nullptr};
  double *colpart = nullptr;
  float *evalpart = nullptr;
  double *evalcs = nullptr;
  uint32_t *evalchunk = nullptr;
  double *rowpart = nullptr, *colblk = nullptr, *cacc = nullptr, *colchunk = nullptr;
  DevState *S = nullptr;   // device
  DevState *hS = nullptr;  // pinned host shadow
  // host data
  std::vector<int32_t> h_deg_col;
  int32_t maxdeg_col = 0, maxdeg_row = 0;
  double sumw = 0.0;
  std::vector<Bin> bins;
  int32_t total_wg = 0;
  int lds_row = 0, lds_eval = 0;
  size_t lds_cap = 0;  // LDS bytes a workgroup may use
  int col_blocks = 0;
  // Goods relabelled by degree (most bought first) when their LDS data does
  // not fit: perm[internal] = caller's id, inv[caller's id] = internal (both
  // device, null without relabelling); goods [0, hot) use LDS.
  int32_t hot = 0;
  int32_t *perm = nullptr, *inv = nullptr;
  uint16_t *col16 = nullptr;  // 2-byte good ids (LDS modes 1 and 3)
  int32_t *cold_ptr = nullptr, *cold_idx = nullptr;  // goods beyond LDS by column (mode 7)
  // every entry of the goods beyond LDS by column, with its row, and the
  // rows' dual values, for the KKT pass (mode 7)
  int32_t *ecold_ptr = nullptr, *ecold_idx = nullptr, *ecold_row = nullptr;
  double *yrow = nullptr;
  int32_t ecold_mean_degree = 0;
  // panel buffers of the cold entries of team-kernel rows (mode 7)
  float *pval = nullptr;
  uint16_t *pid = nullptr;
  int32_t *proff = nullptr;
  int32_t *cslot = nullptr;
  int64_t *pbeg = nullptr;
  double *ppart = nullptr;
  int32_t npanel = 0, pchunks = 0;
  float *srow = nullptr;  // [n] roots of long rows between solver passes (markets with long rows)
  int32_t cold_mean_degree = 0;  // mean degree of the goods beyond LDS
  uint32_t *gmax = nullptr;  // [2][m] KKT column maxima of the goods from hot on
  double *gsum = nullptr;    // [m] KKT column sums of the goods from hot on
  // restarted PDHG (Alg. 1): buyers' t, y, g in three roles and the anchors
  // of t and y, allocated at the first pdhcg_pdhg_solve
  double *pdhg_buf = nullptr;
  PdhgDev pdhg{};

  MarketDev dev() const {
    MarketDev d;
    d.n = n;
    d.m = m;
    d.nnz = nnz;
    d.hot = hot;
    d.pad_hot = 0;
    d.col16 = col16;
    d.cold_ptr = cold_ptr;
    d.cold_idx = cold_idx;
    d.pval = pval;
    d.pid = pid;
    d.proff = proff;
    d.cslot = cslot;
    d.npanel = npanel;
    d.pad_panel = 0;
    d.ecold_ptr = ecold_ptr;
    d.ecold_idx = ecold_idx;
    d.ecold_row = ecold_row;
    d.yrow = yrow;
    d.srow = srow;
    d.row_ptr = row_ptr;
    d.col = col;
    d.uh = uh;
    d.w = w;
    d.X0 = X[0];
    d.X1 = X[1];
    d.X2 = X[2];
    d.P0 = P[0];
    d.P1 = P[1];
    d.P2 = P[2];
    d.C0 = C[0];
    d.C1 = C[1];
    d.C2 = C[2];
    d.XA = XA;
    d.PA = PA;
    d.colpart = colpart;
    d.rowpart = rowpart;
    d.colblk = colblk;
    d.colchunk = colchunk;
    d.S = S;
    return d;
  }
  BinDev bindev(const Bin &b) const {
    BinDev d;
    d.rows = b.d_rows;
    d.rlo = b.d_rows ? b.d_rbeg : row_ptr;
    d.rhi = b.d_rows ? b.d_rend : row_ptr + 1;
    d.nrows = b.nrows;
    d.wg_offset = b.wg_offset;
    d.rows_per_wg = b.rows_per_wg;
    d.team_off = b.team_off;
    return d;
  }
};

extern "C" {

int32_t pdhcg_abi_version(void) { return PDHCG_ABI_VERSION; }

const char *pdhcg_status_string(int32_t st) {
  switch (st) {
    case PDHCG_OK: return "ok";
    case PDHCG_MAX_ITER: return "iteration limit reached";
    case PDHCG_ERR_ARG: return "invalid argument";
    case PDHCG_ERR_ASSUMPTION: return "Assumption 1 violated (buyer or good without positive utility)";
    case PDHCG_ERR_NUMERIC: return "numerical failure";
    case PDHCG_ERR_OOM: return "out of memory";
    case PDHCG_ERR_HIP: return "HIP runtime error";
    case PDHCG_ERR_UNSUPPORTED: return "unsupported shape";
    default: return "unknown status";
  }
}

const char *pdhcg_last_error(void) { return g_err.c_str(); }

void pdhcg_default_params(pdhcg_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tol = 1e-4;
  p->max_iter = 100000;
  p->eval_every = 64;
  p->search = PDHCG_SEARCH_ACTIVESET;
  p->sections = 32;
  p->max_search_rounds = 16;
  p->search_rtol = 1e-10;
  p->step_mode = PDHCG_STEP_ADAPTIVE;
  p->restart = PDHCG_RESTART_ADAPTIVE;
  p->beta_sufficient = 0.2;
  p->beta_necessary = 0.8;
  p->beta_artificial = 0.2;
  p->theta = 0.2;
  p->omega_check_every = 3;
  p->output = PDHCG_OUTPUT_CANDIDATE;
  p->omega_bound = 1e4;
  p->eta0 = 0.0;
  p->omega0 = 0.0;
  p->normalize_rows = 1;
  p->verbose = 0;
}

int32_t pdhcg_validate_host(int32_t n, int32_t m, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col, const float *u, const float *w) {
  if (n <= 0 || m <= 0 || nnz <= 0 || nnz > INT32_MAX)
    return fail(PDHCG_ERR_ARG, "sizes must satisfy n, m > 0 and 0 < nnz <= 2^31-1");
  if (!row_ptr || !col || !u || !w) return fail(PDHCG_ERR_ARG, "null pointer");
  if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz)
    return fail(PDHCG_ERR_ARG, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
  std::vector<char> good((size_t)m, 0);
  for (int32_t i = 0; i < n; ++i) {
    const int32_t b = row_ptr[i], e = row_ptr[i + 1];
    if (e < b) return fail(PDHCG_ERR_ARG, "row_ptr decreases at row " + std::to_string(i));
    if (!(w[i] > 0.0f) || !std::isfinite(w[i]))
      return fail(PDHCG_ERR_ARG, "budget w[" + std::to_string(i) + "] must be finite and > 0");
    bool liked = false;
    for (int32_t k = b; k < e; ++k) {
      const int32_t c = col[k];
      if (c < 0 || c >= m) return fail(PDHCG_ERR_ARG, "column index out of range at " + std::to_string(k));
      if (k > b && c <= col[k - 1])
        return fail(PDHCG_ERR_ARG, "columns not strictly increasing in row " + std::to_string(i));
      if (!(u[k] >= 0.0f) || !std::isfinite(u[k]))
        return fail(PDHCG_ERR_ARG, "utility u[" + std::to_string(k) + "] must be finite and >= 0");
      if (u[k] > 0.0f) {
        liked = true;
        good[(size_t)c] = 1;
      }
    }
    if (!liked)
      return fail(PDHCG_ERR_ASSUMPTION, "buyer " + std::to_string(i) + " has no positive utility");
  }
  for (int32_t j = 0; j < m; ++j)
    if (!good[(size_t)j])
      return fail(PDHCG_ERR_ASSUMPTION, "good " + std::to_string(j) + " has no positive utility");
  return PDHCG_OK;
}

void pdhcg_market_destroy(pdhcg_market mk) {
  if (!mk) return;
  auto f = [](void *p) {
    if (p) (void)hipFree(p);
  };
  f(mk->row_ptr); f(mk->col); f(mk->deg); f(mk->uh); f(mk->rowmax); f(mk->w);
  for (int q = 0; q < 3; ++q) { f(mk->X[q]); f(mk->P[q]); f(mk->C[q]); }
  f(mk->XA); f(mk->PA); f(mk->Pk); f(mk->T[0]); f(mk->T[1]);
  f(mk->colpart); f(mk->evalpart); f(mk->evalcs); f(mk->evalchunk);
  f(mk->rowpart); f(mk->colblk); f(mk->cacc); f(mk->S);
  f(mk->colchunk); f(mk->perm); f(mk->inv); f(mk->col16); f(mk->cold_ptr); f(mk->cold_idx); f(mk->srow);
  f(mk->pval); f(mk->pid); f(mk->proff); f(mk->pbeg); f(mk->ppart); f(mk->cslot); f(mk->gmax); f(mk->gsum);
  f(mk->ecold_ptr); f(mk->ecold_idx); f(mk->ecold_row); f(mk->yrow);
  f(mk->pdhg_buf);
  for (auto &b : mk->bins) {
    f(b.d_rows);
    f(b.d_rbeg);
    f(b.d_rend);
  }
  if (mk->hS) (void)hipHostFree(mk->hS);
  delete mk;
}

}  // extern "C"

namespace {

// Row kernel shape for a row of degree d: G lanes x E entries per lane
// covering d with the fewest slots, then the fewest lanes (G >= 8 keeps
// each load of a segment at least 32 contiguous bytes).
void choose_shape(int d, int *G, int *E) {
  static const int Gs[] = {8, 16, 32, 64};
  static const int Es[] = {1, 2, 4, 6, 7, 8};
  int bestG = 64, bestE = 16, best = 1 << 30;
  for (int g : Gs)
    for (int e : Es) {
      const int slots = g * e;
      // fewest slots; among those the fewest lanes per row (fewer
      // reduction steps per row; measured faster on 100-entry rows:
      // G=16,E=8 0.80 ms, 32,4 0.83 ms, 64,2 1.01 ms per pass)
      if (row_variant_exists(g, e) && slots >= d && slots < best) {
        best = slots;
        bestG = g;
        bestE = e;
      }
    }
  if (best == (1 << 30)) {  // beyond 512 entries
    bestG = 64;
    bestE = 16;
  }
  const char *eg = std::getenv("PDHCG_ROW_G");
  const char *ee = std::getenv("PDHCG_ROW_E");
  if (eg && ee) {
    const int g = std::atoi(eg), e = std::atoi(ee);
    if (row_variant_exists(g, e) && g * e >= d) {
      bestG = g;
      bestE = e;
    }
  }
  *G = bestG;
  *E = bestE;
}

int32_t build_bins(pdhcg_market mk, const std::vector<int32_t> &h_row_ptr, int wg_per_cu) {
  // group rows by kernel shape; rows above kLongRow entries take G = 0:
  // the team kernel (E = its shape code) or the one-wave-per-row kernel
  // (E = 0).  Teams hold a row in registers (one read) but need many
  // registers per thread; the one-wave-per-row kernel reads a row two or
  // three times with few registers, so more waves share a CU.  Measured:
  // teams win where the LDS already limits a CU to one workgroup
  // (relabelled markets, LDS mode 7), which is where they are used
  // (PDHCG_TEAM=1, the default); PDHCG_TEAM=0 never uses them, PDHCG_TEAM=2
  // for every row up to kTeamMaxRow entries.
  int team_mode = 1;
  if (const char *e = std::getenv("PDHCG_TEAM")) team_mode = std::atoi(e);
  // Register-resident bins of the same lane count G merge into the one with
  // the most entries per lane: a pass takes 64 / G rows per wave whatever E
  // is, and each bin's launch stages the prices, writes a partial row per
  // workgroup and drains its tail.  Measured per row pass: e-commerce-shaped
  // market (one workgroup per CU by LDS) five bins 1.18 ms, two 0.95 ms;
  // the Table 2 markets (m = 4000, two workgroups per CU by LDS) 8-19% less,
  // also where the wider shape leaves room for one workgroup only.
  // PDHCG_MERGE_BINS=0 keeps a bin per shape.
  bool merge = true;
  if (const char *e = std::getenv("PDHCG_MERGE_BINS")) merge = std::atoi(e) != 0;
  int emax[65] = {0};
  if (merge)
    for (int32_t i = 0; i < mk->n; ++i) {
      const int d = h_row_ptr[(size_t)i + 1] - h_row_ptr[(size_t)i];
      if (d > kLongRow) continue;
      int G = 0, E = 0;
      choose_shape(d, &G, &E);
      emax[G] = std::max(emax[G], E);
    }
  std::vector<std::pair<int, int>> shapes;
  std::vector<int> shape_of((size_t)mk->n);
  for (int32_t i = 0; i < mk->n; ++i) {
    const int d = h_row_ptr[(size_t)i + 1] - h_row_ptr[(size_t)i];
    int G = 0, E = 0;
    if (d <= kLongRow) {
      choose_shape(d, &G, &E);
      if (merge) E = emax[G];
    } else if (team_mode == 2 || (team_mode == 1 && mk->lds_row == 7)) {
      E = team_code(d);
    }
    auto key = std::make_pair(G, E);
    auto it = std::find(shapes.begin(), shapes.end(), key);
    int s;
    if (it == shapes.end()) {
      shapes.push_back(key);
      s = (int)shapes.size() - 1;
    } else {
      s = (int)(it - shapes.begin());
    }
    shape_of[(size_t)i] = s;
  }
  mk->bins.assign(shapes.size(), Bin());
  for (size_t s = 0; s < shapes.size(); ++s) {
    mk->bins[s].G = shapes[s].first;
    mk->bins[s].E = shapes[s].second;
  }
  for (int32_t i = 0; i < mk->n; ++i) {
    Bin &b = mk->bins[(size_t)shape_of[(size_t)i]];
    b.rows.push_back(i);
    b.nnz += h_row_ptr[(size_t)i + 1] - h_row_ptr[(size_t)i];
  }
  // workgroup budget: the resident workgroups per CU (at most two), so that
  // each bin's launch fills the chip in one round.  The bins are launched one
  // after the other, so every bin gets the whole budget; each workgroup
  // writes one partial row, reduced by the column kernels.
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, mk->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const int budget = std::max(1, std::min(2, wg_per_cu)) * cus;
  int off = 0;
  const int kWaves = kRowBlock / kWave;
  for (auto &b : mk->bins) {
    b.nrows = (int32_t)b.rows.size();
    // rows per workgroup pass: the segments of its waves, a wave per row for
    // the long-row kernel (whose solver pass runs more waves per workgroup)
    const int per_pass = b.G ? kWaves * (kWave / b.G) : (b.E == 0 ? long_row_threads() / kWave : kWaves);
    const int64_t passes = (b.nrows + per_pass - 1) / per_pass;
    int nwg = (int)std::max<int64_t>(1, std::min<int64_t>(passes, budget));
    const int64_t passes_per_wg = (passes + nwg - 1) / nwg;
    b.rows_per_wg = (int32_t)(passes_per_wg * per_pass);
    b.nwg = (int32_t)((b.nrows + b.rows_per_wg - 1) / b.rows_per_wg);
    b.wg_offset = off;
    off += b.nwg;
    if (mk->bins.size() == 1) {
      b.rows.clear();  // identity
      b.d_rows = nullptr;
    } else {
      std::vector<int32_t> rbeg(b.rows.size()), rend(b.rows.size());
      for (size_t q = 0; q < b.rows.size(); ++q) {
        rbeg[q] = h_row_ptr[(size_t)b.rows[q]];
        rend[q] = h_row_ptr[(size_t)b.rows[q] + 1];
      }
      HIPC(dalloc(&b.d_rows, b.rows.size()));
      HIPC(dalloc(&b.d_rbeg, b.rows.size()));
      HIPC(dalloc(&b.d_rend, b.rows.size()));
      HIPC(hipMemcpy(b.d_rows, b.rows.data(), b.rows.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
      HIPC(hipMemcpy(b.d_rbeg, rbeg.data(), rbeg.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
      HIPC(hipMemcpy(b.d_rend, rend.data(), rend.size() * sizeof(int32_t),
                     hipMemcpyHostToDevice));
    }
  }
  mk->total_wg = off;
  int32_t toff = 0;
  for (auto &b : mk->bins)
    if (b.G == 0 && b.E > 0) {
      b.team_off = toff;
      toff += b.nrows;
    }
  return PDHCG_OK;
}

}  // namespace

extern "C" int32_t pdhcg_market_create(int32_t n, int32_t m, int64_t nnz, const int32_t *row_ptr,
                                       const int32_t *col, const float *u, const float *w,
                                       void *stream, pdhcg_market *out) {
  if (!out) return fail(PDHCG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (n <= 0 || m <= 0 || nnz <= 0 || nnz > INT32_MAX)
    return fail(PDHCG_ERR_ARG, "sizes must satisfy n, m > 0 and 0 < nnz <= 2^31-1");
  if (!row_ptr || !col || !u || !w) return fail(PDHCG_ERR_ARG, "null pointer");
  if (nnz > kMaxBufferEntries)
    return fail(PDHCG_ERR_UNSUPPORTED, "markets with more than 2^29 stored entries are not "
                                       "supported (32-bit buffer offsets)");
  hipStream_t st = (hipStream_t)stream;
  // validate on the host
  std::vector<int32_t> h_rp((size_t)n + 1), h_col((size_t)nnz);
  std::vector<float> h_u((size_t)nnz), h_w((size_t)n);
  HIPC(hipMemcpyAsync(h_rp.data(), row_ptr, h_rp.size() * 4, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(h_col.data(), col, h_col.size() * 4, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(h_u.data(), u, h_u.size() * 4, hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(h_w.data(), w, h_w.size() * 4, hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  int32_t rc = pdhcg_validate_host(n, m, nnz, h_rp.data(), h_col.data(), h_u.data(), h_w.data());
  if (rc != PDHCG_OK) return rc;

  pdhcg_market mk = new (std::nothrow) pdhcg_market_s();
  if (!mk) return fail(PDHCG_ERR_OOM, "host allocation failed");
  mk->n = n;
  mk->m = m;
  mk->nnz = nnz;
  mk->stream = st;
  (void)hipGetDevice(&mk->device);
  auto cleanup = [&](int32_t code) {
    pdhcg_market_destroy(mk);
    return code;
  };
  mk->h_deg_col.assign((size_t)m, 0);
  for (int64_t k = 0; k < nnz; ++k) mk->h_deg_col[(size_t)h_col[(size_t)k]] += 1;
  mk->maxdeg_col = *std::max_element(mk->h_deg_col.begin(), mk->h_deg_col.end());
  for (int32_t i = 0; i < n; ++i)
    mk->maxdeg_row = std::max(mk->maxdeg_row, h_rp[(size_t)i + 1] - h_rp[(size_t)i]);
  mk->sumw = 0.0;
  for (int32_t i = 0; i < n; ++i) mk->sumw += (double)h_w[(size_t)i];

#define MK_HIPC(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      int32_t code_ = (e_ == hipErrorOutOfMemory) ? PDHCG_ERR_OOM : PDHCG_ERR_HIP;    \
      fail(code_, std::string(#call) + ": " + hipGetErrorString(e_));                 \
      return cleanup(code_);                                                          \
    }                                                                                 \
  } while (0)

  size_t lds_cap = 64 * 1024, lds_cu = 64 * 1024;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, mk->device) == hipSuccess && prop.sharedMemPerBlock > 0) {
      lds_cap = prop.sharedMemPerBlock;
      lds_cu = std::max(lds_cap, (size_t)prop.maxSharedMemoryPerMultiProcessor);
    }
  }
  mk->lds_cap = lds_cap;
  const size_t static_lds = 1024;  // the kernels' own __shared__ arrays
  // Row pass: float64 column partials and a float64 copy of the prices in
  // LDS when both fit.  Float64 LDS atomics: float32 LDS atomic adds measured
  // about 8x slower than float64 ones on gfx950 (198 vs 25 cycles per wave
  // instruction per CU, random slots of a 1e4-entry array), and they were
  // the limit of the pass.  Price gathers from global memory miss the vector
  // L1 on most lanes and hold its miss slots, which starves the stream of
  // row data (1e8-edge market: 0.90 ms per pass with global gathers, 0.80
  // ms with prices in LDS).  PDHCG_P_LDS=0 keeps the prices in global memory.
  //
  // When 16 bytes per good do not fit, the goods are relabelled by degree
  // (most bought first) and only the first `hot` of them keep their prices
  // and partials in LDS (LDS mode 7); the others are gathered from global
  // memory (the price vector stays in L2) and summed with device atomics.
  // On popularity-skewed markets the hot goods carry most of the entries.
  // PDHCG_HOT=k forces the relabelled mode with k LDS goods.
  const size_t per_good = 2 * sizeof(double);
  mk->lds_row = 0;
  mk->hot = m;
  if ((size_t)m * sizeof(double) + static_lds <= lds_cap) mk->lds_row = 1;
  if ((size_t)m * per_good + static_lds <= lds_cap) mk->lds_row = 3;
  int force_hot = -1;
  if (const char *e = std::getenv("PDHCG_HOT")) force_hot = std::max(0, std::atoi(e));
  if ((mk->lds_row != 3 || force_hot >= 0) && m > 1) {
    const int fit = (int)(((lds_cap - static_lds) / per_good - 1) / 64 * 64);
    mk->hot = std::min(m - 1, force_hot >= 0 ? std::min(force_hot, fit) : fit);
    mk->hot = std::max(mk->hot, 1);
    mk->lds_row = 7;
  }
  if (const char *e = std::getenv("PDHCG_P_LDS")) {
    if (!std::atoi(e) && mk->lds_row == 3) mk->lds_row = 1;
  }
  mk->lds_eval = ((size_t)mk->hot * (sizeof(double) + 2 * sizeof(uint32_t)) + static_lds <=
                  lds_cap) ? 1 : 0;
  if (const char *e = std::getenv("PDHCG_NO_LDS")) {
    if (std::atoi(e)) {
      mk->lds_row = 0;
      mk->lds_eval = 0;
      mk->hot = m;
    }
  }
  std::vector<int32_t> h_perm, h_inv;
  if (mk->lds_row == 7) {
    h_perm.resize((size_t)m);
    std::iota(h_perm.begin(), h_perm.end(), 0);
    std::stable_sort(h_perm.begin(), h_perm.end(), [&](int32_t a, int32_t b) {
      return mk->h_deg_col[(size_t)a] > mk->h_deg_col[(size_t)b];
    });
    h_inv.resize((size_t)m);
    for (int32_t j = 0; j < m; ++j) h_inv[(size_t)h_perm[(size_t)j]] = j;
    for (int64_t k = 0; k < nnz; ++k) h_col[(size_t)k] = h_inv[(size_t)h_col[(size_t)k]];
    std::vector<int32_t> deg((size_t)m);
    for (int32_t j = 0; j < m; ++j) deg[(size_t)j] = mk->h_deg_col[(size_t)h_perm[(size_t)j]];
    mk->h_deg_col.swap(deg);
  }
  mk->col_blocks = (m + kColBlock - 1) / kColBlock;
  {
    const size_t lh = (mk->lds_row == 7) ? (size_t)mk->hot + 1 : (size_t)m;
    const size_t row_lds = lh * (((mk->lds_row & 2) ? sizeof(double) : 0) +
                                 ((mk->lds_row & 1) ? sizeof(double) : 0)) + static_lds;
    rc = build_bins(mk, h_rp, (int)(lds_cu / row_lds));
    if (rc != PDHCG_OK) return cleanup(rc);
  }

  MK_HIPC(dalloc(&mk->row_ptr, (size_t)n + 1));
  MK_HIPC(dalloc(&mk->col, (size_t)nnz));
  MK_HIPC(dalloc(&mk->deg, (size_t)m));
  MK_HIPC(dalloc(&mk->uh, (size_t)nnz));
  MK_HIPC(dalloc(&mk->rowmax, (size_t)n));
  MK_HIPC(dalloc(&mk->w, (size_t)n));
  for (int q = 0; q < 3; ++q) {
    MK_HIPC(dalloc(&mk->X[q], (size_t)nnz));
    MK_HIPC(dalloc(&mk->P[q], (size_t)m));
    MK_HIPC(dalloc(&mk->C[q], (size_t)m));
  }
  MK_HIPC(dalloc(&mk->XA, (size_t)nnz));
  MK_HIPC(dalloc(&mk->PA, (size_t)m));
  MK_HIPC(dalloc(&mk->Pk, (size_t)m));
  MK_HIPC(dalloc(&mk->T[0], (size_t)n));
  MK_HIPC(dalloc(&mk->T[1], (size_t)n));
  const size_t hot = (size_t)std::max(mk->hot, 1);
  MK_HIPC(dalloc(&mk->colpart, (mk->lds_row & 1) ? (size_t)mk->total_wg * hot : 1));
  MK_HIPC(dalloc(&mk->evalpart, mk->lds_eval ? (size_t)2 * mk->total_wg * hot : (size_t)2 * m));
  MK_HIPC(dalloc(&mk->evalcs, mk->lds_eval ? (size_t)mk->total_wg * hot : (size_t)1));
  MK_HIPC(dalloc(&mk->gmax, mk->lds_eval ? (size_t)2 * m : (size_t)1));
  MK_HIPC(dalloc(&mk->gsum, mk->lds_eval ? (size_t)m : (size_t)1));
  if (!h_perm.empty()) {
    MK_HIPC(dalloc(&mk->perm, (size_t)m));
    MK_HIPC(dalloc(&mk->inv, (size_t)m));
  }
  // Goods beyond LDS (mode 7): their entries go to panel buffers (panels of
  // kPanelW goods, laid out panel by panel) or are gathered column by column
  // (in row order) by k_cold_sums.  Inside panel p the runs of the
  // team-kernel rows come first (row by row; each team fills its row's run
  // through LDS counters), then the entries of the other rows at fixed
  // slots (cslot, row by row) with their fixed in-panel good index.  The
  // other rows use fixed slots when at least kSlotShare of their entries
  // are of such goods (the slot of every entry is read, so a small share is
  // cheaper to gather); with more than kMaxPanels panels every entry of
  // these goods is gathered.  PDHCG_SLOT_SHARE overrides the share.
  constexpr double kSlotShare = 0.1;
  std::vector<int32_t> h_cold_ptr, h_cold_idx, h_proff, h_cslot;
  std::vector<int64_t> h_pbeg;
  std::vector<uint16_t> h_pid;
  int64_t panel_entries = 0;
  if (mk->lds_row == 7) {
    const int32_t hot = mk->hot, ncold = m - hot;
    const int np = (ncold + kPanelW - 1) / kPanelW;
    std::vector<char> in_team((size_t)n, 0);
    std::vector<int32_t> team_rows;
    if (np <= kMaxPanels)
      for (const Bin &b : mk->bins)
        if (b.G == 0 && b.E > 0)
          for (int32_t q = 0; q < b.nrows; ++q) {
            const int32_t i = b.rows.empty() ? q : b.rows[(size_t)q];
            team_rows.push_back(i);
            in_team[(size_t)i] = 1;
          }
    int64_t other = 0, other_cold = 0;
    for (int32_t i = 0; i < n; ++i) {
      if (in_team[(size_t)i]) continue;
      for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k) {
        other += 1;
        other_cold += h_col[(size_t)k] >= hot ? 1 : 0;
      }
    }
    double share = kSlotShare;
    if (const char *e = std::getenv("PDHCG_SLOT_SHARE")) share = std::atof(e);
    const bool fixed = np <= kMaxPanels && other_cold > 0 &&
                       (double)other_cold >= share * (double)other;
    if (!team_rows.empty() || fixed) {
      mk->npanel = np;
      auto panel_of = [&](int32_t c) { return (size_t)((c - hot) >> kPanelShift); };
      std::vector<int64_t> tot_team((size_t)np, 0), tot_fixed((size_t)np, 0);
      h_proff.assign(team_rows.size() * (size_t)np, 0);
      for (size_t r = 0; r < team_rows.size(); ++r) {
        const int32_t i = team_rows[r];
        for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k)
          if (h_col[(size_t)k] >= hot) h_proff[r * (size_t)np + panel_of(h_col[(size_t)k])] += 1;
      }
      for (size_t r = 0; r < team_rows.size(); ++r)
        for (int p = 0; p < np; ++p) tot_team[(size_t)p] += h_proff[r * (size_t)np + (size_t)p];
      if (fixed)
        for (int32_t i = 0; i < n; ++i) {
          if (in_team[(size_t)i]) continue;
          for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k)
            if (h_col[(size_t)k] >= hot) tot_fixed[panel_of(h_col[(size_t)k])] += 1;
        }
      h_pbeg.assign((size_t)np + 1, 0);
      for (int p = 0; p < np; ++p)
        h_pbeg[(size_t)p + 1] = h_pbeg[(size_t)p] + tot_team[(size_t)p] + tot_fixed[(size_t)p];
      panel_entries = h_pbeg[(size_t)np];
      // team runs
      std::vector<int64_t> run(h_pbeg.begin(), h_pbeg.end() - 1);
      for (size_t r = 0; r < team_rows.size(); ++r)
        for (int p = 0; p < np; ++p) {
          const int32_t c = h_proff[r * (size_t)np + (size_t)p];
          h_proff[r * (size_t)np + (size_t)p] = (int32_t)run[(size_t)p];
          run[(size_t)p] += c;
        }
      // fixed slots of the other rows
      h_pid.assign((size_t)std::max<int64_t>(panel_entries, 1), 0);
      if (fixed) {
        h_cslot.assign((size_t)nnz, -1);
        for (int32_t i = 0; i < n; ++i) {
          if (in_team[(size_t)i]) continue;
          for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k) {
            const int32_t c = h_col[(size_t)k];
            if (c < hot) continue;
            const int64_t sl = run[panel_of(c)]++;
            h_cslot[(size_t)k] = (int32_t)sl;
            h_pid[(size_t)sl] = (uint16_t)((c - hot) & (kPanelW - 1));
          }
        }
      }
      int cus = 256;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, mk->device) == hipSuccess && prop.multiProcessorCount > 0)
        cus = prop.multiProcessorCount;
      // chunks per panel for k_panel_part: about two blocks per CU, but no
      // block below 32768 entries (the partial sums are 64 KiB per block)
      int64_t most = 1;
      for (int p = 0; p < np; ++p) most = std::max(most, h_pbeg[(size_t)p + 1] - h_pbeg[(size_t)p]);
      mk->pchunks = (int)std::max<int64_t>(
          1, std::min<int64_t>({64, 2 * cus / np, (most + 32767) / 32768}));
      MK_HIPC(dalloc(&mk->pval, (size_t)std::max<int64_t>(panel_entries, 1)));
      MK_HIPC(dalloc(&mk->pid, h_pid.size()));
      MK_HIPC(dalloc(&mk->proff, std::max<size_t>(h_proff.size(), 1)));
      MK_HIPC(dalloc(&mk->pbeg, h_pbeg.size()));
      if (fixed) MK_HIPC(dalloc(&mk->cslot, (size_t)nnz));
      MK_HIPC(dalloc(&mk->ppart, (size_t)np * mk->pchunks * kPanelW));
    }
    if (!fixed && other_cold > 0) {
      // the other rows' entries of these goods, gathered by column
      h_cold_ptr.assign((size_t)ncold + 1, 0);
      for (int32_t i = 0; i < n; ++i) {
        if (in_team[(size_t)i]) continue;
        for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k)
          if (h_col[(size_t)k] >= hot) h_cold_ptr[(size_t)(h_col[(size_t)k] - hot) + 1] += 1;
      }
      for (int32_t g = 0; g < ncold; ++g) h_cold_ptr[(size_t)g + 1] += h_cold_ptr[(size_t)g];
      h_cold_idx.resize((size_t)h_cold_ptr[(size_t)ncold]);
      std::vector<int32_t> fill(h_cold_ptr.begin(), h_cold_ptr.end() - 1);
      for (int32_t i = 0; i < n; ++i) {
        if (in_team[(size_t)i]) continue;
        for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k)
          if (h_col[(size_t)k] >= hot) h_cold_idx[(size_t)fill[(size_t)(h_col[(size_t)k] - hot)]++] = k;
      }
      mk->cold_mean_degree = (int32_t)(h_cold_idx.size() / (size_t)std::max(ncold, 1));
      MK_HIPC(dalloc(&mk->cold_ptr, h_cold_ptr.size()));
      MK_HIPC(dalloc(&mk->cold_idx, std::max<size_t>(h_cold_idx.size(), 1)));
    }
  }
  // KKT pass of the goods beyond LDS (mode 7): their entries column by
  // column (in row order) with their rows, so that one segment of lanes per
  // good takes its maxima and sums (device atomics on these goods, three per
  // entry, ran at about 22 G/s)
  std::vector<int32_t> h_ecold_ptr, h_ecold_idx, h_ecold_row;
  if (mk->lds_row == 7 && mk->lds_eval && mk->hot < m) {
    const int32_t hot = mk->hot, ncold = m - hot;
    h_ecold_ptr.assign((size_t)ncold + 1, 0);
    for (int64_t k = 0; k < nnz; ++k)
      if (h_col[(size_t)k] >= hot) h_ecold_ptr[(size_t)(h_col[(size_t)k] - hot) + 1] += 1;
    for (int32_t g = 0; g < ncold; ++g) h_ecold_ptr[(size_t)g + 1] += h_ecold_ptr[(size_t)g];
    const size_t tot = (size_t)h_ecold_ptr[(size_t)ncold];
    h_ecold_idx.resize(std::max<size_t>(tot, 1), 0);
    h_ecold_row.resize(std::max<size_t>(tot, 1), 0);
    std::vector<int32_t> fill(h_ecold_ptr.begin(), h_ecold_ptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = h_rp[(size_t)i]; k < h_rp[(size_t)i + 1]; ++k) {
        const int32_t c = h_col[(size_t)k];
        if (c < hot) continue;
        const int32_t sl = fill[(size_t)(c - hot)]++;
        h_ecold_idx[(size_t)sl] = k;
        h_ecold_row[(size_t)sl] = i;
      }
    mk->ecold_mean_degree = (int32_t)(tot / (size_t)std::max(ncold, 1));
    MK_HIPC(dalloc(&mk->ecold_ptr, h_ecold_ptr.size()));
    MK_HIPC(dalloc(&mk->ecold_idx, h_ecold_idx.size()));
    MK_HIPC(dalloc(&mk->ecold_row, h_ecold_row.size()));
    MK_HIPC(dalloc(&mk->yrow, (size_t)2 * n));
  }
  // roots of long rows between solver passes (start of each search)
  if (std::any_of(mk->bins.begin(), mk->bins.end(), [](const Bin &b) { return b.G == 0; }))
    MK_HIPC(dalloc(&mk->srow, (size_t)n));
  std::vector<uint16_t> h_col16;
  if (mk->lds_row == 1 || mk->lds_row == 3) {
    if (m > 65536) return cleanup(fail(PDHCG_ERR_ARG, "internal: 16-bit good ids need m <= 65536"));
    h_col16.resize((size_t)nnz);
    for (int64_t k = 0; k < nnz; ++k) h_col16[(size_t)k] = (uint16_t)h_col[(size_t)k];
    MK_HIPC(dalloc(&mk->col16, (size_t)nnz));
  }
  MK_HIPC(dalloc(&mk->evalchunk, mk->lds_eval ? (size_t)2 * kColChunks * m : (size_t)1));
  MK_HIPC(dalloc(&mk->cacc, (size_t)kColChunks * m));  // chunk sums in LDS mode
  MK_HIPC(dalloc(&mk->rowpart, (size_t)mk->total_wg *
                                   std::max(std::max(kRowStats, kEvalRowStats), kPdhgEvalStats)));
  MK_HIPC(dalloc(&mk->colblk, (size_t)mk->col_blocks * std::max(kColStats, kEvalColStats)));
  MK_HIPC(dalloc(&mk->colchunk, (size_t)kColChunks * m));
  MK_HIPC(dalloc(&mk->S, 1));
  MK_HIPC(hipHostMalloc((void **)&mk->hS, sizeof(DevState), hipHostMallocDefault));
  std::memset(mk->hS, 0, sizeof(DevState));

  MK_HIPC(hipMemcpyAsync(mk->row_ptr, row_ptr, ((size_t)n + 1) * 4, hipMemcpyDeviceToDevice, st));
  if (mk->npanel > 0) {
    if (!h_proff.empty())
      MK_HIPC(hipMemcpyAsync(mk->proff, h_proff.data(), h_proff.size() * 4, hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->pbeg, h_pbeg.data(), h_pbeg.size() * 8, hipMemcpyHostToDevice, st));
    if (!h_cslot.empty())
      MK_HIPC(hipMemcpyAsync(mk->cslot, h_cslot.data(), h_cslot.size() * 4, hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->pid, h_pid.data(), h_pid.size() * 2, hipMemcpyHostToDevice, st));
  }
  if (!h_cold_ptr.empty()) {
    MK_HIPC(hipMemcpyAsync(mk->cold_ptr, h_cold_ptr.data(), h_cold_ptr.size() * 4,
                           hipMemcpyHostToDevice, st));
    if (!h_cold_idx.empty())
      MK_HIPC(hipMemcpyAsync(mk->cold_idx, h_cold_idx.data(), h_cold_idx.size() * 4,
                             hipMemcpyHostToDevice, st));
  }
  if (!h_ecold_ptr.empty()) {
    MK_HIPC(hipMemcpyAsync(mk->ecold_ptr, h_ecold_ptr.data(), h_ecold_ptr.size() * 4,
                           hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->ecold_idx, h_ecold_idx.data(), h_ecold_idx.size() * 4,
                           hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->ecold_row, h_ecold_row.data(), h_ecold_row.size() * 4,
                           hipMemcpyHostToDevice, st));
  }
  if (!h_col16.empty())
    MK_HIPC(hipMemcpyAsync(mk->col16, h_col16.data(), (size_t)nnz * 2, hipMemcpyHostToDevice, st));
  if (h_perm.empty()) {
    MK_HIPC(hipMemcpyAsync(mk->col, col, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
  } else {
    MK_HIPC(hipMemcpyAsync(mk->col, h_col.data(), (size_t)nnz * 4, hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->perm, h_perm.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
    MK_HIPC(hipMemcpyAsync(mk->inv, h_inv.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
  }
  MK_HIPC(hipMemcpyAsync(mk->w, w, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  MK_HIPC(hipMemcpyAsync(mk->deg, mk->h_deg_col.data(), (size_t)m * 4, hipMemcpyHostToDevice, st));
  MK_HIPC(launch_normalize(mk->row_ptr, u, mk->uh, mk->rowmax, n, st));
  MK_HIPC(hipMemsetAsync(mk->S, 0, sizeof(DevState), st));
  MK_HIPC(hipStreamSynchronize(st));
  *out = mk;
  return PDHCG_OK;
#undef MK_HIPC
}

extern "C" int32_t pdhcg_set_budgets(pdhcg_market mk, const float *w) {
  if (!mk || !w) return fail(PDHCG_ERR_ARG, "null argument");
  std::vector<float> h((size_t)mk->n);
  HIPC(hipMemcpyAsync(h.data(), w, h.size() * 4, hipMemcpyDeviceToHost, mk->stream));
  HIPC(hipStreamSynchronize(mk->stream));
  double s = 0.0;
  for (int32_t i = 0; i < mk->n; ++i) {
    if (!(h[(size_t)i] > 0.0f) || !std::isfinite(h[(size_t)i]))
      return fail(PDHCG_ERR_ARG, "budget w[" + std::to_string(i) + "] must be finite and > 0");
    s += (double)h[(size_t)i];
  }
  mk->sumw = s;
  HIPC(hipMemcpyAsync(mk->w, w, (size_t)mk->n * 4, hipMemcpyDeviceToDevice, mk->stream));
  HIPC(hipStreamSynchronize(mk->stream));
  return PDHCG_OK;
}

extern "C" int32_t pdhcg_market_lds_goods(pdhcg_market mk) {
  if (!mk) return fail(PDHCG_ERR_ARG, "null market");
  return (mk->lds_row & 1) ? mk->hot : 0;
}

extern "C" int32_t pdhcg_market_bins(pdhcg_market mk, int32_t cap, int32_t *lanes,
                                     int32_t *entries, int32_t *rows) {
  if (!mk) return fail(PDHCG_ERR_ARG, "null market");
  const int32_t nb = (int32_t)mk->bins.size();
  for (int32_t b = 0; b < nb && b < cap; ++b) {
    if (lanes) lanes[b] = mk->bins[(size_t)b].G;
    if (entries) entries[b] = mk->bins[(size_t)b].E;
    if (rows) rows[b] = mk->bins[(size_t)b].nrows;
  }
  return nb;
}

namespace {

int32_t check_params(const pdhcg_params *p) {
  if (!p) return fail(PDHCG_ERR_ARG, "params is NULL");
  if (!(p->tol >= 0.0) || p->max_iter < 0 || p->eval_every <= 0)
    return fail(PDHCG_ERR_ARG, "tol >= 0, max_iter >= 0 and eval_every > 0 required");
  if (p->search != PDHCG_SEARCH_ACTIVESET && p->search != PDHCG_SEARCH_KSECTION &&
      p->search != PDHCG_SEARCH_KSECTION_WAVE)
    return fail(PDHCG_ERR_ARG, "unknown search");
  if (p->search == PDHCG_SEARCH_KSECTION && (p->sections < 1 || p->sections > kMaxSections))
    return fail(PDHCG_ERR_ARG, "sections must be in [1, 32]");
  if (p->search == PDHCG_SEARCH_KSECTION_WAVE &&
      (p->sections < 1 || p->sections > kMaxWaveSections))
    return fail(PDHCG_ERR_ARG, "sections must be in [1, 64]");
  if (p->max_search_rounds < 1) return fail(PDHCG_ERR_ARG, "max_search_rounds must be >= 1");
  if (p->step_mode != PDHCG_STEP_FIXED && p->step_mode != PDHCG_STEP_ADAPTIVE)
    return fail(PDHCG_ERR_ARG, "unknown step_mode");
  if (p->output < 0 || p->output > 2) return fail(PDHCG_ERR_ARG, "unknown output");
  if (!p->normalize_rows)
    return fail(PDHCG_ERR_UNSUPPORTED, "normalize_rows = 0 is not supported");
  return PDHCG_OK;
}

// The k-section searches are built for rows of at most 512 entries; the
// one-lane-per-candidate kernel also keeps every good's column partial in
// LDS beside its row staging.
int32_t check_search(pdhcg_market mk, const pdhcg_params *p) {
  if (p->search == PDHCG_SEARCH_KSECTION)
    for (const Bin &b : mk->bins)
      if (b.G == 0)
        return fail(PDHCG_ERR_UNSUPPORTED, "the k-section search is not built for rows of more "
                                           "than 512 entries");
  if (p->search == PDHCG_SEARCH_KSECTION_WAVE) {
    if (mk->maxdeg_row > kKwaveMaxRow)
      return fail(PDHCG_ERR_UNSUPPORTED, "the one-lane-per-candidate k-section search is not "
                                         "built for rows of more than 512 entries");
    if (!(mk->lds_row & 1) || mk->hot != mk->m || kwave_lds_bytes(mk->m) + 1024 > mk->lds_cap)
      return fail(PDHCG_ERR_UNSUPPORTED, "the one-lane-per-candidate k-section search needs every "
                                         "good's column partial in LDS beside the row staging "
                                         "(m <= 14000 on gfx950)");
  }
  return PDHCG_OK;
}

RowIO row_io_state(const pdhcg_params *p) {
  RowIO io;
  std::memset(&io, 0, sizeof(io));
  io.use_state = 1;
  io.colsum = 1;
  io.search = p->search;
  io.sections = p->sections;
  io.max_rounds = p->max_search_rounds;
  io.rtol = p->search_rtol;
  return io;
}

// One trial step: price step, row pass over every bin, column kernel.
// ev0/ev1 (optional) bracket the row-pass launches.
// Column sums of the goods beyond LDS (mode 7) of the allocation x (or of
// the trial allocation when use_state) into out: the panel sums, or the
// gathers by column when the goods do not fit the panels.
// With sum_panels = 0 the panel partials are left for k_col_decide to sum.
int32_t enqueue_cold_sums(pdhcg_market mk, const MarketDev &md, int use_state, const float *x,
                          double *out, hipStream_t st, int sum_panels = 1) {
  HIPC(launch_cold_sums(md, use_state, x, out, mk->cold_mean_degree, st));
  HIPC(launch_panel_sums(md, use_state, out, mk->pval, mk->pid, mk->pbeg, mk->ppart, mk->pchunks,
                         mk->cold_ptr != nullptr, sum_panels, st));
  return PDHCG_OK;
}

int32_t enqueue_step(pdhcg_market mk, const RowIO &io, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr) {
  const MarketDev md = mk->dev();
  // c_try is zeroed when its goods are summed by device atomics (no LDS)
  HIPC(launch_pstep(md, mk->lds_row == 0 ? 1 : 0, mk->stream));
  if (ev0) HIPC(hipEventRecord(ev0, mk->stream));
  if (io.search == PDHCG_SEARCH_KSECTION_WAVE)
    HIPC(launch_row_kwave(md, io, mk->total_wg, mk->stream));
  else
    for (const Bin &b : mk->bins)
      HIPC(launch_row_pass(md, mk->bindev(b), b.G, b.E, mk->lds_row, io, b.nwg, mk->stream));
  // the panel partials (goods beyond LDS) are summed by k_col_decide
  const bool panels = mk->lds_row == 7 && md.npanel > 0 && mk->hot < mk->m;
  if (mk->lds_row == 7) {
    const int32_t rc = enqueue_cold_sums(mk, md, 1, nullptr, nullptr, mk->stream, panels ? 0 : 1);
    if (rc != PDHCG_OK) return rc;
  }
  if (ev1) HIPC(hipEventRecord(ev1, mk->stream));
  HIPC(launch_col_decide(md, mk->total_wg, mk->lds_row & 1, panels ? mk->ppart : nullptr,
                         mk->pchunks, mk->cold_ptr != nullptr, mk->stream));
  return PDHCG_OK;
}

// Per-solve HIP events for timing the row passes.
struct EventPool {
  std::vector<hipEvent_t> ev;
  ~EventPool() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// KKT pass over (xc, pc) and optionally the averaged point.
int32_t enqueue_eval(pdhcg_market mk, EvalIO io) {
  const MarketDev md = mk->dev();
  io.evalpart = mk->evalpart;
  io.cacc = mk->cacc;
  if (!mk->lds_eval) {
    HIPC(hipMemsetAsync(mk->evalpart, 0, (size_t)2 * mk->m * sizeof(float), mk->stream));
    HIPC(hipMemsetAsync(mk->cacc, 0, (size_t)mk->m * sizeof(double), mk->stream));
  }
  io.evalcs = mk->evalcs;
  io.evalchunk = mk->evalchunk;
  io.gmax = mk->gmax;
  io.gsum = mk->gsum;
  if (mk->lds_eval && mk->hot < mk->m) {
    HIPC(launch_zero_f32(reinterpret_cast<float *>(mk->gmax), (int64_t)2 * mk->m, mk->stream));
    HIPC(launch_zero_f64(mk->gsum, mk->m, mk->stream));
  }
  for (const Bin &b : mk->bins)
    HIPC(launch_eval_row(md, mk->bindev(b), b.G, b.E, mk->lds_eval, io, b.nwg, mk->total_wg,
                         mk->stream));
  if (mk->lds_eval) HIPC(launch_eval_cold(md, io, mk->ecold_mean_degree, mk->stream));
  if (mk->lds_eval) HIPC(launch_eval_chunks(md, io, mk->total_wg, mk->stream));
  HIPC(launch_eval_col(md, io, mk->total_wg, mk->lds_eval, mk->stream));
  return PDHCG_OK;
}

int32_t pull_state(pdhcg_market mk) {
  HIPC(hipMemcpyAsync(mk->hS, mk->S, sizeof(DevState), hipMemcpyDeviceToHost, mk->stream));
  HIPC(hipStreamSynchronize(mk->stream));
  return PDHCG_OK;
}

int32_t push_state(pdhcg_market mk) {
  HIPC(hipMemcpyAsync(mk->S, mk->hS, sizeof(DevState), hipMemcpyHostToDevice, mk->stream));
  return PDHCG_OK;
}

double kkt_max(const double *k) { return std::max(k[0], std::max(k[1], k[2])); }

}  // namespace

extern "C" int32_t pdhcg_kkt(pdhcg_market mk, const float *p, const float *x, pdhcg_info *info) {
  if (!mk || !p || !x) return fail(PDHCG_ERR_ARG, "null argument");
  HIPC(launch_gather_f32_to_f64(p, mk->perm, mk->Pk, mk->m, mk->stream));
  EvalIO io;
  std::memset(&io, 0, sizeof(io));
  io.xc = x;
  io.pc = mk->Pk;
  io.want_cc = 1;
  io.rowscale = mk->rowmax;
  int32_t rc = enqueue_eval(mk, io);
  if (rc != PDHCG_OK) return rc;
  rc = pull_state(mk);
  if (rc != PDHCG_OK) return rc;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->rel_primal = mk->hS->kkt[0][0];
    info->rel_dual = mk->hS->kkt[0][1];
    info->rel_gap = mk->hS->kkt[0][2];
    info->rel_kkt = kkt_max(mk->hS->kkt[0]);
    info->status = PDHCG_OK;
  }
  return PDHCG_OK;
}

extern "C" int32_t pdhcg_row_prox(pdhcg_market mk, const float *x_in, const float *p, double tau,
                                  const pdhcg_params *params, float *x_out, float *s_out) {
  if (!mk || !x_in || !p || !x_out) return fail(PDHCG_ERR_ARG, "null argument");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(PDHCG_ERR_ARG, "tau must be finite and > 0");
  pdhcg_params dflt;
  pdhcg_default_params(&dflt);
  const pdhcg_params *prm = params ? params : &dflt;
  int32_t rc = check_params(prm);
  if (rc == PDHCG_OK) rc = check_search(mk, prm);
  if (rc != PDHCG_OK) return rc;
  RowIO io = row_io_state(prm);
  io.use_state = 0;
  io.colsum = 0;
  HIPC(launch_gather_f32_to_f64(p, mk->perm, mk->Pk, mk->m, mk->stream));
  io.xin = x_in;
  io.p = mk->Pk;
  io.xout = x_out;
  io.s_out = s_out;
  io.tau = tau;
  io.wfold = 0.0f;
  const MarketDev md = mk->dev();
  if (io.search == PDHCG_SEARCH_KSECTION_WAVE)
    HIPC(launch_row_kwave(md, io, mk->total_wg, mk->stream));
  else
    for (const Bin &b : mk->bins)
      HIPC(launch_row_pass(md, mk->bindev(b), b.G, b.E, mk->lds_row, io, b.nwg, mk->stream));
  return PDHCG_OK;
}

extern "C" int32_t pdhcg_solve(pdhcg_market mk, const pdhcg_params *params, int32_t warm,
                               float *p, float *x, float *t, pdhcg_info *info) {
  if (!mk || !p || !x) return fail(PDHCG_ERR_ARG, "null argument");
  pdhcg_params dflt;
  pdhcg_default_params(&dflt);
  const pdhcg_params *prm = params ? params : &dflt;
  int32_t rc = check_params(prm);
  if (rc == PDHCG_OK) rc = check_search(mk, prm);
  if (rc != PDHCG_OK) return rc;
  hipStream_t st = mk->stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int m = mk->m;
  const int64_t nnz = mk->nnz;

  // Initial point (reading of Alg. 2's unspecified start): x0_ij = 1/deg_j
  // (every column sums to one), p0_j = sum(w)/m (Sec. 3, Fact 1: the prices
  // sum to the budgets).  A warm start copies the caller's point.
  if (warm) {
    HIPC(hipMemcpyAsync(mk->X[0], x, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
    HIPC(launch_gather_f32_to_f64(p, mk->perm, mk->P[0], m, st));
  } else {
    HIPC(launch_init_point(mk->col, mk->deg, nnz, mk->X[0], mk->P[0], m,
                           mk->sumw / (double)m, st));
  }
  if (mk->srow) HIPC(launch_zero_f32(mk->srow, mk->n, st));  // no previous roots
  DevState &S = *mk->hS;
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;

  // Column sums and KKT error of the starting point.
  {
    EvalIO io;
    std::memset(&io, 0, sizeof(io));
    io.xc = mk->X[0];
    io.pc = mk->P[0];
    io.want_cc = 1;
    io.cavg_out = mk->C[1];
    io.rowscale = mk->rowmax;
    rc = enqueue_eval(mk, io);
    if (rc != PDHCG_OK) return rc;
  }
  rc = pull_state(mk);
  if (rc != PDHCG_OK) return rc;
  double kkt0 = kkt_max(S.kkt[0]);
  HIPC(launch_copy_f64(mk->C[1], mk->C[0], m, st));
  HIPC(launch_copy_f32(mk->X[0], mk->XA, nnz, st));
  HIPC(launch_copy_f64(mk->P[0], mk->PA, m, st));

  // Steps (Sec. 5): tau = eta/omega, sigma = eta*omega.
  const double knorm = std::sqrt((double)mk->maxdeg_col);
  const bool adaptive = prm->step_mode == PDHCG_STEP_ADAPTIVE;
  const double eta0 = prm->eta0 > 0.0 ? prm->eta0 : (adaptive ? 1.0 : 0.9 / knorm);
  const double omega0 = prm->omega0 > 0.0 ? prm->omega0 : 0.05 * mk->sumw / (double)m;
  double omega = omega0;
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  S.step_mode = adaptive ? 1 : 0;
  S.eta = eta0;
  S.eta0 = eta0;
  S.eta_lo = 0.01 * eta0;
  S.eta_hi = adaptive ? 3.0 * eta0 : eta0;
  S.omega = omega;
  S.tau = eta0 / omega;
  S.sigma = eta0 * omega;
  rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;

  const RowIO step_io = row_io_state(prm);
  EventPool pool;
  if (prm->timing) {
    pool.ev.resize(2 * (size_t)prm->eval_every, nullptr);
    for (auto &e : pool.ev) HIPC(hipEventCreate(&e));
  }
  double row_seconds = 0.0;
  int64_t row_launches = 0;
  double kkt_prev = INFINITY, kbest = INFINITY, kout[3] = {NAN, NAN, NAN};
  int32_t restarts = 0, evals = 0, status = PDHCG_MAX_ITER;
  bool cand_avg = false;
  int64_t total = 0;
  while (true) {
    const int64_t left = prm->max_iter - total;
    const int64_t nstep = std::min<int64_t>(prm->eval_every - (total % prm->eval_every), left);
    for (int64_t q = 0; q < nstep; ++q) {
      if (prm->timing)
        rc = enqueue_step(mk, step_io, pool.ev[2 * (size_t)q], pool.ev[2 * (size_t)q + 1]);
      else
        rc = enqueue_step(mk, step_io);
      if (rc != PDHCG_OK) return rc;
    }
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    if (prm->timing) {
      for (int64_t q = 0; q < nstep; ++q) {
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, pool.ev[2 * (size_t)q], pool.ev[2 * (size_t)q + 1]));
        row_seconds += 1e-3 * (double)ms;
        ++row_launches;
      }
    }
    if (S.total != total + nstep)
      return fail(PDHCG_ERR_HIP, "device iteration counter did not advance as expected");
    total = S.total;
    // KKT check of the current and the averaged point (Sec. 5 Criteria).
    const bool has_avg = S.k_in > 0;
    EvalIO io;
    std::memset(&io, 0, sizeof(io));
    io.xc = mk->X[S.ix[0]];
    io.pc = mk->P[S.ip[0]];
    io.xa = has_avg ? mk->X[S.ix[2]] : nullptr;
    io.pa = mk->P[S.ip[2]];
    io.wfold = (has_avg && S.fold) ? (float)(1.0 / (double)S.k_in) : 0.0f;
    io.xanc = mk->XA;
    io.panc = mk->PA;
    io.tc = mk->T[0];
    io.ta = mk->T[1];
    io.rowscale = mk->rowmax;
    io.want_cc = 0;
    io.ccur = mk->C[S.ic[1]];
    io.cavg_out = mk->C[S.ic[2]];
    io.pa_out = mk->P[S.ip[2]];
    rc = enqueue_eval(mk, io);
    if (rc != PDHCG_OK) return rc;
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    S.fold = 0;
    ++evals;
    const double kc = kkt_max(S.kkt[0]);
    const double ka = has_avg ? kkt_max(S.kkt[1]) : INFINITY;
    if (!std::isfinite(kc) && !std::isfinite(ka)) {
      status = PDHCG_ERR_NUMERIC;
      fail(status, "non-finite KKT error at iteration " + std::to_string(total));
      break;
    }
    cand_avg = ka < kc;
    const double kcand = cand_avg ? ka : kc;
    std::memcpy(kout, cand_avg ? S.kkt[1] : S.kkt[0], sizeof(kout));
    kbest = kcand;
    if (prm->verbose)
      std::fprintf(stderr,
                   "[pdhcg] it=%lld kin=%lld acc=%lld cur=%.3e (%.2e %.2e %.2e) avg=%.3e "
                   "(%.2e %.2e %.2e) eta=%.3e omega=%.3e emax=%.3e dx2=%.3e/%.3e "
                   "dp2=%.3e/%.3e\n",
                   (long long)total, (long long)S.k_in, (long long)S.accepted, kc,
                   S.kkt[0][0], S.kkt[0][1], S.kkt[0][2], ka, S.kkt[1][0], S.kkt[1][1],
                   S.kkt[1][2], S.eta, omega, S.emax_last, S.dxa2[0], S.dxa2[1], S.dpa2[0],
                   S.dpa2[1]);
    if (kcand <= prm->tol) {
      status = PDHCG_OK;
      break;
    }
    if (total >= prm->max_iter) {
      status = PDHCG_MAX_ITER;
      break;
    }
    if (prm->restart == PDHCG_RESTART_ADAPTIVE) {
      const bool do_restart =
          (kcand <= prm->beta_sufficient * kkt0) ||
          (kcand <= prm->beta_necessary * kkt0 && kcand > kkt_prev) ||
          ((double)S.since >= prm->beta_artificial * (double)S.total);
      if (do_restart) {
        if (cand_avg) {
          std::swap(S.ix[0], S.ix[2]);
          std::swap(S.ip[0], S.ip[2]);
          std::swap(S.ic[1], S.ic[2]);  // column sums of the average are in the trial slot
        }
        HIPC(launch_copy_f64(mk->C[S.ic[1]], mk->C[S.ic[0]], m, st));
        HIPC(launch_copy_f32(mk->X[S.ix[0]], mk->XA, nnz, st));
        HIPC(launch_copy_f64(mk->P[S.ip[0]], mk->PA, m, st));
        const double dx = std::sqrt(S.dxa2[cand_avg ? 1 : 0]);
        const double dp = std::sqrt(S.dpa2[cand_avg ? 1 : 0]);
        if (dx > 1e-10 && dp > 1e-10)
          omega = std::exp(prm->theta * std::log(dp / dx) + (1.0 - prm->theta) * std::log(omega));
        ++restarts;
        if (prm->omega_check_every > 0 && restarts % prm->omega_check_every == 0 &&
            (omega < omega0 / prm->omega_bound || omega > omega0 * prm->omega_bound))
          omega = omega0;
        kkt0 = kcand;
        kkt_prev = INFINITY;
        S.k_in = 0;
        S.since = 0;
        cand_avg = false;
      } else {
        kkt_prev = kcand;
      }
    }
    S.omega = omega;
    S.tau = S.eta / omega;
    S.sigma = S.eta * omega;
    rc = push_state(mk);
    if (rc != PDHCG_OK) return rc;
  }

  // Output the requested point.
  bool out_avg = false;
  if (prm->output == PDHCG_OUTPUT_CANDIDATE) out_avg = cand_avg;
  if (prm->output == PDHCG_OUTPUT_AVERAGE) out_avg = S.k_in > 0;
  const float *xs = mk->X[out_avg ? S.ix[2] : S.ix[0]];
  const double *ps = mk->P[out_avg ? S.ip[2] : S.ip[0]];
  HIPC(hipMemcpyAsync(x, xs, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
  HIPC(launch_gather_f64_to_f32(ps, mk->inv, p, m, st));
  if (t) HIPC(hipMemcpyAsync(t, mk->T[out_avg ? 1 : 0], (size_t)mk->n * 4, hipMemcpyDeviceToDevice, st));
  if (prm->output != PDHCG_OUTPUT_CANDIDATE) {
    const int z = out_avg ? 1 : 0;
    std::memcpy(kout, S.kkt[z], sizeof(kout));
    kbest = kkt_max(S.kkt[z]);
  }
  HIPC(hipStreamSynchronize(st));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    info->rel_kkt = kbest;
    info->rel_primal = kout[0];
    info->rel_dual = kout[1];
    info->rel_gap = kout[2];
    info->eta = S.eta;
    info->omega = omega;
    info->seconds = secs;
    info->iters = S.total;
    info->accepted = S.accepted;
    info->restarts = restarts;
    info->status = status;
    info->evals = evals;
    info->search_rounds_max = (int32_t)S.rounds_max;
    info->search_rounds_mean =
        S.rows_searched ? (double)S.rounds_sum / (double)S.rows_searched : 0.0;
    info->row_pass_seconds = row_seconds;
    info->row_pass_launches = row_launches;
  }
  return status;
}

extern "C" int32_t pdhcg_solve_fixed_restart(pdhcg_market mk, int32_t K, int32_t restarts,
                                             double eta, const float *p_ref, double *dist,
                                             double *kkt, float *p, float *x, pdhcg_info *info) {
  if (!mk || !p || !x) return fail(PDHCG_ERR_ARG, "null argument");
  if (K < 1 || restarts < 0) return fail(PDHCG_ERR_ARG, "K >= 1 and restarts >= 0 required");
  if (!(eta >= 0.0) || !std::isfinite(eta)) return fail(PDHCG_ERR_ARG, "eta must be finite");
  hipStream_t st = mk->stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int m = mk->m;
  const int64_t nnz = mk->nnz;
  const double knorm = std::sqrt((double)std::max(1, mk->maxdeg_col));
  if (!(eta > 0.0)) eta = 1.0 / (2.0 * knorm);
  pdhcg_params prm;
  pdhcg_default_params(&prm);

  HIPC(launch_init_point(mk->col, mk->deg, nnz, mk->X[0], mk->P[0], m, mk->sumw / (double)m, st));
  if (mk->srow) HIPC(launch_zero_f32(mk->srow, mk->n, st));
  // the price anchor of the KKT pass holds the reference prices, so the pass
  // returns |p - p_ref|^2 for the current and the averaged point
  if (p_ref)
    HIPC(launch_gather_f32_to_f64(p_ref, mk->perm, mk->PA, m, st));
  else
    HIPC(launch_copy_f64(mk->P[0], mk->PA, m, st));
  HIPC(launch_copy_f32(mk->X[0], mk->XA, nnz, st));
  DevState &S = *mk->hS;
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  int32_t rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;
  {
    EvalIO io;
    std::memset(&io, 0, sizeof(io));
    io.xc = mk->X[0];
    io.pc = mk->P[0];
    io.want_cc = 1;
    io.cavg_out = mk->C[1];
    io.rowscale = mk->rowmax;
    io.panc = mk->PA;
    rc = enqueue_eval(mk, io);
    if (rc != PDHCG_OK) return rc;
  }
  rc = pull_state(mk);
  if (rc != PDHCG_OK) return rc;
  if (dist) dist[0] = p_ref ? std::sqrt(S.dpa2[0]) : 0.0;
  if (kkt) kkt[0] = kkt_max(S.kkt[0]);
  double klast = kkt_max(S.kkt[0]);
  double kparts[3] = {S.kkt[0][0], S.kkt[0][1], S.kkt[0][2]};
  HIPC(launch_copy_f64(mk->C[1], mk->C[0], m, st));
  // fixed steps sigma = tau = eta (primal weight one)
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  S.step_mode = 0;
  S.eta = S.eta0 = S.eta_lo = S.eta_hi = eta;
  S.omega = 1.0;
  S.tau = eta;
  S.sigma = eta;
  rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;
  const RowIO step_io = row_io_state(&prm);
  for (int32_t r = 0; r < restarts; ++r) {
    for (int32_t q = 0; q < K; ++q) {
      rc = enqueue_step(mk, step_io);
      if (rc != PDHCG_OK) return rc;
    }
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    // the average of the K iterates (with the lagged fold of the last one)
    EvalIO io;
    std::memset(&io, 0, sizeof(io));
    io.xc = mk->X[S.ix[0]];
    io.pc = mk->P[S.ip[0]];
    io.xa = mk->X[S.ix[2]];
    io.pa = mk->P[S.ip[2]];
    io.wfold = S.fold ? (float)(1.0 / (double)S.k_in) : 0.0f;
    io.xanc = mk->XA;
    io.panc = mk->PA;
    io.tc = mk->T[0];
    io.ta = mk->T[1];
    io.rowscale = mk->rowmax;
    io.ccur = mk->C[S.ic[1]];
    io.cavg_out = mk->C[S.ic[2]];
    io.pa_out = mk->P[S.ip[2]];
    rc = enqueue_eval(mk, io);
    if (rc != PDHCG_OK) return rc;
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    if (dist) dist[r + 1] = p_ref ? std::sqrt(S.dpa2[1]) : 0.0;
    klast = kkt_max(S.kkt[1]);
    std::memcpy(kparts, S.kkt[1], sizeof(kparts));
    if (kkt) kkt[r + 1] = klast;
    if (!std::isfinite(klast)) return fail(PDHCG_ERR_NUMERIC, "non-finite KKT error");
    // restart to the average (Alg. 2); no extrapolation after a restart
    std::swap(S.ix[0], S.ix[2]);
    std::swap(S.ip[0], S.ip[2]);
    std::swap(S.ic[1], S.ic[2]);
    HIPC(launch_copy_f64(mk->C[S.ic[1]], mk->C[S.ic[0]], m, st));
    S.fold = 0;
    S.k_in = 0;
    S.since = 0;
    rc = push_state(mk);
    if (rc != PDHCG_OK) return rc;
  }
  HIPC(hipMemcpyAsync(x, mk->X[S.ix[0]], (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
  HIPC(launch_gather_f64_to_f32(mk->P[S.ip[0]], mk->inv, p, m, st));
  HIPC(hipStreamSynchronize(st));
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->rel_kkt = klast;
    info->rel_primal = kparts[0];
    info->rel_dual = kparts[1];
    info->rel_gap = kparts[2];
    info->eta = eta;
    info->omega = 1.0;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->iters = S.total;
    info->accepted = S.accepted;
    info->restarts = restarts;
    info->status = PDHCG_OK;
    info->search_rounds_max = (int32_t)S.rounds_max;
    info->search_rounds_mean =
        S.rows_searched ? (double)S.rounds_sum / (double)S.rows_searched : 0.0;
  }
  return PDHCG_OK;
}

namespace {

// PDHG needs every good's price and column partial in LDS, 2-byte good ids
// and register-resident rows (at most 512 entries).
int32_t check_pdhg(pdhcg_market mk) {
  if (mk->lds_row != 3 || !mk->col16 || !mk->lds_eval || mk->hot != mk->m)
    return fail(PDHCG_ERR_UNSUPPORTED, "restarted PDHG is built for markets whose goods all fit in "
                                       "LDS (m <= 10000 on gfx950)");
  for (const Bin &b : mk->bins)
    if (b.G == 0)
      return fail(PDHCG_ERR_UNSUPPORTED, "restarted PDHG is built for rows of at most 512 entries");
  return PDHCG_OK;
}

int32_t pdhg_buffers(pdhcg_market mk) {
  if (mk->pdhg_buf) return PDHCG_OK;
  const size_t n = (size_t)mk->n;
  HIPC(dalloc(&mk->pdhg_buf, 11 * n));
  double *b = mk->pdhg_buf;
  PdhgDev &d = mk->pdhg;
  d.T0 = b; d.T1 = b + n; d.T2 = b + 2 * n;
  d.Y0 = b + 3 * n; d.Y1 = b + 4 * n; d.Y2 = b + 5 * n;
  d.G0 = b + 6 * n; d.G1 = b + 7 * n; d.G2 = b + 8 * n;
  d.TA = b + 9 * n; d.YA = b + 10 * n;
  return PDHCG_OK;
}

double *pick_d(double *a, double *b, double *c, int i) { return i == 0 ? a : (i == 1 ? b : c); }

// KKT pass of PDHG over the current point and, when has_avg, the average
// (with the lagged fold of the kept iterate).
int32_t enqueue_pdhg_eval(pdhcg_market mk, const DevState &S, bool has_avg, float wfold,
                          bool want_cc) {
  const MarketDev md = mk->dev();
  const PdhgDev &pd = mk->pdhg;
  EvalIO io;
  std::memset(&io, 0, sizeof(io));
  io.xc = mk->X[S.ix[0]];
  io.pc = mk->P[S.ip[0]];
  io.xa = has_avg ? mk->X[S.ix[2]] : nullptr;
  io.pa = mk->P[S.ip[2]];
  io.wfold = wfold;
  io.xanc = mk->XA;
  io.panc = mk->PA;
  io.tc = mk->T[0];
  io.ta = mk->T[1];
  io.rowscale = mk->rowmax;
  io.want_cc = want_cc ? 1 : 0;
  io.ccur = mk->C[S.ic[1]];
  io.cavg_out = want_cc ? mk->C[S.ic[1]] : mk->C[S.ic[2]];
  io.pa_out = has_avg ? mk->P[S.ip[2]] : nullptr;
  io.evalpart = mk->evalpart;
  io.evalcs = mk->evalcs;
  io.evalchunk = mk->evalchunk;
  io.cacc = mk->cacc;
  io.gmax = mk->gmax;
  io.gsum = mk->gsum;
  const double *tc = pick_d(pd.T0, pd.T1, pd.T2, S.ix[0]);
  const double *yc = pick_d(pd.Y0, pd.Y1, pd.Y2, S.ip[0]);
  double *ta = pick_d(pd.T0, pd.T1, pd.T2, S.ix[2]);
  double *ya = pick_d(pd.Y0, pd.Y1, pd.Y2, S.ip[2]);
  double *gavg = has_avg ? pick_d(pd.G0, pd.G1, pd.G2, S.ic[2]) : nullptr;
  for (const Bin &b : mk->bins)
    HIPC(launch_pdhg_eval(md, pd, mk->bindev(b), b.G, b.E, io, tc, yc, ta, ya, gavg, b.nwg,
                          mk->total_wg, mk->stream));
  HIPC(launch_eval_chunks(md, io, mk->total_wg, mk->stream));
  HIPC(launch_eval_col_stats(md, io, mk->total_wg, 1, mk->stream));
  HIPC(launch_pdhg_eval_final(md, mk->total_wg, mk->stream));
  return PDHCG_OK;
}

}  // namespace

extern "C" int32_t pdhcg_pdhg_solve(pdhcg_market mk, const pdhcg_params *params, int32_t warm,
                                    float *p, float *x, float *t, float *y, pdhcg_info *info) {
  if (!mk || !p || !x) return fail(PDHCG_ERR_ARG, "null argument");
  pdhcg_params dflt;
  pdhcg_default_params(&dflt);
  const pdhcg_params *prm = params ? params : &dflt;
  int32_t rc = check_params(prm);
  if (rc == PDHCG_OK) rc = check_pdhg(mk);
  if (rc == PDHCG_OK) rc = pdhg_buffers(mk);
  if (rc != PDHCG_OK) return rc;
  hipStream_t st = mk->stream;
  const auto t0 = std::chrono::steady_clock::now();
  const int n = mk->n, m = mk->m;
  const int64_t nnz = mk->nnz;
  const MarketDev md = mk->dev();
  const PdhgDev &pd = mk->pdhg;

  // Initial point (readings shared with the oracle): x0_ij = 1/deg_j,
  // p0_j = sum(w)/m, t0 = U x0, y0 = w / t0; a warm start takes p, x and,
  // when given, t and y (caller's units).  g_prev = g = t - U x.
  if (warm) {
    HIPC(hipMemcpyAsync(mk->X[0], x, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
    HIPC(launch_gather_f32_to_f64(p, mk->perm, mk->P[0], m, st));
  } else {
    HIPC(launch_init_point(mk->col, mk->deg, nnz, mk->X[0], mk->P[0], m, mk->sumw / (double)m, st));
  }
  HIPC(launch_pdhg_rows_init(md, mk->X[0], warm ? t : nullptr, warm ? y : nullptr, mk->rowmax,
                             pd.T0, pd.Y0, pd.G0, pd.G1, st));
  DevState &S = *mk->hS;
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;
  // column sums and KKT error of the starting point
  rc = enqueue_pdhg_eval(mk, S, false, 0.0f, true);
  if (rc != PDHCG_OK) return rc;
  rc = pull_state(mk);
  if (rc != PDHCG_OK) return rc;
  double kkt0 = kkt_max(S.kkt[0]);
  HIPC(launch_copy_f64(mk->C[1], mk->C[0], m, st));
  HIPC(launch_copy_f32(mk->X[0], mk->XA, nnz, st));
  HIPC(launch_copy_f64(mk->P[0], mk->PA, m, st));
  HIPC(launch_copy_f64(pd.T0, pd.TA, n, st));
  HIPC(launch_copy_f64(pd.Y0, pd.YA, n, st));

  // Steps (Sec. 5): tau = eta/omega, sigma = eta*omega.  Fixed mode:
  // eta = 0.9 / B, B = sqrt(max col degree) + 1 + sqrt(max col degree * max
  // row degree) >= ||K|| for K = [1^T 0; -U I] with |u_ij| <= 1.
  const double kbound = std::sqrt((double)mk->maxdeg_col) + 1.0 +
                        std::sqrt((double)mk->maxdeg_col * (double)mk->maxdeg_row);
  const bool adaptive = prm->step_mode == PDHCG_STEP_ADAPTIVE;
  const double eta0 = prm->eta0 > 0.0 ? prm->eta0 : (adaptive ? 1.0 : 0.9 / kbound);
  const double omega0 = prm->omega0 > 0.0 ? prm->omega0 : 0.05 * mk->sumw / (double)m;
  double omega = omega0;
  std::memset(&S, 0, sizeof(S));
  S.ix[0] = 0; S.ix[1] = 1; S.ix[2] = 2;
  S.ip[0] = 0; S.ip[1] = 1; S.ip[2] = 2;
  S.ic[0] = 0; S.ic[1] = 1; S.ic[2] = 2;
  S.step_mode = adaptive ? 1 : 0;
  S.eta = eta0;
  S.eta0 = eta0;
  S.eta_lo = 0.01 * eta0;
  S.eta_hi = adaptive ? 3.0 * eta0 : eta0;
  S.omega = omega;
  S.tau = eta0 / omega;
  S.sigma = eta0 * omega;
  rc = push_state(mk);
  if (rc != PDHCG_OK) return rc;

  EventPool pool;
  if (prm->timing) {
    pool.ev.resize(2 * (size_t)prm->eval_every, nullptr);
    for (auto &e : pool.ev) HIPC(hipEventCreate(&e));
  }
  double row_seconds = 0.0;
  int64_t row_launches = 0;
  double kkt_prev = INFINITY, kbest = INFINITY, kout[3] = {NAN, NAN, NAN};
  int32_t restarts = 0, evals = 0, status = PDHCG_MAX_ITER;
  bool cand_avg = false;
  int64_t total = 0;
  while (true) {
    const int64_t left = prm->max_iter - total;
    const int64_t nstep = std::min<int64_t>(prm->eval_every - (total % prm->eval_every), left);
    for (int64_t q = 0; q < nstep; ++q) {
      HIPC(launch_pstep(md, 0, st));
      if (prm->timing) HIPC(hipEventRecord(pool.ev[2 * (size_t)q], st));
      for (const Bin &b : mk->bins)
        HIPC(launch_pdhg_row(md, pd, mk->bindev(b), b.G, b.E, b.nwg, st));
      if (prm->timing) HIPC(hipEventRecord(pool.ev[2 * (size_t)q + 1], st));
      HIPC(launch_col_decide_pdhg(md, mk->total_wg, st));
    }
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    if (prm->timing) {
      for (int64_t q = 0; q < nstep; ++q) {
        float ms = 0.0f;
        HIPC(hipEventElapsedTime(&ms, pool.ev[2 * (size_t)q], pool.ev[2 * (size_t)q + 1]));
        row_seconds += 1e-3 * (double)ms;
        ++row_launches;
      }
    }
    if (S.total != total + nstep)
      return fail(PDHCG_ERR_HIP, "device iteration counter did not advance as expected");
    total = S.total;
    const bool has_avg = S.k_in > 0;
    const float wfold = (has_avg && S.fold) ? (float)(1.0 / (double)S.k_in) : 0.0f;
    rc = enqueue_pdhg_eval(mk, S, has_avg, wfold, false);
    if (rc != PDHCG_OK) return rc;
    rc = pull_state(mk);
    if (rc != PDHCG_OK) return rc;
    S.fold = 0;
    ++evals;
    const double kc = kkt_max(S.kkt[0]);
    const double ka = has_avg ? kkt_max(S.kkt[1]) : INFINITY;
    if (!std::isfinite(kc) && !std::isfinite(ka)) {
      status = PDHCG_ERR_NUMERIC;
      fail(status, "non-finite KKT error at iteration " + std::to_string(total));
      break;
    }
    cand_avg = ka < kc;
    const double kcand = cand_avg ? ka : kc;
    std::memcpy(kout, cand_avg ? S.kkt[1] : S.kkt[0], sizeof(kout));
    kbest = kcand;
    if (prm->verbose)
      std::fprintf(stderr, "[pdhg] it=%lld cur=%.3e avg=%.3e eta=%.3e omega=%.3e\n",
                   (long long)total, kc, ka, S.eta, omega);
    if (kcand <= prm->tol) {
      status = PDHCG_OK;
      break;
    }
    if (total >= prm->max_iter) {
      status = PDHCG_MAX_ITER;
      break;
    }
    if (prm->restart == PDHCG_RESTART_ADAPTIVE) {
      const bool do_restart =
          (kcand <= prm->beta_sufficient * kkt0) ||
          (kcand <= prm->beta_necessary * kkt0 && kcand > kkt_prev) ||
          ((double)S.since >= prm->beta_artificial * (double)S.total);
      if (do_restart) {
        if (cand_avg) {
          std::swap(S.ix[0], S.ix[2]);
          std::swap(S.ip[0], S.ip[2]);
          std::swap(S.ic[1], S.ic[2]);  // column sums and g of the average are in the trial slot
        }
        HIPC(launch_copy_f64(mk->C[S.ic[1]], mk->C[S.ic[0]], m, st));
        HIPC(launch_copy_f64(pick_d(pd.G0, pd.G1, pd.G2, S.ic[1]),
                             pick_d(pd.G0, pd.G1, pd.G2, S.ic[0]), n, st));
        HIPC(launch_copy_f32(mk->X[S.ix[0]], mk->XA, nnz, st));
        HIPC(launch_copy_f64(mk->P[S.ip[0]], mk->PA, m, st));
        HIPC(launch_copy_f64(pick_d(pd.T0, pd.T1, pd.T2, S.ix[0]), pd.TA, n, st));
        HIPC(launch_copy_f64(pick_d(pd.Y0, pd.Y1, pd.Y2, S.ip[0]), pd.YA, n, st));
        const double dx = std::sqrt(S.dxa2[cand_avg ? 1 : 0]);
        const double dp = std::sqrt(S.dpa2[cand_avg ? 1 : 0]);
        if (dx > 1e-10 && dp > 1e-10)
          omega = std::exp(prm->theta * std::log(dp / dx) + (1.0 - prm->theta) * std::log(omega));
        ++restarts;
        if (prm->omega_check_every > 0 && restarts % prm->omega_check_every == 0 &&
            (omega < omega0 / prm->omega_bound || omega > omega0 * prm->omega_bound))
          omega = omega0;
        kkt0 = kcand;
        kkt_prev = INFINITY;
        S.k_in = 0;
        S.since = 0;
        cand_avg = false;
      } else {
        kkt_prev = kcand;
      }
    }
    S.omega = omega;
    S.tau = S.eta / omega;
    S.sigma = S.eta * omega;
    rc = push_state(mk);
    if (rc != PDHCG_OK) return rc;
  }

  bool out_avg = false;
  if (prm->output == PDHCG_OUTPUT_CANDIDATE) out_avg = cand_avg;
  if (prm->output == PDHCG_OUTPUT_AVERAGE) out_avg = S.k_in > 0;
  const float *xs = mk->X[out_avg ? S.ix[2] : S.ix[0]];
  const double *ps = mk->P[out_avg ? S.ip[2] : S.ip[0]];
  HIPC(hipMemcpyAsync(x, xs, (size_t)nnz * 4, hipMemcpyDeviceToDevice, st));
  HIPC(launch_gather_f64_to_f32(ps, mk->inv, p, m, st));
  if (t || y)
    HIPC(launch_pdhg_rows_out(pick_d(pd.T0, pd.T1, pd.T2, out_avg ? S.ix[2] : S.ix[0]),
                              pick_d(pd.Y0, pd.Y1, pd.Y2, out_avg ? S.ip[2] : S.ip[0]),
                              mk->rowmax, t, y, n, st));
  if (prm->output != PDHCG_OUTPUT_CANDIDATE) {
    const int z = out_avg ? 1 : 0;
    std::memcpy(kout, S.kkt[z], sizeof(kout));
    kbest = kkt_max(S.kkt[z]);
  }
  HIPC(hipStreamSynchronize(st));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->rel_kkt = kbest;
    info->rel_primal = kout[0];
    info->rel_dual = kout[1];
    info->rel_gap = kout[2];
    info->eta = S.eta;
    info->omega = omega;
    info->seconds = secs;
    info->iters = S.total;
    info->accepted = S.accepted;
    info->restarts = restarts;
    info->status = status;
    info->evals = evals;
    info->row_pass_seconds = row_seconds;
    info->row_pass_launches = row_launches;
  }
  return status;
}

extern "C" int32_t pdhcg_arrow_debreu(pdhcg_market mk, const int32_t *e_row_ptr,
                                      const int32_t *e_col, const float *e_val, int64_t e_nnz,
                                      const pdhcg_params *inner, double outer_tol,
                                      int32_t outer_max, float *w, float *p, float *x,
                                      int32_t *outer_iters, int64_t *inner_iters,
                                      pdhcg_info *info) {
  if (!mk || !e_row_ptr || !e_col || !e_val || !w || !p || !x)
    return fail(PDHCG_ERR_ARG, "null argument");
  if (e_nnz <= 0 || outer_max <= 0 || !(outer_tol >= 0.0))
    return fail(PDHCG_ERR_ARG, "e_nnz > 0, outer_max > 0 and outer_tol >= 0 required");
  hipStream_t st = mk->stream;
  const int n = mk->n, m = mk->m;
  // Validate E on the host: CSR shape, e >= 0, every agent owns something,
  // every column sums to one (Sec. 4 normalisation) within 1e-4.
  {
    std::vector<int32_t> rp((size_t)n + 1), cl((size_t)e_nnz);
    std::vector<float> ev((size_t)e_nnz);
    HIPC(hipMemcpyAsync(rp.data(), e_row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(cl.data(), e_col, cl.size() * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipMemcpyAsync(ev.data(), e_val, ev.size() * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (rp[0] != 0 || (int64_t)rp[(size_t)n] != e_nnz) return fail(PDHCG_ERR_ARG, "bad E row_ptr");
    std::vector<double> cs((size_t)m, 0.0);
    for (int i = 0; i < n; ++i) {
      if (rp[(size_t)i + 1] < rp[(size_t)i]) return fail(PDHCG_ERR_ARG, "bad E row_ptr");
      bool owns = false;
      for (int32_t k = rp[(size_t)i]; k < rp[(size_t)i + 1]; ++k) {
        if (cl[(size_t)k] < 0 || cl[(size_t)k] >= m || !(ev[(size_t)k] >= 0.0f) ||
            !std::isfinite(ev[(size_t)k]))
          return fail(PDHCG_ERR_ARG, "bad E entry " + std::to_string(k));
        cs[(size_t)cl[(size_t)k]] += ev[(size_t)k];
        owns |= ev[(size_t)k] > 0.0f;
      }
      if (!owns) return fail(PDHCG_ERR_ASSUMPTION, "agent " + std::to_string(i) + " owns nothing");
    }
    for (int j = 0; j < m; ++j)
      if (std::fabs(cs[(size_t)j] - 1.0) > 1e-4)
        return fail(PDHCG_ERR_ARG, "column " + std::to_string(j) + " of E does not sum to one");
  }
  std::vector<float> pprev((size_t)m), pcur((size_t)m);
  int32_t rc = PDHCG_MAX_ITER, k = 0;
  int64_t tot_inner = 0;
  pdhcg_info last;
  std::memset(&last, 0, sizeof(last));
  const auto t0 = std::chrono::steady_clock::now();
  for (k = 0; k < outer_max; ++k) {
    int32_t r = pdhcg_set_budgets(mk, w);
    if (r != PDHCG_OK) return r;
    r = pdhcg_solve(mk, inner, k > 0 ? 1 : 0, p, x, nullptr, &last);
    tot_inner += last.iters;
    if (r < 0) {
      rc = r;
      break;
    }
    HIPC(hipMemcpyAsync(pcur.data(), p, (size_t)m * 4, hipMemcpyDeviceToHost, st));
    HIPC(launch_budget_spmv(e_row_ptr, e_col, e_val, p, w, n, st));
    HIPC(hipStreamSynchronize(st));
    double change = INFINITY;
    if (k > 0) {
      double num = 0.0, den = 0.0;
      for (int j = 0; j < m; ++j) {
        num = std::max(num, (double)std::fabs(pcur[(size_t)j] - pprev[(size_t)j]));
        den = std::max(den, (double)std::fabs(pprev[(size_t)j]));
      }
      change = num / den;
    }
    pprev.swap(pcur);
    if (inner && inner->verbose)
      std::fprintf(stderr, "[pdhcg-ad] outer=%d inner_iters=%lld kkt=%.3e change=%.3e\n", k,
                   (long long)last.iters, last.rel_kkt, change);
    if (k > 0 && change <= outer_tol) {
      // the stop compares p^k = p(E p^{k-1}) with p^{k-1}: it certifies a
      // fixed point only when the solve that produced p^k reached its
      // tolerance (an inner solve cut off by max_iter may barely move the
      // warm-started prices)
      rc = (r == PDHCG_OK) ? PDHCG_OK : PDHCG_MAX_ITER;
      if (rc != PDHCG_OK)
        fail(rc, "outer change below tolerance but the last inner solve stopped at max_iter");
      ++k;
      break;
    }
  }
  if (outer_iters) *outer_iters = k;
  if (inner_iters) *inner_iters = tot_inner;
  if (info) {
    *info = last;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->iters = tot_inner;
    info->status = rc;
  }
  return rc;
}

// ------------------------------------------------------------ reverse mode --

namespace {

// Device buffers of one backward call (freed on every exit path).
struct AdjBuffers {
  std::vector<void *> owned;
  ~AdjBuffers() {
    for (void *p : owned)
      if (p) (void)hipFree(p);
  }
  template <typename T>
  hipError_t get(T **p, size_t count) {
    hipError_t e = dalloc(p, count);
    if (e == hipSuccess) owned.push_back(*p);
    return e;
  }
};

// Goods whose column sums come from LDS partials ([0, hot)); the others are
// summed by device atomics.
int lds_goods(pdhcg_market mk) { return (mk->lds_row & 1) ? mk->hot : 0; }

// Column sums of the row pass just launched (explicit mode) into out.
int32_t finish_colsum(pdhcg_market mk, double *chunk, double *atomic_sum, double *out) {
  const int h = lds_goods(mk);
  HIPC(launch_sum_partials(mk->colpart, mk->total_wg, h, mk->m, chunk, mk->stream));
  HIPC(launch_finish_colsum(chunk, atomic_sum, h, mk->m, out, mk->stream));
  return PDHCG_OK;
}

// Bump allocation over a caller-provided device region (the no-allocation
// entry point's static workspace): 256-byte aligned pieces, never freed.
struct ArenaBuffers {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  template <typename T>
  hipError_t get(T **p, size_t count) {
    const size_t bytes = ((std::max<size_t>(count, 1) * sizeof(T)) + 255) & ~size_t(255);
    *p = nullptr;
    if (used + bytes > cap) return hipErrorOutOfMemory;
    *p = reinterpret_cast<T *>(base + used);
    used += bytes;
    return hipSuccess;
  }
};

// Device bytes the reverse mode's buffers take (as ArenaBuffers lays them
// out): checkpoints of x, p, c, c_prev; one segment of recomputed
// allocations; five nnz work arrays; the budget adjoint; seven goods arrays,
// the column-chunk sums and the per-good support counts.
size_t backward_bytes(int64_t nnz, int n, int m, int K, int L) {
  auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); };
  const size_t nck = (size_t)((K + L - 1) / L);
  size_t b = al(nck * nnz * 4) + al((size_t)L * nnz * 4) + 5 * al((size_t)nnz * 4) +
             al((size_t)n * 4) + 3 * al(nck * m * 8) + al((size_t)kColChunks * m * 8) +
             7 * al((size_t)m * 8) + al(((size_t)m + 1) * 4);
  return b;
}

template <typename Buffers>
int32_t backward_impl(pdhcg_market mk, const float *x, const float *p, double omega,
                      int32_t unroll, int32_t ckpt_every, const float *dL_dp, float *dL_du,
                      float *dL_dw, Buffers &buf) {
  const int n = mk->n, m = mk->m;
  const int64_t nnz = mk->nnz;
  const hipStream_t st = mk->stream;
  const MarketDev md = mk->dev();
  const int K = unroll, L = std::min(ckpt_every, unroll);
  const int nck = (K + L - 1) / L;

  float *ck_x = nullptr, *seg_x = nullptr, *xa = nullptr, *xb = nullptr;
  float *R0 = nullptr, *R1 = nullptr, *duh = nullptr, *dw = nullptr;
  double *ck_p = nullptr, *ck_c = nullptr, *ck_cp = nullptr, *pw = nullptr, *c = nullptr;
  double *cp = nullptr, *chunk = nullptr, *asum = nullptr, *P = nullptr, *B = nullptr,
         *Cn = nullptr;
  HIPC(buf.get(&ck_x, (size_t)nck * nnz));
  HIPC(buf.get(&seg_x, (size_t)L * nnz));
  HIPC(buf.get(&xa, (size_t)nnz));
  HIPC(buf.get(&xb, (size_t)nnz));
  HIPC(buf.get(&R0, (size_t)nnz));
  HIPC(buf.get(&R1, (size_t)nnz));
  HIPC(buf.get(&duh, (size_t)nnz));
  HIPC(buf.get(&dw, (size_t)n));
  HIPC(buf.get(&ck_p, (size_t)nck * m));
  HIPC(buf.get(&ck_c, (size_t)nck * m));
  HIPC(buf.get(&ck_cp, (size_t)nck * m));
  HIPC(buf.get(&pw, (size_t)m));
  HIPC(buf.get(&c, (size_t)m));
  HIPC(buf.get(&cp, (size_t)m));
  HIPC(buf.get(&chunk, (size_t)kColChunks * m));
  HIPC(buf.get(&asum, (size_t)m));
  HIPC(buf.get(&P, (size_t)m));
  HIPC(buf.get(&B, (size_t)m));
  HIPC(buf.get(&Cn, (size_t)m));
  int32_t *cnt = nullptr;
  HIPC(buf.get(&cnt, (size_t)m + 1));

  // Fixed step of the unrolled iteration: Lemma 1's condition
  // sigma tau ||K||^2 < 1 for the operator that moves near the start point.
  // Entries off the support of x stay at zero there (the prox clips them),
  // so K is the column-sum operator on the support: ||K|| = sqrt(largest
  // number of buyers with x_ij > 0 of a good).  eta = 0.9 / ||K||.
  HIPC(launch_active_colmax(mk->col, x, nnz, cnt, m, cnt + m, st));
  int32_t maxact = 0;
  HIPC(hipMemcpyAsync(&maxact, cnt + m, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const double eta = 0.9 / std::sqrt((double)std::max(1, maxact));
  const double tau = eta / omega, sigma = eta * omega;

  pdhcg_params dflt;
  pdhcg_default_params(&dflt);
  RowIO io = row_io_state(&dflt);
  io.use_state = 0;
  io.colsum = 1;
  io.tau = tau;
  io.wfold = 0.0f;
  io.csum = asum;
  io.p = pw;
  // One forward step from (xin, pw = p^j, c = c^j, cp = c^{j-1}) to xout,
  // pw = p^{j+1}, c = c^{j+1}, cp = c^j.
  auto forward = [&](const float *xin, float *xout) -> int32_t {
    HIPC(launch_adj_pstep(pw, c, cp, sigma, m, st));
    HIPC(hipMemcpyAsync(cp, c, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (lds_goods(mk) < m) HIPC(launch_zero_f64(asum, m, st));
    io.xin = xin;
    io.xout = xout;
    for (const Bin &b : mk->bins)
      HIPC(launch_row_pass(md, mk->bindev(b), b.G, b.E, mk->lds_row, io, b.nwg, st));
    if (mk->lds_row == 7) {
      const int32_t rc = enqueue_cold_sums(mk, md, 0, xout, asum, st);
      if (rc != PDHCG_OK) return rc;
    }
    return finish_colsum(mk, chunk, asum, c);
  };

  // forward sweep from the given point, one checkpoint every L steps
  HIPC(launch_gather_f32_to_f64(p, mk->perm, pw, m, st));
  HIPC(launch_colsum_atomic(mk->col, x, nnz, c, m, st));
  HIPC(hipMemcpyAsync(cp, c, (size_t)m * sizeof(double), hipMemcpyDeviceToDevice, st));
  // (it stops at the last checkpoint: the steps after it are recomputed by
  // the reverse sweep anyway)
  const float *xcur = x;
  const int jlast = (nck - 1) * L;
  for (int j = 0; j <= jlast; ++j) {
    if (j % L == 0) {
      const int q = j / L;
      HIPC(hipMemcpyAsync(ck_x + (size_t)q * nnz, xcur, (size_t)nnz * sizeof(float),
                          hipMemcpyDeviceToDevice, st));
      HIPC(hipMemcpyAsync(ck_p + (size_t)q * m, pw, (size_t)m * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
      HIPC(hipMemcpyAsync(ck_c + (size_t)q * m, c, (size_t)m * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
      HIPC(hipMemcpyAsync(ck_cp + (size_t)q * m, cp, (size_t)m * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
    }
    if (j == jlast) break;
    float *xnext = (j % 2 == 0) ? xa : xb;
    int32_t rc = forward(xcur, xnext);
    if (rc != PDHCG_OK) return rc;
    xcur = xnext;
  }

  // reverse sweep, one segment at a time (recomputed from its checkpoint)
  HIPC(launch_zero_f32(R0, nnz, st));
  HIPC(launch_zero_f32(duh, nnz, st));
  HIPC(launch_zero_f32(dw, n, st));
  HIPC(launch_zero_f64(B, m, st));
  HIPC(launch_zero_f64(Cn, m, st));
  HIPC(launch_gather_f32_to_f64(dL_dp, mk->perm, P, m, st));
  float *rin = R0, *rout = R1;
  for (int q = nck - 1; q >= 0; --q) {
    const int j0 = q * L, j1 = std::min(K, j0 + L);
    HIPC(hipMemcpyAsync(pw, ck_p + (size_t)q * m, (size_t)m * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    HIPC(hipMemcpyAsync(c, ck_c + (size_t)q * m, (size_t)m * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    HIPC(hipMemcpyAsync(cp, ck_cp + (size_t)q * m, (size_t)m * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    const float *xin = ck_x + (size_t)q * nnz;
    for (int j = j0; j < j1; ++j) {
      float *xo = seg_x + (size_t)(j - j0) * nnz;  // x^{j+1}
      int32_t rc = forward(xin, xo);
      if (rc != PDHCG_OK) return rc;
      xin = xo;
    }
    for (int j = j1 - 1; j >= j0; --j) {
      AdjIO aio;
      aio.xn = seg_x + (size_t)(j - j0) * nnz;
      aio.r_in = rin;
      aio.b = B;
      aio.r_out = rout;
      aio.duh = duh;
      aio.dw = dw;
      aio.csum = asum;
      aio.tau = tau;
      const int h = lds_goods(mk);
      if (h < m) HIPC(launch_zero_f64(asum, m, st));
      for (const Bin &b : mk->bins)
        HIPC(launch_adj_row(md, mk->bindev(b), b.G, b.E, mk->lds_row, aio, b.nwg, st));
      HIPC(launch_sum_partials(mk->colpart, mk->total_wg, h, m, chunk, st));
      HIPC(launch_adj_col(chunk, asum, h, P, B, Cn, tau, sigma, m, st));
      std::swap(rin, rout);
    }
  }
  HIPC(launch_adj_unnormalize(mk->row_ptr, mk->uh, mk->rowmax, duh, n, dL_du, st));
  HIPC(hipMemcpyAsync(dL_dw, dw, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPC(hipStreamSynchronize(st));  // the buffers above are freed or reused after return
  return PDHCG_OK;
}

int32_t check_backward_args(pdhcg_market mk, const float *x, const float *p, double omega,
                            int32_t unroll, int32_t ckpt_every, const float *dL_dp,
                            const float *dL_du, const float *dL_dw) {
  if (!mk || !x || !p || !dL_dp || !dL_du || !dL_dw) return fail(PDHCG_ERR_ARG, "null argument");
  if (!(omega > 0.0) || !std::isfinite(omega))
    return fail(PDHCG_ERR_ARG, "omega must be finite and > 0");
  if (unroll < 1 || ckpt_every < 1) return fail(PDHCG_ERR_ARG, "unroll and ckpt_every must be >= 1");
  return PDHCG_OK;
}

constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// Workspace of pdhcg_backward_noalloc: a fixed array in every GPU's memory,
// held until the process ends.  In host code this name is only a stand-in
// for the symbol: the device address comes from hipGetSymbolAddress, once
// per device, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up on the first call for
// that device (with it current) and cached.
int32_t scratch_address(int device, char **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(PDHCG_ERR_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIPC(hipGetDevice(&cur));
    if (cur != device) HIPC(hipSetDevice(device));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) HIPC(hipSetDevice(cur));
    if (e != hipSuccess)
      return fail(PDHCG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    if (!ptr) return fail(PDHCG_ERR_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_ptr[device] = ptr;
  }
  *out = static_cast<char *>(g_scratch_ptr[device]);
  return PDHCG_OK;
}

}  // namespace

extern "C" int32_t pdhcg_backward(pdhcg_market mk, const float *x, const float *p, double omega,
                                  int32_t unroll, int32_t ckpt_every, const float *dL_dp,
                                  float *dL_du, float *dL_dw) {
  int32_t rc = check_backward_args(mk, x, p, omega, unroll, ckpt_every, dL_dp, dL_du, dL_dw);
  if (rc != PDHCG_OK) return rc;
  AdjBuffers buf;
  return backward_impl(mk, x, p, omega, unroll, ckpt_every, dL_dp, dL_du, dL_dw, buf);
}

extern "C" int32_t pdhcg_backward_noalloc(pdhcg_market mk, const float *x, const float *p,
                                          double omega, int32_t unroll, int32_t ckpt_every,
                                          const float *dL_dp, float *dL_du, float *dL_dw) {
  int32_t rc = check_backward_args(mk, x, p, omega, unroll, ckpt_every, dL_dp, dL_du, dL_dw);
  if (rc != PDHCG_OK) return rc;
  const int L = std::min(ckpt_every, unroll);
  const size_t need = backward_bytes(mk->nnz, mk->n, mk->m, unroll, L);
  if (need > kNoAllocBytes)
    return fail(PDHCG_ERR_UNSUPPORTED,
                "pdhcg_backward_noalloc needs " + std::to_string(need) + " bytes of workspace for "
                "this market and unroll/ckpt_every; its fixed workspace holds " +
                std::to_string(kNoAllocBytes) + " bytes (use pdhcg_backward)");
  ArenaBuffers buf;
  rc = scratch_address(mk->device, &buf.base);
  if (rc != PDHCG_OK) return rc;
  buf.cap = kNoAllocBytes;
  return backward_impl(mk, x, p, omega, unroll, ckpt_every, dL_dp, dL_du, dL_dw, buf);
}
