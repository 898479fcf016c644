// C ABI of the sweep library: validation, context and workspace, and the
// host orchestration of the kernels in kp_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <functional>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/kp.h"
#include "kp_internal.h"

// launchers (kp_kernels.hip)
size_t kp_sweep_lds_bytes(int U, int M, int K, bool scd, int fmt, bool hist = true);
hipError_t kp_launch_sweep(const SweepArgs &a, int U, int grid, bool scd, hipStream_t stream,
                           int *used);
int kp_sweep_resident_grid(int U, int M, int K, bool scd, int fmt, bool hist = true);
int kp_sweep_batched_resident(size_t lds);
hipError_t kp_launch_reduce_stats(const double *partials, int nblk, int K, const double *lam,
                                  const double *B, double *R, double *g, double *P,
                                  hipStream_t stream);
hipError_t kp_launch_scd_init(KState *st, int K, const double *lam_in, const uint8_t *kmask,
                              double *hist, int hinted, int window, int interp, hipStream_t stream);
hipError_t kp_launch_scd_locate_select(KState *st, int K, const double *B, const double *R,
                                       const int *rinst, XSum *hist_sum, uint32_t *hist_cnt,
                                       const double *ev1, const double *ev2, uint32_t emit_cap,
                                       int *pending, unsigned int *win, hipStream_t stream);
hipError_t kp_launch_scd_finish(const KState *st, int K, const double *lam_in, double *lam_out,
                                double *delta_next, hipStream_t stream);
hipError_t kp_launch_dd_update(int K, double alpha, const double *R, const double *B, double *lam,
                               hipStream_t stream);
hipError_t kp_launch_gather_dense(const float *p, const float *b, const int64_t *users, int64_t n, int M,
                                  int K, float *sp, float *sb, hipStream_t stream);
hipError_t kp_launch_gather_csr_ptr(const int64_t *rowptr, const int64_t *users, int64_t n, int M,
                                    int64_t *len, int64_t *subptr, hipStream_t stream);
hipError_t kp_launch_gather_csr(const int64_t *rowptr, const int32_t *col, const float *val,
                                const int64_t *users, int64_t n, int M, const int64_t *subptr,
                                int32_t *scol, float *sval, hipStream_t stream);
hipError_t kp_launch_dual_backward(int K, const double *R, const double *B, const double *gout,
                                   double *glam, hipStream_t stream);
hipError_t kp_launch_validate(const float *v, int64_t n, unsigned int *flags, hipStream_t stream);
hipError_t kp_launch_fixup_pipeline(ProbDev pr, int row_d, uint8_t *x, const double *lam, const int *kv,
                                    const int *vk, const double *Bv, int nv, int nb, const double *R,
                                    const double *P,
                                    double *R_out, double *P_out, int64_t *n_reset, void *scratch,
                                    hipStream_t stream, uint32_t *pinned, int persist,
                                    const std::function<hipError_t(const FixBins &)> &bins_pass);
int kp_fixup_bins(int nv, size_t budget);
size_t kp_fixup_scratch_bytes(int64_t N, int nv, int K);
size_t kp_ell_lds_bytes(int M, int K, int D, int L, int mode, int *region_out);
hipError_t kp_launch_ell(const SweepArgs &a, int D, int grid, int mode, hipStream_t stream, int *used);
int kp_ell_resident_grid(int D, int mode, int M, int K, int L);
hipError_t kp_launch_dense(const SweepArgs &a, int grid, hipStream_t stream, int *used, bool win);
int kp_dense_tile_users();
int kp_dense_resident_grid(int M, int K, int L, bool win);
hipError_t kp_launch_count_modes(const KState *st, int K, int *out, hipStream_t stream);
hipError_t kp_launch_dense_probe(const SweepArgs &a, int *out, hipStream_t stream);
hipError_t kp_launch_ell_check(const int64_t *rowptr, int64_t nrows, int D, unsigned int *bad,
                               hipStream_t stream);
hipError_t kp_launch_sweep_batched(const SweepArgs *descs, const TileGeom *geoms,
                                   const int *block_off, int n_inst, int total_blocks, size_t lds,
                                   hipStream_t stream, const int *n_dev = nullptr);
hipError_t kp_launch_inst_active(const KState *st, const int *koff, int n, int *flags, hipStream_t stream);
size_t kp_resplit_lds(int n);
hipError_t kp_launch_plan_resplit(const ResplitArgs &r, hipStream_t stream);
hipError_t kp_launch_batched_aux(int which, const void *tab, int n, KState *st, const void *lam_ptrs,
                                 const int *kinst, const int *klocal, double *hint, const uint64_t *eoff,
                                 const uint32_t *ecap, hipStream_t stream);
TileGeom kp_tile_geom(const SweepArgs &a, int U);
size_t kp_coldesc_size();
void kp_coldesc_fill(void *dst, const double *partials, const double *lam, const double *B,
                     double *out, int nblk, int K, int col);

hipError_t kp_launch_validate_csr(const int64_t *rowptr, const int32_t *col, int64_t nrows, int K,
                                  unsigned int *flags, hipStream_t stream);
hipError_t kp_launch_fill_f64(double *dst, int64_t n, double v, hipStream_t stream);
hipError_t kp_launch_recenter(KState *st, int K, const double *lam_hat, const double *lam_in, int window,
                              hipStream_t stream);
hipError_t kp_launch_strided_users(int64_t *users, int64_t n, int64_t stride, int64_t off, hipStream_t stream);
hipError_t kp_launch_uniform_rowptr(int64_t *rowptr, int64_t nrows, int D, hipStream_t stream);
hipError_t kp_launch_stream_read(const void *src, int64_t n16, unsigned long long *out, int grid,
                                 hipStream_t stream);

namespace {

// last error message of this thread (a fixed buffer: reporting an error
// allocates nothing)
thread_local char g_err[512];

kp_status fail(kp_status st, const char *fmt, ...) {
  char buf[sizeof g_err];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  memcpy(g_err, buf, sizeof g_err);
  return st;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(KP_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

constexpr int kTileBudget = 24 * 1024;   // bytes of staged costs per tile
constexpr int kTileRowsMin = 160;        // item rows per tile at least, when the rows are long
constexpr size_t kMaxLds = 160 * 1024;   // LDS per workgroup on gfx950
constexpr int kMaxGrid = 2048;
constexpr uint32_t kEmitCapDefault = 1u << 20;
constexpr int kMaxPasses = 96;
constexpr uint32_t kStageCap = 4096;    // staged events per block per pass (at least)
constexpr uint32_t kStageCapMax = 65536;
constexpr int kGraphLaterPasses = 5;     // later passes captured with the first in a batched iteration's graph
constexpr uint32_t kEmitCapBatched = 1u << 16;   // emitted events per (instance, knapsack) per pass (at least)
constexpr double kEmitBytesBatched = 8.0e9;        // bound on a batch's emission buffers
constexpr size_t kBatchedLds = 40 * 1024;          // LDS per block of the batched launch (4 blocks per CU)
constexpr int kMaxInputNodes = 4096;               // local-constraint nodes accepted in a problem

struct Ctx {
  hipStream_t stream = nullptr;
  size_t max_ws = 0;
  void *ws = nullptr;
  size_t ws_cap = 0;
  int *pinned = nullptr;          // host-visible status word
  // central-window hint for the next SCD call (performance only)
  double *delta_dev = nullptr;
  int delta_K = 0;
  bool delta_valid = false;
  // optional timing of the sweep kernel launches (HIP events on the stream)
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
  std::vector<hipEvent_t> ev_free;
  double sweep_ms = 0.0;
  int64_t sweep_launches = 0;
  double sweep_bytes = 0.0;
  int64_t batched_passes = 0;     // sweep passes of the timed batched iterations
  // tuned tile sizes per shape (M, K, format) -> (users per tile, grid)
  std::map<std::tuple<int, int, int>, std::pair<int, int>> tuning;
  bool ell_enabled = true;
  bool window_enabled = true;
  bool alg5 = false;      // Alg.5 map for the users in its setting
  bool interp = false;    // approximate reduce: interpolation inside the threshold's bucket
  // full searches of problems with at least this many users start from the
  // threshold of a strided sample (0: never); the sample's search runs on a
  // child context (no windows, no sampling) in a buffer of this context
  int64_t sample_min = (int64_t)1 << 22;
  struct Ctx *child = nullptr;
  void *sbuf = nullptr;
  size_t sbuf_cap = 0;
  int stats_grid = 0;     // blocks of the last sweep launch (slots of the per-block partials)
  // shape of the last sweep launch: kernel (0 general, 1 uniform-row), users
  // per tile, blocks
  int last_kernel = -1, last_U = 0, last_grid = 0;
  // batched plans created later: LDS per block and blocks per resident block
  // (0: built-in)
  int bt_lds = 0, bt_mult = 0;
  std::map<std::tuple<int, int, int, int>, std::pair<int, int>> ell_grids;  // (D, M, K, L) -> resident grids
  std::map<std::tuple<int, int, int>, int> dense_grids;                     // (M, K, L) -> resident grid
  int64_t win_tried = 0, win_above = 0, win_below = 0;   // window searches since creation
  int64_t win_emitted = 0;                                 // breakpoints emitted inside windows
  int64_t win_listed = 0;                                  // users listed by split window passes
  // budgets on the device (uploaded again only when they change)
  double *B_dev = nullptr;
  int B_cap = 0;
  std::vector<double> B_host;
};

hipEvent_t take_event(Ctx *c) {
  if (!c->ev_free.empty()) {
    hipEvent_t e = c->ev_free.back();
    c->ev_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Resolve finished event pairs into the running totals.
void drain_events(Ctx *c, bool wait) {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> keep;
  for (auto &pr : c->ev_pending) {
    if (wait) (void)hipEventSynchronize(pr.second);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      c->sweep_ms += ms;
      c->ev_free.push_back(pr.first);
      c->ev_free.push_back(pr.second);
    } else {
      keep.push_back(pr);
    }
  }
  c->ev_pending.swap(keep);
}

// Workspace carve: every block 256-byte aligned.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  }
};

kp_status ensure_ws(Ctx *c, size_t bytes) {
  if (!c->pinned) {
    if (hipHostMalloc((void **)&c->pinned, 256, hipHostMallocDefault) != hipSuccess) {
      c->pinned = nullptr;
      return fail(KP_ERR_HIP, "hipHostMalloc of the status word failed");
    }
  }
  if (bytes <= c->ws_cap) return KP_OK;
  if (c->max_ws && bytes > c->max_ws)
    return fail(KP_ERR_NOMEM, "workspace of %zu bytes exceeds the context cap of %zu bytes", bytes,
                c->max_ws);
  if (c->ws) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_cap = 0;
  }
  size_t want = std::max(bytes, (size_t)1 << 20);
  if (c->max_ws) want = std::min(want, c->max_ws);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    c->ws = nullptr;
    return fail(KP_ERR_NOMEM, "hipMalloc of %zu workspace bytes failed", want);
  }
  c->ws_cap = want;
  return KP_OK;
}

// ---- problem validation and tree preparation ----
struct Prepared {
  ProbDev pr;
  TreeDev tree;
  const double *B = nullptr;   // the caller's host budgets [K] (valid during the call)
  int U = 1;
  int64_t ntiles = 0;
  int grid = 1;
  // SCD passes in which no knapsack bins events (every search starts with a
  // window): tiles and grid of the general kernel without the histograms
  int U_nh = 1;
  int64_t ntiles_nh = 0;
  int grid_nh = 1;
  double bytes = 0.0;   // algorithmic input bytes of one sweep launch
  int row_nnz = 0;        // declared entries per CSR item row (0: general rows)
  // uniform-row CSR kernel (0 = not used)
  int ell_D = 0;
  int64_t ell_ntiles = 0;
  int ell_grid = 0;
  int ell_brk_grid = 0;   // smallest grid of the lean kernel's breakpoint launches
  // lane-per-user evaluation of dense costs (0 = not used)
  int dense_grid = 0;
  int64_t dense_ntiles = 0;
  // its SCD window pass (0 = not used)
  int dwin_grid = 0;
  double ell_bytes = 0.0;
  int stage_grid() const {
    return std::max(std::max(std::max(grid, grid_nh), std::max(ell_grid, dense_grid)), dwin_grid);
  }
};

kp_status prepare(const kp_problem *p, bool scd, Prepared &out, const Ctx *ctx = nullptr) {
  if (!p) return fail(KP_ERR_INVALID, "problem is NULL");
  if (p->N < 0) return fail(KP_ERR_INVALID, "N must be >= 0 (got %lld)", (long long)p->N);
  if (p->M < 1) return fail(KP_ERR_INVALID, "M must be >= 1 (got %d)", p->M);
  if (p->M > KP_MAX_M) return fail(KP_ERR_UNSUPPORTED, "M = %d exceeds the built limit %d", p->M, KP_MAX_M);
  if (p->K < 1) return fail(KP_ERR_INVALID, "K must be >= 1 (got %d)", p->K);
  if (scd && p->K > KP_MAX_K_SCD)
    return fail(KP_ERR_UNSUPPORTED, "K = %d exceeds the SCD limit %d", p->K, KP_MAX_K_SCD);
  if (p->b_format != KP_B_DENSE && p->b_format != KP_B_CSR)
    return fail(KP_ERR_INVALID, "b_format must be KP_B_DENSE or KP_B_CSR");
  if (p->b_row_nnz != 0 && (p->b_format != KP_B_CSR || (p->b_row_nnz != 1 && p->b_row_nnz != 2)))
    return fail(KP_ERR_INVALID, "b_row_nnz must be 0, or 1 or 2 with CSR costs (got %d)", p->b_row_nnz);
  out.row_nnz = p->b_row_nnz;
  if (p->N > 0) {
    if (!p->p) return fail(KP_ERR_INVALID, "p is NULL");
    if (p->b_format == KP_B_DENSE && !p->b) return fail(KP_ERR_INVALID, "b is NULL");
    if (p->b_format == KP_B_CSR && (!p->b_rowptr || !p->b_col || !p->b_val))
      return fail(KP_ERR_INVALID, "CSR arrays must not be NULL");
  }
  if (!p->B) return fail(KP_ERR_INVALID, "B is NULL");
  out.B = p->B;
  for (int k = 0; k < p->K; ++k)
    if (!(std::isfinite(out.B[k]) && out.B[k] > 0.0))
      return fail(KP_ERR_INVALID, "B[%d] = %g must be finite and > 0", k, out.B[k]);
  const int L = p->L, M = p->M;
  if (L < 0) return fail(KP_ERR_INVALID, "L must be >= 0");
  if (L > 0 && (!p->parent || !p->cap)) return fail(KP_ERR_INVALID, "parent/cap is NULL");
  if (!p->leaf_of_item) return fail(KP_ERR_INVALID, "leaf_of_item is NULL");
  for (int l = 0; l < L; ++l) {
    if (p->cap[l] < 1) return fail(KP_ERR_INVALID, "cap[%d] = %d must be >= 1", l, p->cap[l]);
    if (p->parent[l] < -1 || p->parent[l] >= L || p->parent[l] == l)
      return fail(KP_ERR_INVALID, "parent[%d] = %d out of range", l, p->parent[l]);
  }
  // acyclic: every chain reaches a root within L steps
  for (int l = 0; l < L; ++l) {
    int x = l, steps = 0;
    while (x >= 0 && steps <= L) { x = p->parent[x]; ++steps; }
    if (x >= 0) return fail(KP_ERR_INVALID, "parent links contain a cycle (node %d)", l);
  }
  if (L > kMaxInputNodes)
    return fail(KP_ERR_UNSUPPORTED, "L = %d local-constraint nodes exceed the limit %d", L, kMaxInputNodes);
  // (fixed-size arrays: validation allocates nothing)
  uint64_t mask[kMaxInputNodes];
  for (int l = 0; l < L; ++l) mask[l] = 0;
  for (int j = 0; j < M; ++j) {
    const int lf = p->leaf_of_item[j];
    if (lf < -1 || lf >= L) return fail(KP_ERR_INVALID, "leaf_of_item[%d] = %d out of range", j, lf);
    for (int x = lf; x >= 0; x = p->parent[x]) mask[x] |= 1ull << j;
  }
  // keep sets that can bind; merge duplicates with the smaller cap
  uint64_t nmask[KP_MAX_NODES];
  int ncap[KP_MAX_NODES];
  int nn = 0;
  for (int l = 0; l < L; ++l) {
    const int sz = __builtin_popcountll(mask[l]);
    if (p->cap[l] >= sz) continue;
    int t = 0;
    while (t < nn && nmask[t] != mask[l]) ++t;
    if (t < nn) {
      ncap[t] = std::min(ncap[t], p->cap[l]);
      continue;
    }
    if (nn == KP_MAX_NODES)
      return fail(KP_ERR_UNSUPPORTED, "more than %d binding local sets", KP_MAX_NODES);
    nmask[nn] = mask[l];
    ncap[nn] = p->cap[l];
    ++nn;
  }
  // subsets first: size ascending, then lowest item (insertion sort, stable)
  auto before = [](uint64_t a, uint64_t b) {
    const int sa = __builtin_popcountll(a), sb = __builtin_popcountll(b);
    if (sa != sb) return sa < sb;
    return __builtin_ctzll(a) < __builtin_ctzll(b);
  };
  for (int a = 1; a < nn; ++a) {
    const uint64_t m = nmask[a];
    const int cp = ncap[a];
    int b = a - 1;
    while (b >= 0 && before(m, nmask[b])) { nmask[b + 1] = nmask[b]; ncap[b + 1] = ncap[b]; --b; }
    nmask[b + 1] = m;
    ncap[b + 1] = cp;
  }
  memset(&out.tree, 0, sizeof(out.tree));
  out.tree.L = nn;
  for (int t = 0; t < nn; ++t) {
    out.tree.mask[t] = nmask[t];
    out.tree.cap[t] = ncap[t];
  }
  ProbDev &pr = out.pr;
  memset(&pr, 0, sizeof(pr));
  pr.N = p->N;
  pr.M = M;
  pr.K = p->K;
  pr.fmt = p->b_format;
  pr.p = p->p;
  pr.b = p->b;
  pr.rowptr = p->b_rowptr;
  pr.col = p->b_col;
  pr.val = p->b_val;
  // tile: as many users as fit the staged-cost budget, at most 64
  const size_t per_user = (size_t)M * p->K * 4;
  int U = (int)std::max<size_t>(1, std::min<size_t>(64, kTileBudget / per_user));
  U = std::min(U, std::max(1, 1024 / M));   // rows per tile <= the prefetched rows
  // long rows (large K): enough rows to keep the block's threads busy
  U = std::max(U, std::min((kTileRowsMin + M - 1) / M, std::max(1, 1024 / M)));
  // dense tiles start 16-byte aligned when U*M*K is a multiple of 4
  if (U >= 4 && (M * p->K) % 4 != 0) U &= ~3;
  int grid_override = 0;
  if (ctx) {
    auto it = ctx->tuning.find(std::make_tuple(M, p->K, p->b_format));
    if (it != ctx->tuning.end()) {
      if (it->second.first > 0) U = std::min(it->second.first, std::max(1, 1024 / M));
      grid_override = it->second.second;
    }
  }
  const int U0 = U;
  while (U > 1 && kp_sweep_lds_bytes(U, M, p->K, scd, p->b_format) > 64 * 1024) --U;
  if (kp_sweep_lds_bytes(U, M, p->K, scd, p->b_format) > kMaxLds)
    return fail(KP_ERR_UNSUPPORTED, "M*K = %d too large for one tile", M * p->K);
  out.U = U;
  out.ntiles = (p->N + U - 1) / U;
  {
    const double Nd = (double)p->N;
    if (p->b_format == KP_B_DENSE) {
      out.bytes = Nd * M * 4.0 + Nd * M * (double)p->K * 4.0;
    } else {
      // p and rowptr here; the stored entries (col + val) are added by the
      // timed launch, which reads the entry count from rowptr[N*M]
      out.bytes = Nd * M * 4.0 + (Nd * M + 1) * 8.0;
    }
  }
  out.grid = (int)std::max<int64_t>(1, std::min<int64_t>(out.ntiles, grid_override > 0 ? grid_override : kMaxGrid));
  // persistent launch: no more blocks than can be resident at once
  if (p->N > 0) {
    const int res = kp_sweep_resident_grid(U, M, p->K, scd, p->b_format);
    if (res > 0) out.grid = std::min(out.grid, res);
  }
  out.U_nh = out.U;
  out.ntiles_nh = out.ntiles;
  out.grid_nh = out.grid;
  if (scd && p->N > 0) {
    // without the K x 64 histogram bins a tile can hold more users, and more
    // blocks fit on a compute unit
    int Un = U0;
    while (Un > 1 && kp_sweep_lds_bytes(Un, M, p->K, true, p->b_format, false) > 64 * 1024) --Un;
    const int64_t nt = (p->N + Un - 1) / Un;
    int g = (int)std::max<int64_t>(1, std::min<int64_t>(nt, grid_override > 0 ? grid_override : kMaxGrid));
    const int res = kp_sweep_resident_grid(Un, M, p->K, true, p->b_format, false);
    if (res > 0) g = std::min(g, res);
    out.U_nh = Un;
    out.ntiles_nh = nt;
    out.grid_nh = g;
  }
  return KP_OK;
}

constexpr int kEllGrid = 1024;

// Decide whether the uniform-row CSR kernel applies: CSR declared with D in
// {1, 2} entries per item row at r*D (b_row_nnz), M <= 16, and its LDS fits.
kp_status choose_kernel(Ctx *c, Prepared &P, bool scd) {
  P.ell_D = 0;
  P.ell_grid = 0;
  P.dense_grid = 0;
  P.dense_ntiles = 0;
  P.dwin_grid = 0;
  if (c->ell_enabled && P.pr.fmt == KP_B_DENSE && P.pr.M <= 16 && P.pr.K <= 16 && P.pr.N > 0) {
    // dense costs with few items and knapsacks: the lane-per-user
    // evaluation (SCD: its window pass; the other passes run the general
    // kernel), unless a tile size was asked for this shape (the general
    // kernel's); a grid-only override sets its grid
    auto tit = c->tuning.find(std::make_tuple((int)P.pr.M, (int)P.pr.K, (int)KP_B_DENSE));
    const bool tiles = tit != c->tuning.end() && tit->second.first > 0;
    if (!tiles) {
      const auto key = std::make_tuple((int)P.pr.M, (int)P.pr.K, (int)P.tree.L * 2 + (scd ? 1 : 0));
      auto it = c->dense_grids.find(key);
      int res = 0;
      if (it != c->dense_grids.end()) {
        res = it->second;
      } else {
        res = kp_dense_resident_grid(P.pr.M, P.pr.K, P.tree.L, scd);
        if (res <= 0) return fail(KP_ERR_HIP, "occupancy query failed");
        c->dense_grids[key] = res;
      }
      const int tu = kp_dense_tile_users();
      P.dense_ntiles = (P.pr.N + tu - 1) / tu;
      int g = (int)std::min<int64_t>(P.dense_ntiles, res);
      if (tit != c->tuning.end() && tit->second.second > 0) g = std::min(tit->second.second, res);
      (scd ? P.dwin_grid : P.dense_grid) = std::max(1, g);
    }
    return KP_OK;
  }
  if (!c->ell_enabled || P.pr.fmt != KP_B_CSR || P.pr.M > 16 || P.pr.N == 0 || P.row_nnz == 0) return KP_OK;
  const int D = P.row_nnz;
  const int64_t nnz = P.pr.N * P.pr.M * (int64_t)D;
  if (kp_ell_lds_bytes(P.pr.M, P.pr.K, D, P.tree.L, scd ? 1 : 0, nullptr) > kMaxLds) return KP_OK;
  P.ell_D = D;
  P.ell_ntiles = (P.pr.N + 63) / 64;
  // per-block buffers for the largest resident grid of the lean kernel's
  // modes; the staging of emitted events is sized for the smallest grid of
  // its breakpoint modes (those blocks each take a larger share of the users)
  int gmax = 0, gbrk = 0;
  const auto gkey = std::make_tuple(D, (int)P.pr.M, (int)P.pr.K, (int)P.tree.L);
  auto git = c->ell_grids.find(gkey);
  if (git != c->ell_grids.end()) {
    gmax = git->second.first;
    gbrk = git->second.second;
  } else {
    for (int mode = 0; mode < 4; ++mode) {
      const int r = kp_ell_resident_grid(D, mode, P.pr.M, P.pr.K, P.tree.L);
      if (r <= 0) return fail(KP_ERR_HIP, "occupancy query failed");
      gmax = std::max(gmax, r);
      if (mode == 1 || mode == 3) gbrk = gbrk ? std::min(gbrk, r) : r;
    }
    c->ell_grids[gkey] = std::make_pair(gmax, gbrk);
  }
  P.ell_grid = (int)std::max<int64_t>(1, std::min<int64_t>((P.ell_ntiles + 3) / 4, std::min(gmax, kEllGrid)));
  // a tuned grid for this shape (the kernel's users per tile are fixed: one
  // lane per user, 64 per wave); never above what can be resident
  auto tit = c->tuning.find(std::make_tuple((int)P.pr.M, (int)P.pr.K, (int)KP_B_CSR));
  if (tit != c->tuning.end() && tit->second.second > 0)
    P.ell_grid = std::max(1, std::min(tit->second.second, gmax));
  P.ell_brk_grid = std::max(1, std::min(gbrk, P.ell_grid));
  // the ABI layout's bytes (p, col, val and rowptr), although the kernel never reads rowptr
  P.ell_bytes = (double)P.pr.N * P.pr.M * 4.0 + (double)nnz * 8.0 + ((double)P.pr.N * P.pr.M + 1.0) * 8.0;
  return KP_OK;
}

// Does every one of the nrows item rows hold exactly D in {1, 2} entries at
// r*D?  *D_out = D, or 0.  Reads rowptr[nrows] and then (when the count fits)
// every offset on the device; synchronous.
kp_status check_rows(Ctx *c, const int64_t *rowptr, int64_t nrows, unsigned int *D_out) {
  *D_out = 0;
  if (!c->pinned) {
    if (hipHostMalloc((void **)&c->pinned, 256, hipHostMallocDefault) != hipSuccess) {
      c->pinned = nullptr;
      return fail(KP_ERR_HIP, "hipHostMalloc failed");
    }
  }
  int64_t *h = (int64_t *)(c->pinned + 8);
  HIP_TRY(hipMemcpyAsync(h, rowptr + nrows, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const int64_t nnz = *h;
  if (!(nnz > 0 && nnz % nrows == 0 && nnz / nrows <= 2)) return KP_OK;
  const int Dc = (int)(nnz / nrows);
  Carve cv;
  const size_t ob = cv.take(16);
  kp_status s = ensure_ws(c, std::max(cv.off, c->ws_cap));
  if (s != KP_OK) return s;
  unsigned int *bad = (unsigned int *)((char *)c->ws + ob);
  HIP_TRY(hipMemsetAsync(bad, 0, 4, c->stream));
  HIP_TRY(kp_launch_ell_check(rowptr, nrows, Dc, bad, c->stream));
  HIP_TRY(hipMemcpyAsync(c->pinned + 12, bad, 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (c->pinned[12] == 0) *D_out = (unsigned int)Dc;
  return KP_OK;
}

struct SweepWs {
  double *partials, *B, *ev1, *ev2, *Rtmp, *gtmp, *Ptmp, *sv1, *sv2;
  XSum *hist_sum;
  uint16_t *sk;
  uint32_t stage_cap;
  uint32_t *hist_cnt;
  KState *st;
  uint8_t *kmask;
  unsigned long long *err;
  int *pending;
  unsigned int *win;    // window searches: [0] tried, [1] threshold above, [2] below
  uint32_t emit_cap;
  unsigned int *flist, *fcount;   // users listed by the window pass
  uint32_t fcap;
  int *modes;           // [0] knapsacks with a window, [1] with another search mode, [2] alternation
                        // windows, [3] dense probe: sampled users with a line above -H
  char *stat;           // status block, followed by the histograms (SCD)
  size_t stat_bytes;    // the status block and the histograms
};

kp_status carve_ws(Ctx *c, const Prepared &P, bool scd, SweepWs &w) {
  const int K = P.pr.K;
  Carve cv;
  size_t o_part = cv.take((size_t)P.stage_grid() * (K + 2) * 8);
  size_t o_B = cv.take((size_t)K * 8);
  size_t o_R = cv.take((size_t)K * 8);
  size_t o_g = cv.take(8);
  size_t o_P = cv.take(8);
  // status block (cleared with the histograms in one memset): [0] pending
  // knapsacks, [8] walk-limit counter, [16] window counters, [32] list
  // counters, [48] search-mode counts
  size_t o_st = 0, o_hs = 0, o_hc = 0, o_km = 0, o_e1 = 0, o_e2 = 0, o_stat = 0;
  uint32_t cap = 0;
  if (scd) o_st = cv.take((size_t)K * sizeof(KState));
  o_stat = cv.take(64);
  if (scd) {
    o_hs = cv.take((size_t)K * KP_NB * sizeof(XSum));
    o_hc = cv.take((size_t)K * KP_NB * 4);
    o_km = cv.take((size_t)K);
    cap = kEmitCapDefault;
    o_e1 = cv.take((size_t)K * cap * 8);
    o_e2 = cv.take((size_t)K * cap * 8);
  }
  size_t o_s1 = 0, o_s2 = 0, o_sk = 0;
  // staged events per block: scale with the block's share of (user, knapsack)
  // pairs so that large window passes do not overflow
  uint32_t scap = 0;
  if (scd) {
    // (sized for the general kernel's smaller grid, the one with histograms)
    const int blocks = P.ell_D ? P.ell_brk_grid : P.grid;
    const double share = (double)P.pr.N * K / std::max(1, blocks) / 64.0;
    scap = (uint32_t)std::min<double>(kStageCapMax, std::max<double>(kStageCap, share));
  }
  if (scd) {
    o_s1 = cv.take((size_t)P.stage_grid() * scap * 8);
    o_s2 = cv.take((size_t)P.stage_grid() * scap * 8);
    o_sk = cv.take((size_t)P.stage_grid() * scap * 2);
  }
  // users listed by a window pass of the uniform-row kernel (room for all)
  size_t o_fl = 0;
  uint32_t fcap = 0;
  if (scd && P.ell_D && P.pr.N < ((int64_t)1 << 32) - ((int64_t)1 << 28)) {
    // every user, plus the unused tails of the waves' reserved chunks
    fcap = (uint32_t)(P.pr.N + (int64_t)KP_LIST_CHUNK * P.ell_grid * 4);
    o_fl = cv.take((size_t)fcap * 4);
  }
  kp_status s = ensure_ws(c, cv.off);
  if (s != KP_OK) return s;
  char *b = (char *)c->ws;
  w.partials = (double *)(b + o_part);
  w.B = (double *)(b + o_B);
  w.Rtmp = (double *)(b + o_R);
  w.gtmp = (double *)(b + o_g);
  w.Ptmp = (double *)(b + o_P);
  w.stat = b + o_stat;
  w.stat_bytes = scd ? (o_hc + (size_t)K * KP_NB * 4) - o_stat : 64;
  w.pending = (int *)(b + o_stat);
  w.err = (unsigned long long *)(b + o_stat + 8);
  w.win = (unsigned int *)(b + o_stat + 16);
  w.st = scd ? (KState *)(b + o_st) : nullptr;
  w.hist_sum = scd ? (XSum *)(b + o_hs) : nullptr;
  w.hist_cnt = scd ? (uint32_t *)(b + o_hc) : nullptr;
  w.kmask = scd ? (uint8_t *)(b + o_km) : nullptr;
  w.ev1 = scd ? (double *)(b + o_e1) : nullptr;
  w.ev2 = scd ? (double *)(b + o_e2) : nullptr;
  w.emit_cap = cap;
  w.sv1 = scd ? (double *)(b + o_s1) : nullptr;
  w.sv2 = scd ? (double *)(b + o_s2) : nullptr;
  w.sk = scd ? (uint16_t *)(b + o_sk) : nullptr;
  w.stage_cap = scap;
  w.fcap = fcap;
  w.flist = fcap ? (unsigned int *)(b + o_fl) : nullptr;
  w.fcount = (unsigned int *)(b + o_stat + 32);
  w.modes = scd ? (int *)(b + o_stat + 48) : nullptr;
  return KP_OK;
}

// Budgets of the problem on the device, in a buffer of the context that
// keeps them between calls: copied only when they differ from the last copy.
kp_status upload_B(Ctx *c, const Prepared &P, SweepWs &w) {
  const int K = P.pr.K;
  if (!c->B_dev || c->B_cap < K) {
    if (c->B_dev) HIP_TRY(hipFree(c->B_dev));
    c->B_dev = nullptr;
    c->B_host.clear();
    HIP_TRY(hipMalloc(&c->B_dev, (size_t)K * 8));
    c->B_cap = K;
  }
  if (c->B_host.size() != (size_t)K || memcmp(c->B_host.data(), P.B, (size_t)K * 8) != 0) {
    c->B_host.assign(P.B, P.B + K);
    HIP_TRY(hipMemcpyAsync(c->B_dev, c->B_host.data(), (size_t)K * 8, hipMemcpyHostToDevice, c->stream));
  }
  w.B = c->B_dev;
  return KP_OK;
}

// Algorithmic bytes of one sweep launch: every input byte of p and b once.
double algo_bytes(const Prepared &P) {
  const double N = (double)P.pr.N, M = P.pr.M, K = P.pr.K;
  if (P.pr.fmt == KP_B_DENSE) return N * M * 4.0 + N * M * K * 4.0;
  return -1.0;  // CSR: filled in by the caller from rowptr[N*M]
}

// One sweep pass between timing events.  split: the window pass of the
// uniform-row kernel as two launches (all users, then the listed ones).
hipError_t timed_sweep(Ctx *c, const SweepArgs &a, const Prepared &P, bool scd, double bytes,
                       bool split = false, bool dwin = false) {
  // a.no_hist: the general kernel's tiles and grid without histograms
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing && P.ell_D) {
    bytes = P.ell_bytes;
  } else if (c->timing && P.pr.fmt == KP_B_CSR && P.pr.N > 0) {
    // stored entries (col + val, 8 bytes each): the count is declared, or
    // read from rowptr[N*M] (only while timing is on)
    const int64_t nrows = P.pr.N * P.pr.M;
    int64_t nnz = nrows * (int64_t)P.row_nnz;
    if (!P.row_nnz) {
      hipError_t e = hipMemcpyAsync(&nnz, P.pr.rowptr + nrows, 8, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return e;
    }
    bytes += (double)nnz * 8.0;
  }
  if (c->timing) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, c->stream);
  }
  hipError_t err;
  if (P.ell_D && split) {
    SweepArgs ae = a;
    ae.ntiles = P.ell_ntiles;
    // the list counters ([0] reserved slots, [1] listed users) were cleared
    // with the status block
    err = kp_launch_ell(ae, P.ell_D, P.ell_grid, 2, c->stream, &c->stats_grid);
    if (err == hipSuccess) {
      SweepArgs af = ae;
      af.want_stats = 0;
      af.x_out = nullptr;
      err = kp_launch_ell(af, P.ell_D, P.ell_grid, 3, c->stream, nullptr);
    }
  } else if (P.ell_D) {
    SweepArgs ae = a;
    ae.ntiles = P.ell_ntiles;
    err = kp_launch_ell(ae, P.ell_D, P.ell_grid, scd ? 1 : 0, c->stream, &c->stats_grid);
  } else if (P.dense_grid && !scd) {
    SweepArgs ae = a;
    ae.ntiles = P.dense_ntiles;
    err = kp_launch_dense(ae, P.dense_grid, c->stream, &c->stats_grid, false);
  } else if (dwin) {
    SweepArgs ae = a;
    ae.ntiles = P.dense_ntiles;
    err = kp_launch_dense(ae, P.dwin_grid, c->stream, &c->stats_grid, true);
  } else {
    err = a.no_hist ? kp_launch_sweep(a, P.U_nh, P.grid_nh, scd, c->stream, &c->stats_grid)
                    : kp_launch_sweep(a, P.U, P.grid, scd, c->stream, &c->stats_grid);
  }
  if (c->timing && e0 && e1) {
    (void)hipEventRecord(e1, c->stream);
    c->ev_pending.push_back({e0, e1});
    c->sweep_launches += 1;
    c->sweep_bytes += bytes;
    if (c->ev_pending.size() > 256) drain_events(c, true);
  }
  if (err == hipSuccess) {
    const bool dense = !P.ell_D && P.dense_grid && !scd;
    c->last_kernel = P.ell_D ? 1 : dense ? 2 : dwin ? 3 : 0;
    c->last_U = P.ell_D ? 64 : (dense || dwin) ? kp_dense_tile_users() : (a.no_hist ? P.U_nh : P.U);
    c->last_grid = c->stats_grid;
  }
  return err;
}

// Q of Alg.5's map for this problem (0: not in its setting or not asked
// for): the uniform-row kernel with one entry per item row, M = K and at most
// one binding set, which holds every item (no binding set: Q = M).  Whether a
// user's entries sit in its items' own knapsacks is checked per user.
int alg5_q(const Ctx *c, const Prepared &P) {
  if (!c->alg5 || P.ell_D != 1 || P.pr.M != P.pr.K) return 0;
  const uint64_t all = P.pr.M >= 64 ? ~0ull : ((1ull << P.pr.M) - 1);
  if (P.tree.L == 0) return P.pr.M;
  if (P.tree.L == 1 && P.tree.mask[0] == all) return P.tree.cap[0];
  return 0;
}

SweepArgs make_args(const Prepared &P, const double *lam, const SweepWs &w, uint8_t *x,
                    bool stats) {
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.pr = P.pr;
  a.tree = P.tree;
  a.lam = lam;
  a.ntiles = P.ntiles;
  a.want_stats = stats ? 1 : 0;
  a.partials = w.partials;
  a.x_out = x;
  a.st = w.st;
  a.hist_sum = w.hist_sum;
  a.hist_cnt = w.hist_cnt;
  a.emit_v1 = w.ev1;
  a.emit_v2 = w.ev2;
  a.emit_cap = w.emit_cap;
  a.stage_v1 = w.sv1;
  a.stage_v2 = w.sv2;
  a.stage_k = w.sk;
  a.stage_cap = w.stage_cap;
  a.err = w.err;
  a.flist = w.flist;
  a.fcount = w.fcount;
  a.fcap = w.fcap;
  return a;
}

kp_status kp_scd_sweep_masked_impl(Ctx *c, const kp_problem *prob, const double *lambda_in, double *lambda_out,
                                   const uint8_t *kmask, double *R, double *g, double *primal);

// Start the full searches of this sweep from a sample's thresholds: every
// stride-th user (n = max(N/64, min(N/2, 2^20)) of them) is gathered into
// the context's sample buffer, the same SCD search runs on that sample with
// every budget scaled by n/N on the child context, and each knapsack in full
// search mode centres its buckets on the sample's threshold.
kp_status sample_center(Ctx *c, const kp_problem *prob, const Prepared &P, const SweepWs &w,
                        const double *lambda_in, const uint8_t *kmask) {
  const int64_t N = P.pr.N;
  const int M = P.pr.M, K = P.pr.K;
  const int64_t n = std::max<int64_t>(N / 64, std::min<int64_t>(N / 2, (int64_t)1 << 20));
  if (n < 1 || n >= N) return KP_OK;
  const int64_t stride = N / n;
  const bool csr = P.pr.fmt == KP_B_CSR;
  const int D = P.row_nnz;
  Carve cv;
  const size_t o_u = cv.take((size_t)n * 8);
  const size_t o_p = cv.take((size_t)n * M * 4);
  const size_t o_b = csr ? 0 : cv.take((size_t)n * M * K * 4);
  const size_t o_len = (csr && !D) ? cv.take((size_t)n * M * 8) : 0;
  const size_t o_rp = csr ? cv.take((size_t)(n * M + 1) * 8) : 0;
  const size_t o_col = (csr && D) ? cv.take((size_t)n * M * D * 4) : 0;
  const size_t o_val = (csr && D) ? cv.take((size_t)n * M * D * 4) : 0;
  const size_t o_lam = cv.take((size_t)K * 8);
  int64_t nnz = n * M * (int64_t)D;
  size_t o_ent = 0;
  if (csr && !D) {
    // the sampled rows' lengths and offsets first, to size the entries
    if (cv.off > c->sbuf_cap) {
      if (c->sbuf) HIP_TRY(hipFree(c->sbuf));
      c->sbuf = nullptr;
      c->sbuf_cap = 0;
      if (hipMalloc(&c->sbuf, cv.off) != hipSuccess) { c->sbuf = nullptr; return fail(KP_ERR_NOMEM, "hipMalloc failed"); }
      c->sbuf_cap = cv.off;
    }
    char *b = (char *)c->sbuf;
    HIP_TRY(kp_launch_strided_users((int64_t *)(b + o_u), n, stride, stride / 2, c->stream));
    HIP_TRY(kp_launch_gather_csr_ptr(P.pr.rowptr, (int64_t *)(b + o_u), n, M, (int64_t *)(b + o_len),
                                     (int64_t *)(b + o_rp), c->stream));
    int64_t *h = (int64_t *)(c->pinned + 8);
    HIP_TRY(hipMemcpyAsync(h, (int64_t *)(b + o_rp) + n * M, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    nnz = *h;
    o_ent = cv.take((size_t)std::max<int64_t>(nnz, 1) * 8);
  }
  if (cv.off > c->sbuf_cap) {
    // (a grown buffer keeps nothing: the general-CSR offsets are rebuilt below)
    if (c->sbuf) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      HIP_TRY(hipFree(c->sbuf));
    }
    c->sbuf = nullptr;
    c->sbuf_cap = 0;
    if (hipMalloc(&c->sbuf, cv.off) != hipSuccess) { c->sbuf = nullptr; return fail(KP_ERR_NOMEM, "hipMalloc failed"); }
    c->sbuf_cap = cv.off;
  }
  char *b = (char *)c->sbuf;
  int64_t *users = (int64_t *)(b + o_u);
  HIP_TRY(kp_launch_strided_users(users, n, stride, stride / 2, c->stream));
  kp_problem sub = *prob;
  sub.N = n;
  sub.p = (const float *)(b + o_p);
  if (!csr) {
    sub.b = (const float *)(b + o_b);
    HIP_TRY(kp_launch_gather_dense(P.pr.p, P.pr.b, users, n, M, K, (float *)(b + o_p), (float *)(b + o_b),
                                   c->stream));
  } else if (D) {
    HIP_TRY(kp_launch_gather_dense(P.pr.p, nullptr, users, n, M, K, (float *)(b + o_p), nullptr, c->stream));
    // a user's entries are M * D consecutive values of col and val
    HIP_TRY(kp_launch_gather_dense((const float *)P.pr.col, nullptr, users, n, M * D, 1, (float *)(b + o_col),
                                   nullptr, c->stream));
    HIP_TRY(kp_launch_gather_dense(P.pr.val, nullptr, users, n, M * D, 1, (float *)(b + o_val), nullptr,
                                   c->stream));
    HIP_TRY(kp_launch_uniform_rowptr((int64_t *)(b + o_rp), n * M, D, c->stream));
    sub.b_rowptr = (const int64_t *)(b + o_rp);
    sub.b_col = (const int32_t *)(b + o_col);
    sub.b_val = (const float *)(b + o_val);
  } else {
    HIP_TRY(kp_launch_gather_dense(P.pr.p, nullptr, users, n, M, K, (float *)(b + o_p), nullptr, c->stream));
    int64_t *subptr = (int64_t *)(b + o_rp);
    HIP_TRY(kp_launch_gather_csr_ptr(P.pr.rowptr, users, n, M, (int64_t *)(b + o_len), subptr, c->stream));
    int32_t *scol = (int32_t *)(b + o_ent);
    float *sval = (float *)(b + o_ent + (size_t)std::max<int64_t>(nnz, 1) * 4);
    HIP_TRY(kp_launch_gather_csr(P.pr.rowptr, P.pr.col, P.pr.val, users, n, M, subptr, scol, sval, c->stream));
    sub.b_rowptr = subptr;
    sub.b_col = scol;
    sub.b_val = sval;
  }
  std::vector<double> Bs(K);
  const double scale = (double)n / (double)N;
  for (int k = 0; k < K; ++k) Bs[k] = P.B[k] * scale;
  sub.B = Bs.data();
  if (!c->child) {
    void *ch = nullptr;
    kp_status st = kp_create(&ch, c->stream, c->max_ws);
    if (st != KP_OK) return st;
    c->child = (Ctx *)ch;
  }
  Ctx *ch = c->child;
  ch->stream = c->stream;
  ch->window_enabled = false;
  ch->sample_min = 0;
  ch->ell_enabled = c->ell_enabled;
  ch->alg5 = c->alg5;
  ch->delta_valid = false;
  ch->B_host.clear();
  double *lam_hat = (double *)(b + o_lam);
  kp_status st = kp_scd_sweep_masked_impl(ch, &sub, lambda_in, lam_hat, kmask, nullptr, nullptr, nullptr);
  if (st != KP_OK) {
    char m[sizeof g_err];
    memcpy(m, g_err, sizeof m);
    return fail(st, "sample search: %s", m);
  }
  // with windows on, the full searches start with a window around the
  // sample's threshold
  HIP_TRY(kp_launch_recenter(w.st, K, lam_hat, lambda_in, (c->window_enabled && !c->interp) ? 1 : 0,
                             c->stream));
  return KP_OK;
}

kp_status eval_into(Ctx *c, const Prepared &P, const SweepWs &w, const double *lam, double *R,
                    double *g, double *primal, uint8_t *x) {
  if (P.pr.N == 0) {
    // nothing to sweep: R = 0, P = 0, g = lambda . B
    HIP_TRY(hipMemsetAsync(w.partials, 0, (size_t)(P.pr.K + 2) * 8, c->stream));
    HIP_TRY(kp_launch_reduce_stats(w.partials, 1, P.pr.K, lam, w.B, R, g, primal, c->stream));
    return KP_OK;
  }
  SweepArgs a = make_args(P, lam, w, x, true);
  HIP_TRY(timed_sweep(c, a, P, false, P.bytes));
  HIP_TRY(kp_launch_reduce_stats(w.partials, c->stats_grid, P.pr.K, lam, w.B, R, g,
                                 primal, c->stream));
  return KP_OK;
}

}  // namespace

// ---- scratch of the allocation-free entry point ----
// Device memory for kp_eval_dual_noalloc: the budgets and the per-block
// partial sums.  Every GPU the library runs on holds its own copy for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).
#define KP_NOALLOC_SCRATCH (8u << 20)
#define KP_MAX_DEVICES 64
static __device__ __align__(256) unsigned char scratch[KP_NOALLOC_SCRATCH];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[KP_MAX_DEVICES] = {};

// The scratch array's device address on the current device (looked up once
// per device, with that device current).
kp_status noalloc_scratch(void **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= KP_MAX_DEVICES) return fail(KP_ERR_UNSUPPORTED, "device %d above the limit %d", dev, KP_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(KP_ERR_HIP, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return KP_OK;
}
}  // namespace

// ===========================================================================
extern "C" {

const char *kp_last_error(void) { return g_err; }

int32_t kp_max_items(void) { return KP_MAX_M; }
int32_t kp_max_knapsacks_scd(void) { return KP_MAX_K_SCD; }

kp_status kp_create(void **ctx_out, void *hip_stream, size_t max_workspace_bytes) {
  if (!ctx_out) return fail(KP_ERR_INVALID, "ctx_out is NULL");
  Ctx *c = new Ctx();
  c->stream = (hipStream_t)hip_stream;
  c->max_ws = max_workspace_bytes;
  *ctx_out = c;   // device resources are allocated on first use
  return KP_OK;
}

kp_status kp_destroy(void *ctx) {
  if (!ctx) return KP_OK;
  Ctx *c = (Ctx *)ctx;
  if (c->ws || c->delta_dev || c->pinned) (void)hipStreamSynchronize(c->stream);
  drain_events(c, true);
  for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  if (c->delta_dev) (void)hipFree(c->delta_dev);
  if (c->B_dev) (void)hipFree(c->B_dev);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->sbuf) (void)hipFree(c->sbuf);
  if (c->child) (void)kp_destroy(c->child);
  delete c;
  return KP_OK;
}

kp_status kp_set_stream(void *ctx, void *hip_stream) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  ((Ctx *)ctx)->stream = (hipStream_t)hip_stream;
  ((Ctx *)ctx)->B_host.clear();   // the cached budgets were copied on the old stream
  return KP_OK;
}

kp_status kp_eval_dual(void *ctx, const kp_problem *prob, const double *lambda, double *R,
                       double *g, double *primal, uint8_t *x) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!lambda) return fail(KP_ERR_INVALID, "lambda is NULL");
  Ctx *c = (Ctx *)ctx;
  Prepared P;
  kp_status s = prepare(prob, false, P, c);
  if (s != KP_OK) return s;
  if ((s = choose_kernel(c, P, false)) != KP_OK) return s;
  SweepWs w;
  if ((s = carve_ws(c, P, false, w)) != KP_OK) return s;
  if ((s = upload_B(c, P, w)) != KP_OK) return s;
  return eval_into(c, P, w, lambda, R ? R : w.Rtmp, g ? g : w.gtmp, primal ? primal : w.Ptmp, x);
}

kp_status kp_dd_step(void *ctx, const kp_problem *prob, double alpha, double *lambda_inout,
                     double *R, double *g, double *primal) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!lambda_inout) return fail(KP_ERR_INVALID, "lambda is NULL");
  if (!std::isfinite(alpha) || alpha < 0) return fail(KP_ERR_INVALID, "alpha must be finite and >= 0");
  Ctx *c = (Ctx *)ctx;
  Prepared P;
  kp_status s = prepare(prob, false, P, c);
  if (s != KP_OK) return s;
  if ((s = choose_kernel(c, P, false)) != KP_OK) return s;
  SweepWs w;
  if ((s = carve_ws(c, P, false, w)) != KP_OK) return s;
  if ((s = upload_B(c, P, w)) != KP_OK) return s;
  double *Rd = R ? R : w.Rtmp;
  if ((s = eval_into(c, P, w, lambda_inout, Rd, g ? g : w.gtmp, primal ? primal : w.Ptmp, nullptr)) != KP_OK)
    return s;
  HIP_TRY(kp_launch_dd_update(P.pr.K, alpha, Rd, w.B, lambda_inout, c->stream));
  return KP_OK;
}

kp_status kp_dual_backward(void *ctx, const kp_problem *prob, const double *R,
                           const double *grad_out, double *grad_lambda) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!prob || !prob->B || prob->K < 1) return fail(KP_ERR_INVALID, "problem/B invalid");
  if (!R || !grad_out || !grad_lambda) return fail(KP_ERR_INVALID, "NULL argument");
  Ctx *c = (Ctx *)ctx;
  const int K = prob->K;
  for (int k = 0; k < K; ++k)
    if (!(std::isfinite(prob->B[k]) && prob->B[k] > 0.0))
      return fail(KP_ERR_INVALID, "B[%d] must be finite and > 0", k);
  Carve cv;
  size_t oB = cv.take((size_t)K * 8);
  kp_status s = ensure_ws(c, cv.off);
  if (s != KP_OK) return s;
  double *Bd = (double *)((char *)c->ws + oB);
  HIP_TRY(hipMemcpyAsync(Bd, prob->B, (size_t)K * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(kp_launch_dual_backward(K, R, Bd, grad_out, grad_lambda, c->stream));
  return KP_OK;
}

kp_status kp_scd_sweep_masked(void *ctx, const kp_problem *prob, const double *lambda_in,
                              double *lambda_out, const uint8_t *kmask, double *R, double *g,
                              double *primal) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  return kp_scd_sweep_masked_impl((Ctx *)ctx, prob, lambda_in, lambda_out, kmask, R, g, primal);
}

}  // extern "C"

namespace {
kp_status kp_scd_sweep_masked_impl(Ctx *c, const kp_problem *prob, const double *lambda_in,
                                   double *lambda_out, const uint8_t *kmask, double *R, double *g,
                                   double *primal) {
  if (!lambda_in || !lambda_out) return fail(KP_ERR_INVALID, "lambda is NULL");
  Prepared P;
  kp_status s = prepare(prob, true, P, c);
  if (s != KP_OK) return s;
  if ((s = choose_kernel(c, P, true)) != KP_OK) return s;
  SweepWs w;
  if ((s = carve_ws(c, P, true, w)) != KP_OK) return s;
  const int K = P.pr.K;
  if ((s = upload_B(c, P, w)) != KP_OK) return s;
  if (kmask) HIP_TRY(hipMemcpyAsync(w.kmask, kmask, (size_t)K, hipMemcpyHostToDevice, c->stream));
  // window hint from the previous call with the same K (performance only)
  if (!c->delta_dev || c->delta_K != K) {
    if (c->delta_dev) HIP_TRY(hipFree(c->delta_dev));
    // [K] bucket widths, [K] last steps, [K] lambda^{t-1}, [K] lambda^{t-2}
    HIP_TRY(hipMalloc(&c->delta_dev, (size_t)K * 32));
    c->delta_K = K;
    c->delta_valid = false;
  }
  if (!c->delta_valid)   // no history: NaN multipliers (all bits set)
    HIP_TRY(hipMemsetAsync(c->delta_dev + 2 * K, 0xFF, (size_t)K * 16, c->stream));
  // the window pass needs the statistics of the same pass (R at lambda_in)
  const int window = (c->window_enabled && P.pr.N > 0 && !c->interp) ? 1 : 0;
  HIP_TRY(kp_launch_scd_init(w.st, K, lambda_in, kmask ? w.kmask : nullptr, c->delta_dev,
                             c->delta_valid ? 1 : 0, window, c->interp ? 1 : 0, c->stream));
  // the first pass runs split (all users, then the listed ones) when every
  // knapsack still searching starts with a window
  // (uniform-row kernel); the general kernel runs such a pass without the
  // histograms of the other search modes
  bool split = false, nohist = false, dwin = false;
  const bool nh_gain = !P.ell_D && (P.U_nh != P.U || P.grid_nh != P.grid);
  const bool sample = c->sample_min > 0 && P.pr.N >= c->sample_min && !c->interp;
  const bool counts = window && c->delta_valid && (w.fcap || nh_gain || P.dwin_grid);
  // the search-mode counts, and for dense costs the probe of the users'
  // lines (read back together), decide the first pass's kernel
  auto count_and_choose = [&]() -> kp_status {
    HIP_TRY(kp_launch_count_modes(w.st, K, w.modes, c->stream));
    const bool probe = counts && P.dwin_grid;
    if (probe) HIP_TRY(kp_launch_dense_probe(make_args(P, lambda_in, w, nullptr, true), w.modes + 3, c->stream));
    HIP_TRY(hipMemcpyAsync(c->pinned + 20, w.modes, 16, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (counts) {
      split = w.fcap && c->pinned[20] > 0 && c->pinned[21] == 0;
      nohist = nh_gain && c->pinned[21] == 0;
      // dense costs: the lane-per-user window pass when every window is
      // centred on lambda^t, or when almost no sampled user has a line that
      // can turn positive in any window (its gap test then settles every
      // pair, whatever the windows); alternation windows otherwise go to the
      // general kernel, whose per-(user, knapsack) tests stop early
      dwin = probe && c->pinned[21] == 0 &&
             (c->pinned[22] == 0 || c->pinned[23] * 64 <= KP_PROBE_USERS);
    }
    return KP_OK;
  };
  if (counts || sample) {
    if ((s = count_and_choose()) != KP_OK) return s;
    // full searches (knapsacks without a window) start from a sample
    if (sample && c->pinned[21] > 0) {
      if ((s = sample_center(c, prob, P, w, lambda_in, kmask)) != KP_OK) return s;
      // the sample's threshold may have opened windows for all of them:
      // choose the first pass's kernel again
      if (counts && window && (s = count_and_choose()) != KP_OK) return s;
    }
  }
  HIP_TRY(hipMemsetAsync(w.stat, 0, w.stat_bytes, c->stream));   // status, histograms
  double *Rd = R ? R : w.Rtmp;
  double *gd = g ? g : w.gtmp;
  double *Pd = primal ? primal : w.Ptmp;
  int pass = 0;
  for (;; ++pass) {
    if (pass >= kMaxPasses) return fail(KP_ERR_INTERNAL, "SCD threshold search exceeded %d passes", kMaxPasses);
    if (P.pr.N > 0) {
      SweepArgs a = make_args(P, lambda_in, w, nullptr, pass == 0);
      a.pass = pass;
      a.alg5_q = alg5_q(c, P);
      if (pass == 0 && nohist) {
        a.no_hist = 1;
        a.ntiles = P.ntiles_nh;
      }
      HIP_TRY(timed_sweep(c, a, P, true, P.bytes, split && pass == 0, dwin && pass == 0));
    }
    if (pass == 0) {
      if (P.pr.N > 0) {
        HIP_TRY(kp_launch_reduce_stats(w.partials, c->stats_grid, K, lambda_in, w.B, Rd,
                                       gd, Pd, c->stream));
      } else {
        HIP_TRY(hipMemsetAsync(w.partials, 0, (size_t)(K + 2) * 8, c->stream));
        HIP_TRY(kp_launch_reduce_stats(w.partials, 1, K, lambda_in, w.B, Rd, gd, Pd, c->stream));
      }
    }
    HIP_TRY(kp_launch_scd_locate_select(w.st, K, w.B, Rd, nullptr, w.hist_sum, w.hist_cnt, w.ev1, w.ev2,
                                        w.emit_cap, w.pending, w.win, c->stream));
    // one copy of the status block: pending, walk-limit counter, window and
    // list counters
    int *st = c->pinned + 32;
    HIP_TRY(hipMemcpyAsync(st, w.stat, 48, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (pass == 0 && window) {
      c->win_tried += (unsigned)st[4];
      c->win_above += (unsigned)st[5];
      c->win_below += (unsigned)st[6];
      c->win_emitted += (unsigned)st[7];
    }
    if (pass == 0 && (split || dwin)) c->win_listed += (unsigned)st[9];
    if (*(unsigned long long *)(st + 2))
      return fail(KP_ERR_INTERNAL, "breakpoint walk exceeded its event limit");
    if (st[0] == 0) break;
  }
  HIP_TRY(kp_launch_scd_finish(w.st, K, lambda_in, lambda_out, c->delta_dev, c->stream));
  c->delta_valid = true;
  return KP_OK;
}
}  // namespace

extern "C" {

kp_status kp_scd_sweep(void *ctx, const kp_problem *prob, const double *lambda_in,
                       double *lambda_out, double *R, double *g, double *primal) {
  return kp_scd_sweep_masked(ctx, prob, lambda_in, lambda_out, nullptr, R, g, primal);
}

// Device buffer owned by one call (freed on every exit path).
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { if (p) (void)hipFree(p); }
};

kp_status kp_presolve(void *ctx, const kp_problem *prob, const int64_t *users, int64_t n,
                      int32_t max_iter, double *lambda_inout, int32_t *iterations_out) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!users || !lambda_inout) return fail(KP_ERR_INVALID, "NULL argument");
  if (max_iter < 1) return fail(KP_ERR_INVALID, "max_iter must be >= 1");
  Ctx *c = (Ctx *)ctx;
  Prepared P;
  kp_status s = prepare(prob, true, P, c);
  if (s != KP_OK) return s;
  const int64_t N = prob->N;
  const int M = prob->M, K = prob->K;
  if (n < 1 || n > N) return fail(KP_ERR_INVALID, "sample size must be in [1, N]");
  {
    std::vector<int64_t> u(users, users + n);
    std::sort(u.begin(), u.end());
    if (u.front() < 0 || u.back() >= N) return fail(KP_ERR_INVALID, "sampled user out of [0, N)");
    if (std::adjacent_find(u.begin(), u.end()) != u.end())
      return fail(KP_ERR_INVALID, "sampled users must be distinct");
  }
  const bool csr = prob->b_format == KP_B_CSR;
  HIP_TRY(hipStreamSynchronize(c->stream));
  // the sub-instance: users, p, costs (dense rows, or CSR rows with new offsets)
  Carve cv;
  const size_t o_u = cv.take((size_t)n * 8);
  const size_t o_p = cv.take((size_t)n * M * 4);
  const size_t o_b = csr ? 0 : cv.take((size_t)n * M * K * 4);
  const size_t o_len = csr ? cv.take((size_t)n * M * 8) : 0;
  const size_t o_ptr = csr ? cv.take((size_t)(n * M + 1) * 8) : 0;
  const size_t o_lam = cv.take((size_t)K * 8);
  DevBuf buf;
  if (hipMalloc(&buf.p, cv.off) != hipSuccess) { buf.p = nullptr; return fail(KP_ERR_NOMEM, "hipMalloc failed"); }
  char *b = (char *)buf.p;
  int64_t *ud = (int64_t *)(b + o_u);
  HIP_TRY(hipMemcpyAsync(ud, users, (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
  kp_problem sub = *prob;
  sub.N = n;
  sub.p = (const float *)(b + o_p);
  DevBuf ent;
  if (!csr) {
    sub.b = (const float *)(b + o_b);
    HIP_TRY(kp_launch_gather_dense(prob->p, prob->b, ud, n, M, K, (float *)(b + o_p), (float *)(b + o_b),
                                   c->stream));
  } else {
    HIP_TRY(kp_launch_gather_dense(prob->p, nullptr, ud, n, M, K, (float *)(b + o_p), nullptr, c->stream));
    int64_t *subptr = (int64_t *)(b + o_ptr);
    HIP_TRY(kp_launch_gather_csr_ptr(prob->b_rowptr, ud, n, M, (int64_t *)(b + o_len), subptr, c->stream));
    int64_t nnz = 0;
    HIP_TRY(hipMemcpyAsync(&nnz, subptr + n * M, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hipMalloc(&ent.p, (size_t)std::max<int64_t>(nnz, 1) * 8) != hipSuccess) {
      ent.p = nullptr;
      return fail(KP_ERR_NOMEM, "hipMalloc failed");
    }
    int32_t *scol = (int32_t *)ent.p;
    float *sval = (float *)((char *)ent.p + (size_t)std::max<int64_t>(nnz, 1) * 4);
    HIP_TRY(kp_launch_gather_csr(prob->b_rowptr, prob->b_col, prob->b_val, ud, n, M, subptr, scol, sval,
                                 c->stream));
    sub.b_rowptr = subptr;
    sub.b_col = scol;
    sub.b_val = sval;
  }
  // budgets scaled by the sample's share of the users
  std::vector<double> Bs(K);
  const double scale = (double)n / (double)N;
  for (int k = 0; k < K; ++k) Bs[k] = prob->B[k] * scale;
  sub.B = Bs.data();
  // SCD on the sample until the multipliers repeat (the window hints of the
  // full problem do not carry over)
  c->delta_valid = false;
  double *lam_b = (double *)(b + o_lam);
  double *cur = lambda_inout, *nxt = lam_b;
  std::vector<double> hc(K), hn(K);
  int it = 0;
  kp_status rs = KP_OK;
  while (it < max_iter) {
    rs = kp_scd_sweep(ctx, &sub, cur, nxt, nullptr, nullptr, nullptr);
    if (rs != KP_OK) break;
    ++it;
    HIP_TRY(hipMemcpyAsync(hc.data(), cur, (size_t)K * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hn.data(), nxt, (size_t)K * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::swap(cur, nxt);
    if (memcmp(hc.data(), hn.data(), (size_t)K * 8) == 0) break;
  }
  if (rs == KP_OK && cur != lambda_inout)
    HIP_TRY(hipMemcpyAsync(lambda_inout, cur, (size_t)K * 8, hipMemcpyDeviceToDevice, c->stream));
  (void)hipStreamSynchronize(c->stream);
  c->delta_valid = false;
  if (rs != KP_OK) return rs;
  if (iterations_out) *iterations_out = it;
  return KP_OK;
}

kp_status kp_validate_inputs(void *ctx, const kp_problem *prob) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  Prepared P;
  kp_status s = prepare(prob, false, P, c);
  if (s != KP_OK) return s;
  Carve cv;
  size_t of = cv.take(16);
  if ((s = ensure_ws(c, cv.off)) != KP_OK) return s;
  unsigned int *flags = (unsigned int *)((char *)c->ws + of);
  HIP_TRY(hipMemsetAsync(flags, 0, 16, c->stream));
  const int64_t nrows = prob->N * prob->M;
  HIP_TRY(kp_launch_validate(prob->p, nrows, flags, c->stream));
  if (prob->b_format == KP_B_DENSE) {
    HIP_TRY(kp_launch_validate(prob->b, nrows * prob->K, flags, c->stream));
  } else {
    int64_t nnz = 0;
    if (nrows > 0)
      HIP_TRY(hipMemcpyAsync(&nnz, prob->b_rowptr + nrows, 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(kp_launch_validate(prob->b_val, nnz, flags, c->stream));
    HIP_TRY(kp_launch_validate_csr(prob->b_rowptr, prob->b_col, nrows, prob->K, flags, c->stream));
    if (prob->b_row_nnz && nrows > 0 && nnz != nrows * (int64_t)prob->b_row_nnz) {
      (void)hipStreamSynchronize(c->stream);
      return fail(KP_ERR_INVALID, "b_row_nnz = %d declared, but rowptr[N*M] = %lld", prob->b_row_nnz,
                  (long long)nnz);
    }
    if (prob->b_row_nnz && nrows > 0)
      HIP_TRY(kp_launch_ell_check(prob->b_rowptr, nrows, prob->b_row_nnz, flags + 3, c->stream));
  }
  HIP_TRY(hipMemcpyAsync(c->pinned, flags, 16, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const unsigned int *f = (const unsigned int *)c->pinned;
  if (f[2]) return fail(KP_ERR_INVALID, "CSR rows must have ascending columns in [0,K)");
  if (f[3]) return fail(KP_ERR_INVALID, "b_row_nnz = %d declared, but some row does not hold its entries at r*D",
                        prob->b_row_nnz);
  if (f[0]) return fail(KP_ERR_NONFINITE, "p or b holds a NaN or Inf");
  if (f[1]) return fail(KP_ERR_NEGATIVE, "p or b holds a negative value");
  return KP_OK;
}

kp_status kp_tree_from_sets(int32_t M, int32_t L, const int32_t *set_offsets,
                            const int32_t *set_items, const int32_t *caps, int32_t *L_out,
                            int32_t *parent_out, int32_t *cap_out, int32_t *leaf_of_item_out) {
  if (M < 1 || M > KP_MAX_M) return fail(KP_ERR_UNSUPPORTED, "M must be in 1..%d", KP_MAX_M);
  if (L < 0) return fail(KP_ERR_INVALID, "L must be >= 0");
  if (L > 0 && (!set_offsets || !set_items || !caps))
    return fail(KP_ERR_INVALID, "NULL set arrays");
  if (!L_out || !leaf_of_item_out || (L > 0 && (!parent_out || !cap_out)))
    return fail(KP_ERR_INVALID, "NULL outputs");
  std::vector<uint64_t> mask;
  std::vector<int> cap;
  for (int l = 0; l < L; ++l) {
    if (caps[l] < 1) return fail(KP_ERR_INVALID, "caps[%d] must be >= 1", l);
    uint64_t m = 0;
    for (int e = set_offsets[l]; e < set_offsets[l + 1]; ++e) {
      const int j = set_items[e];
      if (j < 0 || j >= M) return fail(KP_ERR_INVALID, "set %d holds item %d outside [0,M)", l, j);
      m |= 1ull << j;
    }
    if (!m) continue;  // an empty set constrains nothing
    bool merged = false;
    for (size_t t = 0; t < mask.size(); ++t)
      if (mask[t] == m) { cap[t] = std::min(cap[t], caps[l]); merged = true; break; }
    if (!merged) { mask.push_back(m); cap.push_back(caps[l]); }
  }
  const int n = (int)mask.size();
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b) {
      const uint64_t x = mask[a] & mask[b];
      if (x && x != mask[a] && x != mask[b])
        return fail(KP_ERR_NOT_LAMINAR, "sets %d and %d overlap without nesting", a, b);
    }
  // parent = smallest strict superset
  for (int a = 0; a < n; ++a) {
    int best = -1;
    for (int b = 0; b < n; ++b) {
      if (b == a) continue;
      if ((mask[a] & mask[b]) == mask[a] && mask[b] != mask[a]) {
        if (best < 0 || __builtin_popcountll(mask[b]) < __builtin_popcountll(mask[best])) best = b;
      }
    }
    parent_out[a] = best;
    cap_out[a] = cap[a];
  }
  for (int j = 0; j < M; ++j) {
    int best = -1;
    for (int a = 0; a < n; ++a)
      if ((mask[a] >> j & 1) && (best < 0 || __builtin_popcountll(mask[a]) < __builtin_popcountll(mask[best])))
        best = a;
    leaf_of_item_out[j] = best;
  }
  *L_out = n;
  return KP_OK;
}

kp_status kp_set_tuning(void *ctx, int32_t M, int32_t K, int32_t b_format, int32_t users_per_tile,
                        int32_t grid) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (users_per_tile < 0 || grid < 0) return fail(KP_ERR_INVALID, "negative tuning value");
  Ctx *c = (Ctx *)ctx;
  if (users_per_tile == 0 && grid == 0) c->tuning.erase(std::make_tuple(M, K, b_format));
  else c->tuning[std::make_tuple(M, K, b_format)] = std::make_pair(users_per_tile, grid);
  return KP_OK;
}

kp_status kp_get_launch_shape(void *ctx, int32_t *kernel, int32_t *users_per_tile, int32_t *grid) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  const Ctx *c = (const Ctx *)ctx;
  if (kernel) *kernel = c->last_kernel;
  if (users_per_tile) *users_per_tile = c->last_U;
  if (grid) *grid = c->last_grid;
  return KP_OK;
}

kp_status kp_set_batched_tuning(void *ctx, int32_t lds_bytes, int32_t block_mult) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (lds_bytes < 0 || block_mult < 0) return fail(KP_ERR_INVALID, "negative tuning value");
  if (lds_bytes > (int32_t)kMaxLds) return fail(KP_ERR_UNSUPPORTED, "LDS budget above %zu bytes", kMaxLds);
  if (block_mult > 1024) return fail(KP_ERR_UNSUPPORTED, "block multiple above 1024");
  Ctx *c = (Ctx *)ctx;
  c->bt_lds = lds_bytes;
  c->bt_mult = block_mult;
  return KP_OK;
}

kp_status kp_set_kernel_choice(void *ctx, int32_t allow_uniform_rows) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  ((Ctx *)ctx)->ell_enabled = allow_uniform_rows != 0;
  return KP_OK;
}

kp_status kp_set_reduce(void *ctx, int32_t mode) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (mode != 0 && mode != 1) return fail(KP_ERR_INVALID, "reduce mode must be 0 (exact) or 1 (interpolated)");
  ((Ctx *)ctx)->interp = mode == 1;
  return KP_OK;
}

kp_status kp_set_sampled_start(void *ctx, int64_t min_users) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (min_users < 0) return fail(KP_ERR_INVALID, "min_users must be >= 0");
  ((Ctx *)ctx)->sample_min = min_users;
  return KP_OK;
}

kp_status kp_set_alg5(void *ctx, int32_t on) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  ((Ctx *)ctx)->alg5 = on != 0;
  return KP_OK;
}

kp_status kp_set_window(void *ctx, int32_t on) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  ((Ctx *)ctx)->window_enabled = on != 0;
  return KP_OK;
}

kp_status kp_get_window_stats(void *ctx, int64_t *tried, int64_t *above, int64_t *below,
                              int64_t *emitted) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  const Ctx *c = (const Ctx *)ctx;
  if (tried) *tried = c->win_tried;
  if (above) *above = c->win_above;
  if (below) *below = c->win_below;
  if (emitted) *emitted = c->win_emitted;
  return KP_OK;
}

kp_status kp_get_window_listed(void *ctx, int64_t *listed) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (listed) *listed = ((const Ctx *)ctx)->win_listed;
  return KP_OK;
}

kp_status kp_csr_row_nnz(void *ctx, const kp_problem *prob, int32_t *D_out) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!prob || !D_out) return fail(KP_ERR_INVALID, "NULL argument");
  if (prob->b_format != KP_B_CSR) return fail(KP_ERR_INVALID, "kp_csr_row_nnz needs CSR costs");
  if (prob->N < 0 || prob->M < 1) return fail(KP_ERR_INVALID, "bad N or M");
  Ctx *c = (Ctx *)ctx;
  *D_out = 0;
  const int64_t nrows = prob->N * prob->M;
  if (nrows == 0) return KP_OK;
  if (!prob->b_rowptr) return fail(KP_ERR_INVALID, "b_rowptr is NULL");
  unsigned int D = 0;
  kp_status s = check_rows(c, prob->b_rowptr, nrows, &D);
  if (s != KP_OK) return s;
  *D_out = (int32_t)D;
  return KP_OK;
}

kp_status kp_set_timing(void *ctx, int32_t on) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  drain_events(c, true);
  c->timing = on != 0;
  c->sweep_ms = 0.0;
  c->sweep_launches = 0;
  c->sweep_bytes = 0.0;
  c->batched_passes = 0;
  return KP_OK;
}

kp_status kp_get_batched_passes(void *ctx, int64_t *passes) {
  if (!ctx || !passes) return fail(KP_ERR_INVALID, "NULL argument");
  *passes = ((const Ctx *)ctx)->batched_passes;
  return KP_OK;
}

kp_status kp_stream_read(void *hip_stream, const void *src, size_t bytes, uint64_t *out) {
  if (!src || !out) return fail(KP_ERR_INVALID, "NULL argument");
  if (((uintptr_t)src & 15) != 0 || (bytes & 15) != 0)
    return fail(KP_ERR_INVALID, "src must be 16-byte aligned and bytes a multiple of 16");
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(kp_launch_stream_read(src, (int64_t)(bytes / 16), (unsigned long long *)out, 0, st));
  return KP_OK;
}

kp_status kp_get_timing(void *ctx, double *sweep_ms_total, int64_t *sweep_launches,
                        double *sweep_bytes_total) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  Ctx *c = (Ctx *)ctx;
  drain_events(c, true);
  if (sweep_ms_total) *sweep_ms_total = c->sweep_ms;
  if (sweep_launches) *sweep_launches = c->sweep_launches;
  if (sweep_bytes_total) *sweep_bytes_total = c->sweep_bytes;
  return KP_OK;
}

kp_status kp_primal_fixup(void *ctx, const kp_problem *prob, const double *lambda, uint8_t *x_out,
                          double *primal_out, double *R_out, int64_t *n_reset_out) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  if (!lambda || !primal_out || !R_out || !n_reset_out) return fail(KP_ERR_INVALID, "NULL argument");
  Ctx *c = (Ctx *)ctx;
  Prepared P;
  kp_status s = prepare(prob, false, P, c);
  if (s != KP_OK) return s;
  if (P.pr.N >= (int64_t)1 << 32) return fail(KP_ERR_UNSUPPORTED, "post-processing supports N < 2^32");
  if ((s = choose_kernel(c, P, false)) != KP_OK) return s;
  const int K = P.pr.K;
  const int64_t N = P.pr.N;
  // pass 1: x(lambda), R, P
  SweepWs w;
  if ((s = carve_ws(c, P, false, w)) != KP_OK) return s;
  // workspace beyond the sweep's: x (when the caller gives none), the
  // violated slots, the post-processing scratch
  Carve cv;
  cv.off = 0;
  {
    Carve base;
    base.take((size_t)P.stage_grid() * (K + 2) * 8); base.take((size_t)K * 8); base.take((size_t)K * 8);
    base.take(8); base.take(8); base.take(8); base.take(8);
    cv.off = base.off;
  }
  const size_t o_x = cv.take(x_out ? 0 : (size_t)N * P.pr.M);
  const size_t o_Rv = cv.take((size_t)K * 8);
  const size_t o_Pv = cv.take(8);
  const size_t o_kv = cv.take((size_t)K * 4);
  const size_t o_vk = cv.take((size_t)K * 4);
  const size_t o_Bv = cv.take((size_t)K * 8);
  // sized for the worst case (every knapsack violated)
  const size_t o_scr = cv.take(kp_fixup_scratch_bytes(N, K, K));
  if ((s = ensure_ws(c, cv.off)) != KP_OK) return s;
  if ((s = carve_ws(c, P, false, w)) != KP_OK) return s;   // re-carve after a possible regrow
  char *b = (char *)c->ws;
  uint8_t *xd = x_out ? x_out : (uint8_t *)(b + o_x);
  double *Rv = (double *)(b + o_Rv), *Pv = (double *)(b + o_Pv);
  int *kvd = (int *)(b + o_kv), *vkd = (int *)(b + o_vk);
  double *Bvd = (double *)(b + o_Bv);
  if ((s = upload_B(c, P, w)) != KP_OK) return s;
  if ((s = eval_into(c, P, w, lambda, Rv, w.gtmp, Pv, xd)) != KP_OK) return s;
  std::vector<double> Rh(K);
  HIP_TRY(hipMemcpyAsync(Rh.data(), Rv, (size_t)K * 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<int> kv(K, -1), vk;
  std::vector<double> bv;
  int nv = 0;
  for (int k = 0; k < K; ++k)
    if (Rh[k] > P.B[k]) { kv[k] = nv++; vk.push_back(k); bv.push_back(P.B[k]); }
  if (nv == 0) {
    HIP_TRY(hipMemcpyAsync(R_out, Rv, (size_t)K * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(primal_out, Pv, 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(n_reset_out, 0, 8, c->stream));
    return KP_OK;
  }
  HIP_TRY(hipMemcpyAsync(kvd, kv.data(), (size_t)K * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(vkd, vk.data(), (size_t)nv * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(Bvd, bv.data(), (size_t)nv * 8, hipMemcpyHostToDevice, c->stream));
  // blocks of the passes over users: a few per compute unit
  const int64_t nch = (N + 4095) / 4096;
  const int persist = (int)std::max<int64_t>(1, std::min<int64_t>(nch, 1024));
  // the per-user bin pass: the uniform-row kernel's evaluation with the bins
  // (LDS for the sums kept to 24 KB, next to its staged tiles) when it
  // applies, else a thread per user
  std::function<hipError_t(const FixBins &)> lean;
  int nb = kp_fixup_bins(nv, 40 * 1024);
  if (P.ell_D) {
    nb = kp_fixup_bins(nv, 24 * 1024);
    lean = [&](const FixBins &fb) -> hipError_t {
      SweepArgs a = make_args(P, lambda, w, nullptr, false);
      a.ntiles = P.ell_ntiles;
      a.fx = fb;
      return kp_launch_ell(a, P.ell_D, P.ell_grid, 4, c->stream, nullptr);
    };
  }
  HIP_TRY(kp_launch_fixup_pipeline(P.pr, P.row_nnz, xd, lambda, kvd, vkd, Bvd, nv, nb, Rv, Pv, R_out, primal_out,
                                   n_reset_out, b + o_scr, c->stream, (uint32_t *)(c->pinned + 48), persist,
                                   lean));
  return KP_OK;
}

// ---- batched plan: tables built once, one iteration replayable as a graph ----
struct BatchPlan {
  Ctx *c = nullptr;
  int n = 0, Kf = 0, GB = 0, ncol = 0;
  int Umin = 0, Umax = 0;   // users per tile over the instances
  double bytes = 0.0;   // algorithmic bytes of one sweep pass over every instance
  int64_t T = 0;
  size_t lds = 0;
  uint32_t cap = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // device tables
  SweepArgs *d[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [dir][first pass?]
  TileGeom *geom = nullptr;
  int *boff = nullptr, *kin = nullptr, *klo = nullptr, *pend = nullptr;
  void *lam_tab[2] = {nullptr, nullptr};   // [dir]: lambda_in pointer table; the other dir's is lambda_out
  void *coltab[2] = {nullptr, nullptr};    // [dir]: statistics column table (reads lambda_in)
  KState *kst = nullptr;
  double *hint = nullptr;   // [2 Kf] bucket widths and last steps carried between iterations
  uint64_t *eoff = nullptr; // [Kf] start of each knapsack's emission buffer
  uint32_t *ecap = nullptr; // [Kf] its capacity
  bool window = true;       // iterations start with a window where the last step allows
  double *Bf = nullptr, *e1 = nullptr, *e2 = nullptr, *stats = nullptr;
  XSum *hs = nullptr;
  uint32_t *hc = nullptr;
  unsigned long long *err = nullptr;
  int *pinned = nullptr;     // [0] pending knapsacks, [2..3] error word, [16..] per-instance flags
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  // later passes: the blocks are split again among the instances still searching
  int *koff = nullptr;      // [n+1] first flat knapsack of every instance
  int *active = nullptr;    // [n] instance needs another pass (written by k_inst_active)
  SweepArgs *rd = nullptr;  // [n] descriptors of the active instances
  TileGeom *rg = nullptr;   // [n]
  int *rboff = nullptr;     // [n+1]
  unsigned char *up = nullptr;   // pinned upload buffer of rd, rg, rboff
  int gmax = 0;             // blocks of a pass over every instance's tiles
  double *s1 = nullptr, *s2 = nullptr;
  uint16_t *sk = nullptr;
  size_t stage_total = 0;   // staged events of the whole launch
  std::vector<SweepArgs> hd[2];   // [dir] host descriptors of the later passes
  std::vector<TileGeom> hg;
  std::vector<int64_t> ntiles;
  std::vector<double> pairs;      // users x knapsacks of every instance
  std::vector<size_t> ilds;       // LDS of every instance's tiles
  std::vector<int> order;         // instances by decreasing tile cost (the block layout's order)
  // the later passes split on the device (graph capture of whole iterations)
  SweepArgs *dhd[2] = {nullptr, nullptr};   // [dir] hd on the device
  TileGeom *dhg = nullptr;
  int *dord = nullptr;
  int64_t *dnt = nullptr;
  double *dpairs = nullptr;
  int *ctl = nullptr;       // [0] open instances of the pass, [1] passes with work, [2] split overflow
  int glater = 0;           // later passes in the iteration's graph (0: only the first pass)
  int gfix = 0;             // blocks of such a pass (an upper bound on any split's)
};

// Split of a later pass: the instances whose knapsacks still search share
// every block (in proportion to their tiles, costliest tiles first), and the staging area of the
// whole launch is divided among their blocks.  Returns the number of active
// instances (0: nothing to sweep).
int plan_resplit(BatchPlan *p, int dir, int *blocks, size_t *lds) {
  const int n = p->n;
  const int *flag = p->pinned + 16;
  std::vector<int> act;
  int64_t TA = 0;
  for (int s : p->order)
    if (flag[s] && p->ntiles[s] > 0) { act.push_back(s); TA += p->ntiles[s]; }
  const int na = (int)act.size();
  if (na == 0) return 0;
  const int G = (int)std::max<int64_t>(na, std::min<int64_t>(TA, p->gmax));
  SweepArgs *d = (SweepArgs *)p->up;
  TileGeom *g = (TileGeom *)(p->up + (size_t)n * sizeof(SweepArgs));
  int *bo = (int *)(p->up + (size_t)n * (sizeof(SweepArgs) + sizeof(TileGeom)));
  std::vector<int64_t> nb(na);
  std::vector<double> want(na);
  double tot = 0.0;
  size_t L = 0;
  for (int i = 0; i < na; ++i) {
    const int s = act[i];
    nb[i] = std::max<int64_t>(1, std::min<int64_t>(p->ntiles[s], std::llround((double)G * p->ntiles[s] / (double)TA)));
    want[i] = std::min<double>(kStageCapMax, std::max<double>(kStageCap, p->pairs[s] / nb[i] / 64.0));
    tot += want[i] * nb[i];
    L = std::max(L, p->ilds[s]);
  }
  const double scale = tot > (double)p->stage_total ? (double)p->stage_total / tot : 1.0;
  size_t so = 0;
  bo[0] = 0;
  for (int i = 0; i < na; ++i) {
    const int s = act[i];
    const uint32_t cap = (uint32_t)std::max(1.0, std::floor(want[i] * scale));
    d[i] = p->hd[dir][s];
    d[i].stage_v1 = p->s1 + so;
    d[i].stage_v2 = p->s2 + so;
    d[i].stage_k = p->sk + so;
    d[i].stage_cap = cap;
    so += (size_t)nb[i] * cap;
    g[i] = p->hg[s];
    bo[i + 1] = bo[i] + (int)nb[i];
  }
  if (so > p->stage_total) return -1;   // cannot happen: the caps were scaled to fit
  *blocks = bo[na];
  *lds = L;
  return na;
}

// The later passes of a whole-iteration graph: each splits the open
// instances' blocks on the device, sweeps them (blocks past the split exit),
// and runs the threshold search; a pass with nothing open does no work.
kp_status plan_later_passes_dev(BatchPlan *p, int dir, hipStream_t s) {
  for (int j = 0; j < p->glater; ++j) {
    ResplitArgs r;
    r.order = p->dord;
    r.active = p->active;
    r.ntiles = p->dnt;
    r.pairs = p->dpairs;
    r.hd = p->dhd[dir];
    r.hg = p->dhg;
    r.n = p->n;
    r.gmax = p->gmax;
    r.cap_min = kStageCap;
    r.cap_max = kStageCapMax;
    r.stage_total = p->stage_total;
    r.s1 = p->s1;
    r.s2 = p->s2;
    r.sk = p->sk;
    r.rd = p->rd;
    r.rg = p->rg;
    r.rboff = p->rboff;
    r.ctl = p->ctl;
    r.reset = j == 0 ? 1 : 0;
    HIP_TRY(kp_launch_plan_resplit(r, s));
    if (p->T > 0) HIP_TRY(kp_launch_sweep_batched(p->rd, p->rg, p->rboff, p->n, p->gfix, p->lds, s, p->ctl));
    HIP_TRY(kp_launch_scd_locate_select(p->kst, p->Kf, p->Bf, p->stats, p->kin, p->hs, p->hc, p->e1, p->e2, p->cap, p->pend, nullptr, s));
    HIP_TRY(kp_launch_batched_aux(2, nullptr, p->Kf, p->kst, p->lam_tab[1 - dir], p->kin, p->klo, p->hint, nullptr,
                                  nullptr, s));
    HIP_TRY(kp_launch_inst_active(p->kst, p->koff, p->n, p->active, s));
  }
  HIP_TRY(hipMemcpyAsync(p->pinned, p->pend, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(p->pinned + 2, p->err, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(p->pinned + 16, p->active, (size_t)p->n * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(p->pinned + 8, p->ctl, 12, hipMemcpyDeviceToHost, s));
  return KP_OK;
}

kp_status plan_first_pass(BatchPlan *p, int dir, hipStream_t s) {
  HIP_TRY(kp_launch_batched_aux(p->window ? 3 : 1, nullptr, p->Kf, p->kst, p->lam_tab[dir], p->kin, p->klo, p->hint,
                                p->eoff, p->ecap, s));
  if (p->T > 0) HIP_TRY(kp_launch_sweep_batched(p->d[dir][1], p->geom, p->boff, p->n, p->GB, p->lds, s));
  HIP_TRY(kp_launch_batched_aux(0, p->coltab[dir], p->ncol, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr, s));
  HIP_TRY(kp_launch_scd_locate_select(p->kst, p->Kf, p->Bf, p->stats, p->kin, p->hs, p->hc, p->e1, p->e2, p->cap, p->pend, nullptr, s));
  HIP_TRY(kp_launch_batched_aux(2, nullptr, p->Kf, p->kst, p->lam_tab[1 - dir], p->kin, p->klo, p->hint, nullptr,
                                nullptr, s));
  HIP_TRY(kp_launch_inst_active(p->kst, p->koff, p->n, p->active, s));
  HIP_TRY(hipMemcpyAsync(p->pinned, p->pend, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(p->pinned + 2, p->err, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(p->pinned + 16, p->active, (size_t)p->n * 4, hipMemcpyDeviceToHost, s));
  return KP_OK;
}

kp_status plan_step(BatchPlan *p, int dir, double *stats_out, bool graph) {
  hipStream_t s = p->c->stream;
  Ctx *c = p->c;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->timing) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) (void)hipEventRecord(e0, s);
  }
  int passes = 1;
  int first_later = 1;   // index of the first later pass run from the host
  if (graph) {
    if (!p->exec[dir]) {
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      kp_status st = plan_first_pass(p, dir, s);
      if (st == KP_OK && p->glater > 0) st = plan_later_passes_dev(p, dir, s);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(s, &g);
      if (st != KP_OK) return st;
      if (e != hipSuccess) return fail(KP_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
      p->graph[dir] = g;
      HIP_TRY(hipGraphInstantiate(&p->exec[dir], g, nullptr, nullptr, 0));
    }
    HIP_TRY(hipGraphLaunch(p->exec[dir], s));
  } else {
    kp_status st = plan_first_pass(p, dir, s);
    if (st != KP_OK) return st;
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (graph && p->glater > 0) {
    if (p->pinned[10]) return fail(KP_ERR_INTERNAL, "batched staging split overflowed");
    passes += p->pinned[9];
    first_later = 1 + p->glater;
  }
  for (int pass = first_later;; ++pass) {
    if (*(unsigned long long *)(p->pinned + 2))
      return fail(KP_ERR_INTERNAL, "breakpoint walk exceeded its event limit");
    if (p->pinned[0] == 0) break;
    if (pass >= kMaxPasses) return fail(KP_ERR_INTERNAL, "SCD threshold search exceeded %d passes", kMaxPasses);
    if (p->T > 0) {
      int blocks = 0;
      size_t lds = 0;
      const int na = plan_resplit(p, dir, &blocks, &lds);
      if (na < 0) return fail(KP_ERR_INTERNAL, "batched staging split overflowed");
      if (na > 0) {
        const size_t nd = (size_t)p->n * sizeof(SweepArgs), ng = (size_t)p->n * sizeof(TileGeom);
        HIP_TRY(hipMemcpyAsync(p->rd, p->up, (size_t)na * sizeof(SweepArgs), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(p->rg, p->up + nd, (size_t)na * sizeof(TileGeom), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(p->rboff, p->up + nd + ng, (size_t)(na + 1) * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(kp_launch_sweep_batched(p->rd, p->rg, p->rboff, na, blocks, lds, s));
      }
    }
    ++passes;
    HIP_TRY(kp_launch_scd_locate_select(p->kst, p->Kf, p->Bf, p->stats, p->kin, p->hs, p->hc, p->e1, p->e2, p->cap, p->pend, nullptr, s));
    HIP_TRY(kp_launch_batched_aux(2, nullptr, p->Kf, p->kst, p->lam_tab[1 - dir], p->kin, p->klo, p->hint, nullptr,
                                nullptr, s));
    HIP_TRY(kp_launch_inst_active(p->kst, p->koff, p->n, p->active, s));
    HIP_TRY(hipMemcpyAsync(p->pinned, p->pend, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p->pinned + 2, p->err, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(p->pinned + 16, p->active, (size_t)p->n * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  if (c->timing && e0 && e1) {
    // the whole iteration (every pass and the search kernels between them),
    // with every input byte of every instance counted once
    (void)hipEventRecord(e1, s);
    c->ev_pending.push_back({e0, e1});
    c->sweep_launches += 1;
    c->sweep_bytes += p->bytes;
    c->batched_passes += passes;
    if (c->ev_pending.size() > 256) drain_events(c, true);
  }
  if (stats_out)
    HIP_TRY(hipMemcpyAsync(stats_out, p->stats, (size_t)p->ncol * 8, hipMemcpyDeviceToDevice, s));
  return KP_OK;
}

void plan_free(BatchPlan *p) {
  if (!p) return;
  if (p->c) (void)hipStreamSynchronize(p->c->stream);
  for (int d = 0; d < 2; ++d) {
    if (p->exec[d]) (void)hipGraphExecDestroy(p->exec[d]);
    if (p->graph[d]) (void)hipGraphDestroy(p->graph[d]);
  }
  if (p->ws) (void)hipFree(p->ws);
  if (p->pinned) (void)hipHostFree(p->pinned);
  if (p->up) (void)hipHostFree(p->up);
  delete p;
}

kp_status plan_create(Ctx *c, const kp_problem *probs, int n, const double *const *lam_a,
                      double *const *lam_b, BatchPlan **out) {
  if (n < 1 || !probs || !lam_a || !lam_b) return fail(KP_ERR_INVALID, "bad batch arguments");
  std::vector<Prepared> P(n);
  for (int s = 0; s < n; ++s) {
    kp_status st = prepare(&probs[s], true, P[s], c);
    if (st != KP_OK) {
      char m[sizeof g_err];
      memcpy(m, g_err, sizeof m);
      return fail(st, "instance %d: %s", s, m);
    }
    if (!lam_a[s] || !lam_b[s]) return fail(KP_ERR_INVALID, "instance %d: lambda is NULL", s);
  }
  BatchPlan *p = new BatchPlan();
  p->c = c;
  p->n = n;
  // every block of the batched launch gets the largest LDS any instance
  // needs, so instances with long rows take smaller tiles: the launch keeps
  // kBatchedBlocksPerCu blocks per compute unit for everyone
  const size_t lds_budget = c->bt_lds > 0 ? (size_t)c->bt_lds : kBatchedLds;
  for (auto &q : P) {
    int U = q.U;
    while (U > 1 && kp_sweep_lds_bytes(U, q.pr.M, q.pr.K, true, q.pr.fmt) > lds_budget) --U;
    while (U > 1 && q.pr.fmt == KP_B_DENSE && ((int64_t)U * q.pr.M * q.pr.K) % 4 != 0) --U;
    if (U != q.U) {
      q.U = U;
      q.ntiles = (q.pr.N + U - 1) / U;
    }
  }
  int64_t T = 0;
  int Kf = 0;
  for (auto &q : P) { T += q.ntiles; Kf += q.pr.K; }
  size_t lds = 0;
  for (int s = 0; s < n; ++s)
    lds = std::max(lds, kp_sweep_lds_bytes(P[s].U, P[s].pr.M, P[s].pr.K, true, P[s].pr.fmt));
  // blocks are split among the instances in proportion to their tiles; many
  // more blocks than can be resident at once keep the split fine-grained, and
  // the hardware dispatcher balances them (every instance gets at least one)
  int gmax = 32768;
  const int res = kp_sweep_batched_resident(lds);
  if (res > 0) gmax = std::min(gmax, (c->bt_mult > 0 ? c->bt_mult : 64) * res);
  const int G = (int)std::max<int64_t>(n, std::min<int64_t>(T, gmax));
  // algorithmic bytes of one pass over every instance
  double bytes = 0.0;
  for (int s = 0; s < n; ++s) {
    bytes += P[s].bytes;
    if (P[s].pr.fmt == KP_B_CSR && P[s].pr.N > 0) {
      int64_t nnz = 0;
      HIP_TRY(hipMemcpy(&nnz, P[s].pr.rowptr + P[s].pr.N * P[s].pr.M, 8, hipMemcpyDeviceToHost));
      bytes += (double)nnz * 8.0;
    }
  }
  std::vector<int> boff(n + 1, 0), koff(n + 1, 0);
  std::vector<size_t> poff(n + 1, 0);
  for (int s = 0; s < n; ++s) {
    int64_t b = T ? (int64_t)std::llround((double)G * P[s].ntiles / (double)T) : 1;
    b = std::max<int64_t>(1, std::min<int64_t>(b, std::max<int64_t>(1, P[s].ntiles)));
    boff[s + 1] = boff[s] + (int)b;
    koff[s + 1] = koff[s] + P[s].pr.K;
    poff[s + 1] = poff[s] + (size_t)b * (P[s].pr.K + 2);
  }
  if (lds > kMaxLds) { plan_free(p); return fail(KP_ERR_UNSUPPORTED, "an instance needs too much LDS"); }
  p->T = T; p->Kf = Kf; p->GB = boff[n]; p->lds = lds; p->cap = kEmitCapBatched;
  p->Umin = P[0].U;
  p->Umax = P[0].U;
  for (auto &q : P) { p->Umin = std::min(p->Umin, q.U); p->Umax = std::max(p->Umax, q.U); }
  p->bytes = bytes;
  const uint32_t cap = p->cap;
  // emission buffers per instance: room for two breakpoints per user and
  // knapsack (at least the uniform capacity, at most 2^20), scaled down when
  // the whole batch would exceed kEmitBytesBatched
  std::vector<uint32_t> icap(n);
  double ebytes = 0.0;
  for (int s = 0; s < n; ++s) {
    icap[s] = (uint32_t)std::min<int64_t>(1 << 20, std::max<int64_t>(cap, 2 * P[s].pr.N));
    ebytes += (double)P[s].pr.K * icap[s] * 16.0;
  }
  if (ebytes > kEmitBytesBatched)
    for (int s = 0; s < n; ++s)
      icap[s] = std::max<uint32_t>(cap, (uint32_t)(icap[s] * (kEmitBytesBatched / ebytes)));
  std::vector<uint64_t> ioff(n + 1, 0);
  for (int s = 0; s < n; ++s) ioff[s + 1] = ioff[s] + (uint64_t)P[s].pr.K * icap[s];
  const int ncol = Kf + 2 * n;
  p->ncol = ncol;
  Carve cv;
  size_t o_d[2][2];
  for (int d = 0; d < 2; ++d) for (int f = 0; f < 2; ++f) o_d[d][f] = cv.take((size_t)n * sizeof(SweepArgs));
  const size_t o_geom = cv.take((size_t)n * sizeof(TileGeom));
  const size_t o_boff = cv.take((size_t)(n + 1) * 4);
  const size_t o_part = cv.take(poff[n] * 8);
  const size_t o_B = cv.take((size_t)Kf * 8);
  const size_t o_st = cv.take((size_t)Kf * sizeof(KState));
  const size_t o_hs = cv.take((size_t)Kf * KP_NB * sizeof(XSum));
  const size_t o_hc = cv.take((size_t)Kf * KP_NB * 4);
  const size_t o_e1 = cv.take((size_t)ioff[n] * 8);
  const size_t o_e2 = cv.take((size_t)ioff[n] * 8);
  const size_t o_eo = cv.take((size_t)Kf * 8);
  const size_t o_ec = cv.take((size_t)Kf * 4);
  // staged events per block, per instance: scaled with the block's share of
  // (user, knapsack) pairs as in the single-instance sweep (a block of a large
  // instance that overflows its staging costs the whole batch another pass)
  std::vector<uint32_t> scap(n);
  std::vector<size_t> soff(n + 1, 0);
  for (int s = 0; s < n; ++s) {
    const int nb = boff[s + 1] - boff[s];
    const double share = (double)P[s].pr.N * P[s].pr.K / std::max(1, nb) / 64.0;
    scap[s] = (uint32_t)std::min<double>(kStageCapMax, std::max<double>(kStageCap, share));
    soff[s + 1] = soff[s] + (size_t)nb * scap[s];
  }
  const size_t o_s1 = cv.take(soff[n] * 8);
  const size_t o_s2 = cv.take(soff[n] * 8);
  const size_t o_sk = cv.take(soff[n] * 2);
  const size_t o_err = cv.take(8);
  const size_t o_pend = cv.take(8);
  const size_t o_kin = cv.take((size_t)Kf * 4);
  const size_t o_klo = cv.take((size_t)Kf * 4);
  const size_t o_lt0 = cv.take((size_t)n * 8);
  const size_t o_lt1 = cv.take((size_t)n * 8);
  const size_t o_tab0 = cv.take((size_t)ncol * kp_coldesc_size());
  const size_t o_tab1 = cv.take((size_t)ncol * kp_coldesc_size());
  const size_t o_stat = cv.take((size_t)ncol * 8);
  const size_t o_hint = cv.take((size_t)Kf * 32);  // per knapsack: bucket width, last step, two past multipliers
  const size_t o_koff = cv.take((size_t)(n + 1) * 4);
  const size_t o_act = cv.take((size_t)n * 4);
  const size_t o_rd = cv.take((size_t)n * sizeof(SweepArgs));
  const size_t o_rg = cv.take((size_t)n * sizeof(TileGeom));
  const size_t o_rbo = cv.take((size_t)(n + 1) * 4);
  // tables of the device-side split (whole-iteration graphs)
  const size_t o_dhd0 = cv.take((size_t)n * sizeof(SweepArgs));
  const size_t o_dhd1 = cv.take((size_t)n * sizeof(SweepArgs));
  const size_t o_dhg = cv.take((size_t)n * sizeof(TileGeom));
  const size_t o_dord = cv.take((size_t)n * 4);
  const size_t o_dnt = cv.take((size_t)n * 8);
  const size_t o_dpr = cv.take((size_t)n * 8);
  const size_t o_ctl = cv.take(16);
  if (c->max_ws && cv.off > c->max_ws) {
    plan_free(p);
    return fail(KP_ERR_NOMEM, "batched plan needs %zu bytes, above the context cap", cv.off);
  }
  if (hipMalloc(&p->ws, cv.off) != hipSuccess) {
    p->ws = nullptr;
    plan_free(p);
    return fail(KP_ERR_NOMEM, "hipMalloc of %zu plan bytes failed", cv.off);
  }
  if (hipHostMalloc((void **)&p->pinned, 64 + (size_t)n * 4, hipHostMallocDefault) != hipSuccess) {
    p->pinned = nullptr;
    plan_free(p);
    return fail(KP_ERR_HIP, "hipHostMalloc failed");
  }
  if (hipHostMalloc((void **)&p->up, (size_t)n * (sizeof(SweepArgs) + sizeof(TileGeom)) + (size_t)(n + 1) * 4,
                    hipHostMallocDefault) != hipSuccess) {
    p->up = nullptr;
    plan_free(p);
    return fail(KP_ERR_HIP, "hipHostMalloc failed");
  }
  p->ws_bytes = cv.off;
  char *w = (char *)p->ws;
  for (int d = 0; d < 2; ++d) for (int f = 0; f < 2; ++f) p->d[d][f] = (SweepArgs *)(w + o_d[d][f]);
  p->geom = (TileGeom *)(w + o_geom);
  p->boff = (int *)(w + o_boff);
  p->kst = (KState *)(w + o_st);
  p->hint = (double *)(w + o_hint);
  p->eoff = (uint64_t *)(w + o_eo);
  p->ecap = (uint32_t *)(w + o_ec);
  p->window = c->window_enabled;
  if (hipMemset(p->hint, 0, (size_t)Kf * 16) != hipSuccess ||
      hipMemset(p->hint + 2 * (size_t)Kf, 0xFF, (size_t)Kf * 16) != hipSuccess) {
    plan_free(p);
    return fail(KP_ERR_HIP, "hipMemset failed");
  }
  p->Bf = (double *)(w + o_B);
  p->hs = (XSum *)(w + o_hs);
  p->hc = (uint32_t *)(w + o_hc);
  p->e1 = (double *)(w + o_e1);
  p->e2 = (double *)(w + o_e2);
  p->err = (unsigned long long *)(w + o_err);
  p->pend = (int *)(w + o_pend);
  p->kin = (int *)(w + o_kin);
  p->klo = (int *)(w + o_klo);
  p->lam_tab[0] = w + o_lt0;
  p->lam_tab[1] = w + o_lt1;
  p->coltab[0] = w + o_tab0;
  p->coltab[1] = w + o_tab1;
  p->stats = (double *)(w + o_stat);
  p->koff = (int *)(w + o_koff);
  p->active = (int *)(w + o_act);
  p->rd = (SweepArgs *)(w + o_rd);
  p->rg = (TileGeom *)(w + o_rg);
  p->rboff = (int *)(w + o_rbo);
  p->dhd[0] = (SweepArgs *)(w + o_dhd0);
  p->dhd[1] = (SweepArgs *)(w + o_dhd1);
  p->dhg = (TileGeom *)(w + o_dhg);
  p->dord = (int *)(w + o_dord);
  p->dnt = (int64_t *)(w + o_dnt);
  p->dpairs = (double *)(w + o_dpr);
  p->ctl = (int *)(w + o_ctl);
  p->s1 = (double *)(w + o_s1);
  p->s2 = (double *)(w + o_s2);
  p->sk = (uint16_t *)(w + o_sk);
  p->stage_total = soff[n];
  p->gmax = gmax;
  p->ntiles.resize(n);
  p->pairs.resize(n);
  p->ilds.resize(n);
  for (int s = 0; s < n; ++s) {
    p->ntiles[s] = P[s].ntiles;
    p->pairs[s] = (double)P[s].pr.N * P[s].pr.K;
    p->ilds[s] = kp_sweep_lds_bytes(P[s].U, P[s].pr.M, P[s].pr.K, true, P[s].pr.fmt);
  }
  std::vector<SweepArgs> hd[2][2];
  for (int d = 0; d < 2; ++d) for (int f = 0; f < 2; ++f) hd[d][f].resize(n);
  std::vector<TileGeom> hg(n);
  std::vector<double> hB(Kf);
  std::vector<int> kin(Kf), klo(Kf);
  std::vector<uint64_t> heo(Kf);
  std::vector<uint32_t> hec(Kf);
  std::vector<const double *> lt0(n), lt1(n);
  std::vector<unsigned char> tab0((size_t)ncol * kp_coldesc_size()), tab1(tab0.size());
  size_t so = 0;
  int col_i = 0;
  for (int s = 0; s < n; ++s) {
    const int K = P[s].pr.K, nb = boff[s + 1] - boff[s];
    SweepArgs a;
    memset(&a, 0, sizeof a);
    a.pr = P[s].pr;
    a.tree = P[s].tree;
    a.ntiles = P[s].ntiles;
    a.partials = (double *)(w + o_part) + poff[s];
    a.st = p->kst + koff[s];
    a.hist_sum = p->hs + (size_t)koff[s] * KP_NB;
    a.hist_cnt = p->hc + (size_t)koff[s] * KP_NB;
    a.emit_v1 = p->e1 + ioff[s];
    a.emit_v2 = p->e2 + ioff[s];
    a.emit_cap = icap[s];
    a.stage_v1 = (double *)(w + o_s1) + soff[s];
    a.stage_v2 = (double *)(w + o_s2) + soff[s];
    a.stage_k = (uint16_t *)(w + o_sk) + soff[s];
    a.stage_cap = scap[s];
    a.err = p->err;
    for (int d = 0; d < 2; ++d) {
      a.lam = d == 0 ? lam_a[s] : lam_b[s];
      a.want_stats = 1;
      hd[d][1][s] = a;
      a.want_stats = 0;
      hd[d][0][s] = a;
    }
    hg[s] = kp_tile_geom(hd[0][1][s], P[s].U);
    for (int k = 0; k < K; ++k) {
      hB[koff[s] + k] = P[s].B[k];
      kin[koff[s] + k] = s;
      klo[koff[s] + k] = k;
      heo[koff[s] + k] = ioff[s] + (uint64_t)k * icap[s];
      hec[koff[s] + k] = icap[s];
    }
    lt0[s] = lam_a[s];
    lt1[s] = lam_b[s];
    // statistics of the first pass are at the direction's input lambda
    for (int cc = 0; cc < K + 2; ++cc) {
      kp_coldesc_fill(tab0.data() + (size_t)col_i * kp_coldesc_size(), hd[0][1][s].partials, lam_a[s],
                      p->Bf + koff[s], p->stats + so + cc, P[s].ntiles ? nb : 0, K, cc);
      kp_coldesc_fill(tab1.data() + (size_t)col_i * kp_coldesc_size(), hd[0][1][s].partials, lam_b[s],
                      p->Bf + koff[s], p->stats + so + cc, P[s].ntiles ? nb : 0, K, cc);
      ++col_i;
    }
    so += (size_t)K + 2;
  }
  hipStream_t st = c->stream;
  auto up = [&](void *dst, const void *src, size_t bytes) { return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st); };
  hipError_t e = hipSuccess;
  // block layout: instances with the costliest tiles first, so that their
  // blocks start early and cheap ones fill the tail of the launch; every
  // table indexed by position follows the same order
  std::vector<int> ord(n);
  for (int s = 0; s < n; ++s) ord[s] = s;
  auto tile_cost = [&](int s) {
    const Prepared &q = P[s];
    const double c1 = q.tree.L == 1 ? (double)q.tree.cap[0] : (double)q.pr.M;
    return (double)q.U * q.pr.M * q.pr.K * (1.0 + c1);
  };
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return tile_cost(x) > tile_cost(y); });
  std::vector<int> bpos(n + 1, 0);
  std::vector<SweepArgs> pd[2][2];
  std::vector<TileGeom> pg(n);
  for (int d = 0; d < 2; ++d) for (int f = 0; f < 2; ++f) pd[d][f].resize(n);
  for (int i = 0; i < n; ++i) {
    const int si = ord[i];
    bpos[i + 1] = bpos[i] + (boff[si + 1] - boff[si]);
    for (int d = 0; d < 2; ++d) for (int f = 0; f < 2; ++f) pd[d][f][i] = hd[d][f][si];
    pg[i] = hg[si];
  }
  for (int d = 0; d < 2 && e == hipSuccess; ++d)
    for (int f = 0; f < 2 && e == hipSuccess; ++f) e = up(p->d[d][f], pd[d][f].data(), (size_t)n * sizeof(SweepArgs));
  if (e == hipSuccess) e = up(p->geom, pg.data(), (size_t)n * sizeof(TileGeom));
  if (e == hipSuccess) e = up(p->boff, bpos.data(), (size_t)(n + 1) * 4);
  if (e == hipSuccess) e = up(p->koff, koff.data(), (size_t)(n + 1) * 4);
  if (e == hipSuccess) e = up(p->Bf, hB.data(), (size_t)Kf * 8);
  if (e == hipSuccess) e = up(p->kin, kin.data(), (size_t)Kf * 4);
  if (e == hipSuccess) e = up(p->klo, klo.data(), (size_t)Kf * 4);
  if (e == hipSuccess) e = up(p->eoff, heo.data(), (size_t)Kf * 8);
  if (e == hipSuccess) e = up(p->ecap, hec.data(), (size_t)Kf * 4);
  if (e == hipSuccess) e = up(p->lam_tab[0], lt0.data(), (size_t)n * 8);
  if (e == hipSuccess) e = up(p->lam_tab[1], lt1.data(), (size_t)n * 8);
  if (e == hipSuccess) e = up(p->coltab[0], tab0.data(), tab0.size());
  if (e == hipSuccess) e = up(p->coltab[1], tab1.data(), tab1.size());
  if (e == hipSuccess) e = up(p->dhd[0], hd[0][0].data(), (size_t)n * sizeof(SweepArgs));
  if (e == hipSuccess) e = up(p->dhd[1], hd[1][0].data(), (size_t)n * sizeof(SweepArgs));
  if (e == hipSuccess) e = up(p->dhg, hg.data(), (size_t)n * sizeof(TileGeom));
  if (e == hipSuccess) e = up(p->dord, ord.data(), (size_t)n * 4);
  if (e == hipSuccess) e = up(p->dnt, p->ntiles.data(), (size_t)n * 8);
  if (e == hipSuccess) e = up(p->dpairs, p->pairs.data(), (size_t)n * 8);
  if (e == hipSuccess) e = hipMemsetAsync(p->ctl, 0, 16, st);
  if (e == hipSuccess) e = hipMemsetAsync(p->hs, 0, (size_t)Kf * KP_NB * sizeof(XSum), st);
  if (e == hipSuccess) e = hipMemsetAsync(p->hc, 0, (size_t)Kf * KP_NB * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(p->err, 0, 8, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables go out of scope
  if (e != hipSuccess) {
    plan_free(p);
    return fail(KP_ERR_HIP, "plan upload failed: %s", hipGetErrorString(e));
  }
  for (int d = 0; d < 2; ++d) p->hd[d] = hd[d][0];
  p->hg = hg;
  p->order = ord;
  // whole-iteration graphs hold this many later passes split on the device
  // (a split's blocks never exceed max(n, gmax) + 2n); further passes, rare,
  // run from the host
  p->glater = kp_resplit_lds(n) ? kGraphLaterPasses : 0;
  p->gfix = std::max(n, gmax) + 2 * n;
  *out = p;
  return KP_OK;
}

kp_status kp_batched_create(void *ctx, const kp_problem *probs, int32_t n, const double *const *lam_a,
                            double *const *lam_b, void **plan_out) {
  if (!ctx || !plan_out) return fail(KP_ERR_INVALID, "NULL argument");
  BatchPlan *p = nullptr;
  kp_status st = plan_create((Ctx *)ctx, probs, n, lam_a, lam_b, &p);
  if (st != KP_OK) return st;
  *plan_out = p;
  return KP_OK;
}

kp_status kp_batched_step(void *plan, int32_t dir, double *stats, int32_t use_graph) {
  if (!plan || (dir != 0 && dir != 1)) return fail(KP_ERR_INVALID, "bad plan or direction");
  return plan_step((BatchPlan *)plan, dir, stats, use_graph != 0);
}

kp_status kp_batched_shape(void *plan, int32_t *blocks, int32_t *lds_bytes, int32_t *min_users_per_tile,
                           int32_t *max_users_per_tile) {
  if (!plan) return fail(KP_ERR_INVALID, "plan is NULL");
  const BatchPlan *p = (const BatchPlan *)plan;
  if (blocks) *blocks = p->GB;
  if (lds_bytes) *lds_bytes = (int32_t)p->lds;
  if (min_users_per_tile) *min_users_per_tile = p->Umin;
  if (max_users_per_tile) *max_users_per_tile = p->Umax;
  return KP_OK;
}

kp_status kp_batched_destroy(void *plan) {
  plan_free((BatchPlan *)plan);
  return KP_OK;
}

kp_status kp_eval_dual_noalloc(void *hip_stream, const kp_problem *prob, const double *lambda,
                               double *R, double *g, double *primal, uint8_t *x) {
  if (!lambda || !R || !g || !primal) return fail(KP_ERR_INVALID, "lambda, R, g and primal must not be NULL");
  Prepared P;
  kp_status s = prepare(prob, false, P, nullptr);
  if (s != KP_OK) return s;
  const int K = P.pr.K;
  // scratch layout: budgets [K], then one [K + 2] row of partial sums per block
  const size_t off_part = ((size_t)K * 8 + 255) & ~(size_t)255;
  const size_t row = (size_t)(K + 2) * 8;
  if (off_part + row > KP_NOALLOC_SCRATCH)
    return fail(KP_ERR_UNSUPPORTED, "K = %d needs more than the %u scratch bytes of kp_eval_dual_noalloc", K,
                (unsigned)KP_NOALLOC_SCRATCH);
  const int max_grid = (int)std::min<size_t>((KP_NOALLOC_SCRATCH - off_part) / row, (size_t)1 << 30);
  void *scr = nullptr;
  if ((s = noalloc_scratch(&scr)) != KP_OK) return s;
  double *Bd = (double *)scr;
  double *partials = (double *)((char *)scr + off_part);
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipMemcpyAsync(Bd, P.B, (size_t)K * 8, hipMemcpyHostToDevice, st));
  if (P.pr.N == 0) {
    HIP_TRY(kp_launch_fill_f64(partials, K + 2, 0.0, st));
    HIP_TRY(kp_launch_reduce_stats(partials, 1, K, lambda, Bd, R, g, primal, st));
    return KP_OK;
  }
  SweepArgs a;
  memset(&a, 0, sizeof(a));
  a.pr = P.pr;
  a.tree = P.tree;
  a.lam = lambda;
  a.want_stats = 1;
  a.partials = partials;
  a.x_out = x;
  int used = 0;
  const bool ell = P.row_nnz && P.pr.M <= 16 &&
                   kp_ell_lds_bytes(P.pr.M, K, P.row_nnz, P.tree.L, 0, nullptr) <= kMaxLds;
  if (ell) {
    a.ntiles = (P.pr.N + 63) / 64;
    const int res = kp_ell_resident_grid(P.row_nnz, 0, P.pr.M, K, P.tree.L);
    if (res <= 0) return fail(KP_ERR_HIP, "occupancy query failed");
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((a.ntiles + 3) / 4,
                                                                   std::min(std::min(res, kEllGrid), max_grid)));
    HIP_TRY(kp_launch_ell(a, P.row_nnz, grid, 0, st, &used));
  } else {
    a.ntiles = P.ntiles;
    HIP_TRY(kp_launch_sweep(a, P.U, std::min(P.grid, max_grid), false, st, &used));
  }
  HIP_TRY(kp_launch_reduce_stats(partials, used, K, lambda, Bd, R, g, primal, st));
  return KP_OK;
}

kp_status kp_scd_sweep_batched(void *ctx, const kp_problem *probs, int32_t n,
                               const double *const *lambda_in, double *const *lambda_out,
                               double *stats) {
  if (!ctx) return fail(KP_ERR_INVALID, "ctx is NULL");
  BatchPlan *p = nullptr;
  kp_status st = plan_create((Ctx *)ctx, probs, n, lambda_in, lambda_out, &p);
  if (st != KP_OK) return st;
  st = plan_step(p, 0, stats, false);
  plan_free(p);
  return st;
}

}  // extern "C"
