// Host entry points of the lean sweep kernel (kp_ell_impl.h): LDS sizing,
// dispatch to the per-mode instantiations, and the uniform-row check.
#include <algorithm>
#include <vector>
#include "kp_ell_impl.h"

static size_t ell_lds(int M, int K, int D, int L, int mode, int waves, int *region_out) {
  auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  const bool brk = mode == KM_SCD || mode == KM_WFAIL;
  size_t region = 0;
  if (mode != KM_WFAIL) {
    // staged tile, plus slack for the reads of up to 16 items per lane past
    // the last lane's row
    region = (size_t)64 * M * 4 + (size_t)64 * M * D * 8 + (size_t)16 * D * 4;
    region = region > (size_t)8 * 65 * 8 ? region : (size_t)8 * 65 * 8;      // statistics rows
    if (mode == KM_WMAIN && region < (size_t)64 * M * 12) region = (size_t)64 * M * 12;  // filter: p~ and bounds by rank
  }
  if (brk) {
    const size_t need = (size_t)ell_scratch(M, D, K).end;                     // p~, costs, masks
    region = region > need ? region : need;
  }
  region = r16(region);
  const int ew = waves;
  size_t s = r16((size_t)(K + 1) * 8) + r16((size_t)L * 8 + 8) + r16((size_t)L * 4 + 4) +
             r16((size_t)ew * (K + 2) * 8);
  if (mode != KM_EVAL && mode != KM_FIX) s += r16((size_t)K * 4) + r16((size_t)K * 8 + 16);
  if (mode == KM_WMAIN) s += r16((size_t)(K + 1) * sizeof(LamW));
  if (brk)   // (the listed users' pass of a window pass bins nothing: no histograms)
    s += r16((size_t)K * sizeof(XSum)) + r16((size_t)K * sizeof(KState)) +
         (mode == KM_SCD ? r16((size_t)K * KP_NB * sizeof(XSum)) + r16((size_t)K * KP_NB * 4) : 0) +
         3 * r16((size_t)K * 4) + 2 * r16((size_t)K * 8) + r16(16);
  s += (size_t)ew * region;
  if (region_out) *region_out = (int)region;
  return s;
}

// Waves per block of a mode: 8 for the full-search pass of the kernels
// instantiated for the exact item count when its LDS fits, else 4 (with 8
// waves a block may hold 256 registers per lane, and the kernels for a
// class of item counts would spill).
int kp_ell_waves(int M, int K, int D, int L, int mode) {
  const bool exact = M == 8 || M == 10 || M == 12 || M == 16;
  if (mode == KM_SCD && exact && ell_lds(M, K, D, L, mode, 8, nullptr) <= (size_t)160 * 1024) return 8;
  return EW;
}

size_t kp_ell_lds_bytes(int M, int K, int D, int L, int mode, int *region_out) {
  return ell_lds(M, K, D, L, mode, kp_ell_waves(M, K, D, L, mode), region_out);
}

// Rank of the laminar matroid on M items (the most items any feasible x_i
// selects): every set (subsets first) holds min(cap, its items outside its
// maximal subsets + their ranks); items in no set count one each.
int laminar_rank(const TreeDev &t, int M) {
  std::vector<int> r(t.L, 0);
  std::vector<char> inner(t.L, 0);   // contained in a later (larger) set
  for (int l = 0; l < t.L; ++l) {
    uint64_t covered = 0;
    int sum = 0;
    for (int c = 0; c < l; ++c) {
      if (inner[c] || (t.mask[c] & ~t.mask[l]) != 0) continue;   // not a maximal subset of l
      covered |= t.mask[c];
      sum += r[c];
      inner[c] = 1;
    }
    sum += __builtin_popcountll(t.mask[l] & ~covered);
    r[l] = std::min(t.cap[l], sum);
  }
  uint64_t covered = 0;
  int total = 0;
  for (int l = 0; l < t.L; ++l)
    if (!inner[l]) { covered |= t.mask[l]; total += r[l]; }
  const uint64_t all = M >= 64 ? ~0ull : ((1ull << M) - 1);
  return total + __builtin_popcountll(all & ~covered);
}

// mode: 0 evaluation, 1 full SCD pass, 2 window main pass, 3 listed users of a window pass,
// 4 evaluation with the post-processing bins (a.fx).
// grid is an upper bound (the size of the per-block buffers); *used receives
// the grid launched (the blocks that can be resident at once, at most grid).
hipError_t kp_launch_ell(const SweepArgs &a, int D, int grid, int mode, hipStream_t stream, int *used) {
  EllGeom g;
  g.M = a.pr.M;
  g.K = a.pr.K;
  if (g.M < 1 || g.M > 16 || (D != 1 && D != 2) || mode < 0 || mode > 4) return hipErrorInvalidValue;
  if (a.ntiles > 0x7fffffffLL) return hipErrorInvalidValue;  // the kernel's tile indices are 32-bit
  if ((mode == KM_FIX) != (a.fx.bin != nullptr)) return hipErrorInvalidValue;
  size_t lds = kp_ell_lds_bytes(g.M, g.K, D, a.tree.L, mode, &g.region);
  if (mode == KM_FIX) {
    // post-processing bins: slot map, splitters, bin sums and counts
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    lds += r16((size_t)g.K * 4) + r16((size_t)a.fx.nb * 8) + r16((size_t)a.fx.nb * a.fx.nv * sizeof(XSum)) +
           r16((size_t)a.fx.nb * 4);
  }
  g.rows = g.region / (65 * 8);
  if (g.rows > g.K + 2) g.rows = g.K + 2;
  g.x4 = (((uintptr_t)a.pr.p | (uintptr_t)a.pr.col | (uintptr_t)a.pr.val) & 15) == 0;
  g.compact = laminar_rank(a.tree, g.M) <= KP_SEL_MAX;
  g.waves = kp_ell_waves(g.M, g.K, D, a.tree.L, mode);
  switch (mode) {
    case KM_EVAL: return kp_launch_ell_mode<KM_EVAL>(a, g, lds, grid, D, stream, used);
    case KM_SCD: return kp_launch_ell_mode<KM_SCD>(a, g, lds, grid, D, stream, used);
    case KM_WMAIN: return kp_launch_ell_mode<KM_WMAIN>(a, g, lds, grid, D, stream, used);
    case KM_FIX: return kp_launch_ell_mode<KM_FIX>(a, g, lds, grid, D, stream, used);
    default: return kp_launch_ell_mode<KM_WFAIL>(a, g, lds, grid, D, stream, used);
  }
}

// Blocks of the given mode that can be resident on the device at once (the
// grid kp_launch_ell launches at most); 0 when the query fails.
int kp_ell_resident_grid(int D, int mode, int M, int K, int L) {
  if (M < 1 || M > 16 || (D != 1 && D != 2) || mode < 0 || mode > 3) return 0;
  const size_t lds = kp_ell_lds_bytes(M, K, D, L, mode, nullptr);
  const int w = kp_ell_waves(M, K, D, L, mode);
  switch (mode) {
    case KM_EVAL: return kp_ell_resident_mode<KM_EVAL>(D, M, lds, w);
    case KM_SCD: return kp_ell_resident_mode<KM_SCD>(D, M, lds, w);
    case KM_WMAIN: return kp_ell_resident_mode<KM_WMAIN>(D, M, lds, w);
    default: return kp_ell_resident_mode<KM_WFAIL>(D, M, lds, w);
  }
}

// row r's entries start at r*D for every row (and row 0 at 0)
__global__ void k_ell_check(const int64_t *rowptr, int64_t nrows, int D, unsigned int *bad) {
  unsigned int b = 0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= nrows;
       r += (int64_t)gridDim.x * blockDim.x)
    b |= rowptr[r] != r * (int64_t)D;
  if (b) atomicOr(bad, 1u);
}

hipError_t kp_launch_ell_check(const int64_t *rowptr, int64_t nrows, int D, unsigned int *bad,
                               hipStream_t stream) {
  int64_t blocks = (nrows + 1 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_ell_check, dim3((unsigned)blocks), dim3(256), 0, stream, rowptr, nrows, D, bad);
  return hipGetLastError();
}
