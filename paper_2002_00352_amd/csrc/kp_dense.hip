// Lane-per-user evaluation of dense costs with few items and knapsacks
// (M <= 16, K <= 16): the dual evaluation of Eq.5 with Alg.1 per user.
//
// One wave owns a tile of 48 users at a time, one lane per user, and a block
// is one wave, so blocks pack as tightly as the LDS of one tile allows.  The
// tile's profits [TU][M] and costs [TU][M][K] (contiguous in the ABI layout)
// are staged with coalesced direct-to-LDS loads; every lane then scores its
// user (FP64, knapsacks ascending, a product then a subtraction: the sweep's
// arithmetic), ranks its items by (p~ desc, index asc), runs Alg.1 in rank
// space (bit r of a mask is the item of rank r; every laminar set, subsets
// first, keeps its cap best live members) and adds its consumption of every
// knapsack, its profit and its group dual value to running sums of its own
// (registers, tile after tile); the wave sums them in a fixed butterfly
// order once, at the end, and a second kernel adds the blocks in order.  No
// barrier or cross-lane step inside the tile loop.
#include <type_traits>
#include "kp_ell_impl.h"

// users per tile (lanes past it stay idle): a smaller tile holds less LDS,
// so more waves fit on a compute unit to hide the loads' latency (c2 DD:
// 64 users 1.18 ms, 56 1.17, 48 1.13, 32 1.96)
#ifndef KP_DENSE_TU
#define KP_DENSE_TU 48
#endif

namespace {

constexpr int TU = KP_DENSE_TU;
static_assert(TU % 4 == 0 && TU <= 64, "users per tile: a multiple of 4, at most a wave");

__host__ __device__ inline size_t dn_r16(size_t b) { return (b + 15) & ~(size_t)15; }

// LDS of one block: lambda [K], the sets' masks and caps, one tile
__host__ __device__ inline size_t dn_lds(int M, int K, int L) {
  return dn_r16((size_t)K * 8) + dn_r16((size_t)L * 8 + 8) + dn_r16((size_t)L * 4 + 4) +
         dn_r16((size_t)TU * M * 4) + (size_t)TU * M * K * 4;
}

// EM: the item-count class (8, 10, 12, 16), M <= EM; EK: 16, the bound of
// the knapsack count (the per-lane sums; the scoring loops run to K).
// (Unrolling the scoring over a compile-time knapsack class, lambda in
// registers, measured slower: 1.30 against 1.19 ms on c2.)
template <int EM, int EK>
__global__ void __launch_bounds__(64) k_dense_eval(const SweepArgs a, int x4) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int M = a.pr.M, K = a.pr.K, L = a.tree.L;
  double *lam = (double *)smem;
  uint64_t *tmask = (uint64_t *)(smem + dn_r16((size_t)K * 8));
  int *tcap = (int *)((unsigned char *)tmask + dn_r16((size_t)L * 8 + 8));
  float *sp = (float *)((unsigned char *)tcap + dn_r16((size_t)L * 4 + 4));   // [TU][M]
  float *sb = (float *)((unsigned char *)sp + dn_r16((size_t)TU * M * 4));    // [TU][M][K]
  for (int t = lane; t < K; t += 64) lam[t] = a.lam[t];
  for (int t = lane; t < L; t += 64) { tmask[t] = a.tree.mask[t]; tcap[t] = a.tree.cap[t]; }
  __syncthreads();
  const int64_t N = a.pr.N;
  double accR[EK];   // this lane's users: consumption of knapsack q (q < K)
  #pragma unroll
  for (int q = 0; q < EK; ++q) accR[q] = 0.0;
  double accG = 0.0, accP = 0.0;
  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t u0 = tile * TU;
    const int nu = (int)((N - u0) < TU ? (N - u0) : TU);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    // 16-byte copies of a full tile (TU a multiple of 4: every tile starts
    // 16-byte aligned when the arrays do)
    if (nu == TU && x4) {
      stage_x4(a.pr.p + u0 * M, 4 * TU * M, sp, lane);
      stage_x4(a.pr.b + u0 * M * K, 4 * TU * M * K, sb, lane);
    } else {
      stage_dwords(a.pr.p + u0 * M, nu * M, sp, lane);
      stage_dwords(a.pr.b + u0 * M * K, nu * M * K, sb, lane);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    // lanes past the end of the last tile read whatever the staging area
    // holds; they select nothing and add zeros (lanes past the tile read row
    // 0 again)
    const bool act = lane < nu;
    const int row = lane < TU ? lane : 0;
    const float *pl = sp + row * M;
    const float *bl = sb + (size_t)row * M * K;
    // ---- cost-adjusted profits ----
    double pt[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      double acc = 0.0;
      if (j < M) {
        acc = (double)pl[j];
        const float *br = bl + j * K;
        for (int k = 0; k < K; ++k) {
          const double prod = lam[k] * (double)br[k];
          acc = acc - prod;
        }
      }
      pt[j] = acc;
    }
    // ---- ranks by (p~ desc, index asc) ----
    int rk[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) rk[j] = j;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      #pragma unroll
      for (int jj = j + 1; jj < EM; ++jj) {
        if (jj < M) {
          const int c = pt[jj] > pt[j] ? 1 : 0;
          rk[j] += c;
          rk[jj] -= c;
        }
      }
    }
    // ---- Alg.1's cap pass in rank space ----
    uint32_t rbit[EM];
    uint32_t alive = 0;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      rbit[j] = j < M ? 1u << rk[j] : 0u;
      if (j < M && pt[j] > 0.0) alive |= rbit[j];
    }
    if (!act) alive = 0;
    for (int l = 0; l < L; ++l) {
      const uint32_t m = (uint32_t)tmask[l];
      uint32_t mr = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j)
        if (m >> j & 1u) mr |= rbit[j];
      uint32_t x = alive & mr;
      for (int c = 0; c < tcap[l]; ++c) x &= x - 1u;
      alive &= ~x;
    }
    uint32_t S = 0;
    #pragma unroll
    for (int j = 0; j < EM; ++j)
      if (alive & rbit[j]) S |= 1u << j;
    // ---- outputs and statistics (sums over the selected items, index order) ----
    if (a.x_out && act) {
      uint8_t *xo = a.x_out + (u0 + lane) * M;
      for (int j = 0; j < M; ++j) xo[j] = (uint8_t)(S >> j & 1u);
    }
    if (a.want_stats) {
      double Pi = 0.0, Gi = 0.0;
      #pragma unroll
      for (int j = 0; j < EM; ++j)
        if (S >> j & 1u) { Pi = Pi + (double)pl[j]; Gi = Gi + pt[j]; }
      accG = accG + Gi;
      accP = accP + Pi;
      #pragma unroll
      for (int q = 0; q < EK; ++q) {
        if (q < K) {
          double v = 0.0;
          for (uint32_t m = S; m; m &= m - 1u) v = v + (double)bl[(__ffs((int)m) - 1) * K + q];
          accR[q] = accR[q] + v;
        }
      }
    }
  }
  if (a.want_stats) {
    double mine = 0.0;   // lane q < K + 2: column q of the block
    #pragma unroll
    for (int q = 0; q < EK; ++q) {
      if (q < K) {
        const double s = wave_sum(accR[q]);
        if (lane == q) mine = s;
      }
    }
    const double sg = wave_sum(accG);
    if (lane == K) mine = sg;
    const double sq = wave_sum(accP);
    if (lane == K + 1) mine = sq;
    if (lane < K + 2) a.partials[(size_t)blockIdx.x * (K + 2) + lane] = mine;
  }
}

template <int EM, int EK>
hipError_t launch_dense_t(const SweepArgs &a, size_t lds, int grid, int x4, hipStream_t stream, int *used) {
  const void *fn = (const void *)k_dense_eval<EM, EK>;
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  const int resident = per_cu * cus;
  if (grid <= 0 || grid > resident) grid = resident;
  if (used) *used = grid;
  hipLaunchKernelGGL((k_dense_eval<EM, EK>), dim3(grid), dim3(64), lds, stream, a, x4);
  return hipGetLastError();
}

template <int EM, int EK>
int resident_dense_t(size_t lds) {
  const void *fn = (const void *)k_dense_eval<EM, EK>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// call f(EM, EK) with the item-count class of M and EK = 16
template <class F>
auto dispatch_dense_k(int K, F f) {
  (void)K;
  return f(std::integral_constant<int, 16>());
}
template <class F>
auto dispatch_dense(int M, int K, F f) {
  if (M <= 8) return dispatch_dense_k(K, [&](auto ek) { return f(std::integral_constant<int, 8>(), ek); });
  if (M <= 10) return dispatch_dense_k(K, [&](auto ek) { return f(std::integral_constant<int, 10>(), ek); });
  if (M <= 12) return dispatch_dense_k(K, [&](auto ek) { return f(std::integral_constant<int, 12>(), ek); });
  return dispatch_dense_k(K, [&](auto ek) { return f(std::integral_constant<int, 16>(), ek); });
}

}  // namespace

int kp_dense_tile_users() { return TU; }

// Evaluation (statistics into a.partials [grid][K + 2] and/or x) over
// a.ntiles tiles of kp_dense_tile_users() users.  grid: an upper bound (the size of the
// per-block buffers); *used receives the blocks launched (at most the
// resident ones).
hipError_t kp_launch_dense(const SweepArgs &a, int grid, hipStream_t stream, int *used) {
  const int M = a.pr.M, K = a.pr.K;
  if (a.pr.fmt != 0 || M < 1 || M > 16 || K < 1 || K > 16 || a.tree.L < 0) return hipErrorInvalidValue;
  const size_t lds = dn_lds(M, K, a.tree.L);
  const int x4 = (((uintptr_t)a.pr.p | (uintptr_t)a.pr.b) & 15) == 0;
  return dispatch_dense(M, K, [&](auto em, auto ek) {
    return launch_dense_t<decltype(em)::value, decltype(ek)::value>(a, lds, grid, x4, stream, used);
  });
}

// Blocks of the dense evaluation that can be resident at once; 0 when the
// shape is outside the kernel's range or the query fails.
int kp_dense_resident_grid(int M, int K, int L) {
  if (M < 1 || M > 16 || K < 1 || K > 16) return 0;
  const size_t lds = dn_lds(M, K, L);
  return dispatch_dense(M, K, [&](auto em, auto ek) {
    return resident_dense_t<decltype(em)::value, decltype(ek)::value>(lds);
  });
}
