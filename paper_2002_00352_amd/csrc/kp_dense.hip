// Lane-per-user evaluation of dense costs with few items and knapsacks
// (M <= 16, K <= 16): the dual evaluation of Eq.5 with Alg.1 per user, and
// the SCD window pass built on it.
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
//
// The SCD window pass (Sec. 5.2's threshold search, every open search with a
// window around lambda_k^t) adds to the evaluation, per lane and per window
// knapsack, a gap test: the user has no breakpoint in the window when every
// line moving with k is farther than h_k b_jk (plus a rounding margin) from
// its rank neighbours and from zero.  The (user, knapsack) pairs it leaves
// open are dealt over the wave and walked exactly through the owner's LDS
// column (the uniform-row kernel's walk); breakpoints inside the window are
// staged per block and corrections C_ik(whi+) - v_ik added exactly.
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

// LDS of one block: lambda [K], the sets' masks and caps, one tile; the
// window pass adds the search states, its per-block event staging counters
// and corrections, and the lanes' p~ columns [M][64] read by the walks.
__host__ __device__ inline size_t dn_lds(int M, int K, int L, bool win) {
  size_t s = dn_r16((size_t)K * 8) + dn_r16((size_t)L * 8 + 8) + dn_r16((size_t)L * 4 + 4) +
             dn_r16((size_t)TU * M * 4) + dn_r16((size_t)TU * M * K * 4);
  if (win)
    s += dn_r16((size_t)K * sizeof(KState)) + dn_r16((size_t)K * 4) + dn_r16((size_t)(K + 1) * 8) +
         dn_r16((size_t)K * sizeof(XSum)) + 3 * dn_r16((size_t)K * 4) + 2 * dn_r16((size_t)K * 8) + dn_r16(16) +
         (size_t)M * 64 * 8;
  return s;
}

// EM: the item-count class (8, 10, 12, 16), M <= EM; EK: 16, the bound of
// the knapsack count (the per-lane sums; the scoring loops run to K).
// KX: the knapsack count when it is fixed at compile time (2 or 10, with M
// equal to EM), else 0: every loop over the knapsacks then has a constant
// trip count and unrolls (c2 DD: 0.94 -> 0.81-0.82 ms).  (Unrolling the
// scoring over the knapsack class instead, each step guarded by k < K and
// lambda in registers, measured slower: 1.12 against 0.94 ms on c2.)
// WIN: the SCD window pass (every knapsack still searching has a window
// around lambda_k^t, Sec. 5.2's threshold search started around its last
// value): after the evaluation, every lane tests its user per window
// knapsack -- calm when every moving item's line is farther than h_k b_jk
// from its rank neighbours and from zero -- and the (user, knapsack) pairs
// left undecided are dealt over the wave and walked exactly (lane_walk_pair).
// EXACT: M equals EM, so every test of an item index against M folds away.
template <int EM, int EK, bool WIN, bool EXACT, int KX>
__global__ void __launch_bounds__(64) k_dense(const SweepArgs a, int x4) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x;
  const int M = EXACT ? EM : a.pr.M, K = KX ? KX : a.pr.K, L = a.tree.L;
  size_t off = 0;
  auto carve = [&](size_t bytes) { unsigned char *p = smem + off; off += dn_r16(bytes); return p; };
  double *lam = (double *)carve((size_t)K * 8);
  uint64_t *tmask = (uint64_t *)carve((size_t)L * 8 + 8);
  int *tcap = (int *)carve((size_t)L * 4 + 4);
  float *sp = (float *)carve((size_t)TU * M * 4);       // [TU][M]
  float *sb = (float *)carve((size_t)TU * M * K * 4);   // [TU][M][K]
  KState *kst = nullptr;
  int *kmode = nullptr;
  double *hwin = nullptr;
  XSum *kcorr = nullptr;
  uint32_t *kcnt = nullptr, *kpos = nullptr, *kovf = nullptr, *nstage = nullptr;
  unsigned long long *hmin = nullptr, *hmax = nullptr;
  double *ptl = nullptr;
  if (WIN) {
    kst = (KState *)carve((size_t)K * sizeof(KState));
    kmode = (int *)carve((size_t)K * 4);
    hwin = (double *)carve((size_t)(K + 1) * 8);   // [K] window half-widths (0: none), [K] their max
    kcorr = (XSum *)carve((size_t)K * sizeof(XSum));
    kcnt = (uint32_t *)carve((size_t)K * 4);
    kpos = (uint32_t *)carve((size_t)K * 4);
    kovf = (uint32_t *)carve((size_t)K * 4);
    hmin = (unsigned long long *)carve((size_t)K * 8);
    hmax = (unsigned long long *)carve((size_t)K * 8);
    nstage = (uint32_t *)carve(16);
    ptl = (double *)carve((size_t)M * 64 * 8);
  }
  for (int t = lane; t < K; t += 64) lam[t] = a.lam[t];
  for (int t = lane; t < L; t += 64) { tmask[t] = a.tree.mask[t]; tcap[t] = a.tree.cap[t]; }
  if (WIN) {
    for (int t = lane; t < K; t += 64) {
      kst[t] = a.st[t];
      kmode[t] = a.st[t].mode;
      hwin[t] = a.st[t].mode == KS_WINDOW ? a.st[t].hw : 0.0;
      kcorr[t] = xs_zero();
      kcnt[t] = 0u; kpos[t] = 0u; kovf[t] = 0u;
      hmin[t] = ~0ull; hmax[t] = 0ull;
    }
    if (lane == 0) *nstage = 0u;
  }
  __syncthreads();
  if (WIN && lane == 0) {
    double m = 0.0;
    for (int k = 0; k < K; ++k) m = hwin[k] > m ? hwin[k] : m;
    hwin[K] = m;
  }
  __syncthreads();
  const int64_t N = a.pr.N;
  double accR[EK];   // this lane's users: consumption of knapsack q (q < K)
  #pragma unroll
  for (int q = 0; q < EK; ++q) accR[q] = 0.0;
  double accG = 0.0, accP = 0.0;
  uint32_t nwalk = 0;   // window pass: users of this wave with a pair to walk
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
    // ---- cost-adjusted profits (window pass: and the largest cost) ----
    double pt[EM];
    float bm = 0.0f;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      double acc = 0.0;
      if (j < M) {
        acc = (double)pl[j];
        const float *br = bl + j * K;
        for (int k = 0; k < K; ++k) {
          const float bv = br[k];
          if (WIN) bm = fmaxf(bm, bv);
          const double prod = lam[k] * (double)bv;
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
    if (WIN) {
      // ---- window tests per knapsack ----
      uint64_t pending = 0, perm = 0, pos = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (j < M) {
          ptl[j * 64 + lane] = pt[j];
          perm |= (uint64_t)j << (4 * rk[j]);
          if (pt[j] > 0.0) pos |= 1ull << j;
        }
      }
      if (!act) pos = 0;
      if (act) {
        // lines below -H (H: the widest window times the user's largest
        // cost) never turn positive in any window; gj: the distance from
        // item j's line to the nearest other line above -H and to zero (its
        // rank neighbours are the nearest lines)
        const double bmax = (double)bm, hm = hwin[K];
        const double H = hm * bmax * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + bmax * hm);
        double top = -INFINITY;
        #pragma unroll
        for (int j = 0; j < EM; ++j)
          if (j < M) top = fmax(top, pt[j]);
        const double gscale = fabs(top) + H;
        // (lines at or below -H are moved to -inf: no finite distance to them)
        double gj[EM], pu[EM];
        bool anyup = false;   // some line can turn positive in some window
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          pu[j] = (j < M && pt[j] > -H) ? pt[j] : -INFINITY;
          gj[j] = pu[j] > -INFINITY ? fabs(pt[j]) : 1e300;
          anyup = anyup | (pu[j] > -INFINITY);
        }
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          #pragma unroll
          for (int jj = j + 1; jj < EM; ++jj) {
            const double d = fabs(pu[j] - pu[jj]);   // inf or NaN (-inf - -inf) unless both are lines
            gj[j] = d < gj[j] ? d : gj[j];
            gj[jj] = d < gj[jj] ? d : gj[jj];
          }
        }
        // (a user without such a line is calm in every window)
        for (int k = 0; anyup && k < K; ++k) {
          if (kmode[k] != KS_WINDOW) continue;
          float bk[EM];
          uint32_t A = 0;
          #pragma unroll
          for (int j = 0; j < EM; ++j) {
            bk[j] = j < M ? bl[j * K + k] : 0.0f;
            if (bk[j] > 0.0f) A |= 1u << j;
          }
          if (!A) continue;   // no moving line: no breakpoint, no consumption
          // every moving item's line must stay farther than h_k b_jk (plus a
          // rounding margin) from its neighbours and from zero (h_k: the
          // distance from lambda_k^t to the window's far edge)
          const double lk = lam[k], h = hwin[k];
          bool calm = true;
          #pragma unroll
          for (int j = 0; j < EM; ++j) {
            if (A >> j & 1) {
              const double b = (double)bk[j];
              const double need = h * b * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + gscale + lk * b + h * b);
              calm = calm & (gj[j] > need);
            }
          }
          if (calm) continue;
          pending |= 1ull << k;
        }
      }
      nwalk += (uint32_t)__popcll(__ballot(pending != 0));
      __builtin_amdgcn_s_waitcnt(0);   // every lane's p~ column is written before any lane reads another's
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
      lane_deal_pairs(lane, pending, (uint64_t)S, pos, perm,
                      [&](int col, int k, uint64_t So, uint64_t poso, uint64_t permo) {
        const float *bc = sb + (size_t)col * M * K + k;   // lane col's costs in k, stride K
        uint64_t A = 0;
        for (int j = 0; j < M; ++j)
          if (bc[j * K] > 0.0f) A |= 1ull << j;
        lane_walk_pair(a, M, L, col, k, A, So, poso, permo,
                       [&](int j, int cc) { return (double)sb[((size_t)cc * M + j) * K + k]; }, ptl, lam, kst,
                       kmode, tmask, tcap, kcorr, nullptr, nullptr, hmin, hmax, kcnt, kovf, nstage);
      });
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
  if (WIN) {
    if (lane == 0 && nwalk && a.fcount) atomicAdd(a.fcount + 1, nwalk);
    __syncthreads();
    publish_block(a, K, nullptr, nullptr, hmin, hmax, kcnt, kpos, kovf, nstage, lane, 64, blockIdx.x, kcorr);
  }
}

template <int EM, int EK, bool WIN, bool EXACT, int KX = 0>
hipError_t launch_dense_t(const SweepArgs &a, size_t lds, int grid, int x4, hipStream_t stream, int *used) {
  const void *fn = (const void *)k_dense<EM, EK, WIN, EXACT, KX>;
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
  hipLaunchKernelGGL((k_dense<EM, EK, WIN, EXACT, KX>), dim3(grid), dim3(64), lds, stream, a, x4);
  return hipGetLastError();
}

template <int EM, int EK, bool WIN, bool EXACT, int KX = 0>
int resident_dense_t(size_t lds) {
  const void *fn = (const void *)k_dense<EM, EK, WIN, EXACT, KX>;
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

// Probe for the window pass of dense costs when some window does not
// contain lambda_k^t: on 4096 users spread over the instance, count those
// with a line above -H (H: the widest window's reach times the user's
// largest cost).  A user without one is settled by the window pass's gap
// test whatever its windows (no line can turn positive in any of them); the
// host runs the lane-per-user pass when almost every sampled user is such.
__global__ void __launch_bounds__(64) k_dense_probe(const float *p, const float *b, const double *lam,
                                                    const KState *st, int64_t N, int M, int K, int *out) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= KP_PROBE_USERS) return;
  const int64_t u = i * N / KP_PROBE_USERS;
  double hm = 0.0;
  for (int k = 0; k < K; ++k)
    if (st[k].mode == KS_WINDOW) hm = fmax(hm, st[k].hw);
  const float *pu = p + u * M;
  const float *bu = b + u * M * K;
  float bm = 0.0f;
  for (int e = 0; e < M * K; ++e) bm = fmaxf(bm, bu[e]);
  const double H = hm * (double)bm * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (double)bm * hm);
  bool up = false;
  for (int j = 0; j < M; ++j) {
    double acc = (double)pu[j];
    for (int k = 0; k < K; ++k) {
      const double prod = lam[k] * (double)bu[j * K + k];
      acc = acc - prod;
    }
    up = up || acc > -H;
  }
  if (up) atomicAdd(out, 1);
}

hipError_t kp_launch_dense_probe(const SweepArgs &a, int *out, hipStream_t stream) {
  if (a.pr.fmt != 0 || a.pr.N <= 0 || !a.st) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dense_probe, dim3(KP_PROBE_USERS / 64), dim3(64), 0, stream, a.pr.p, a.pr.b, a.lam, a.st,
                     (int64_t)a.pr.N, a.pr.M, a.pr.K, out);
  return hipGetLastError();
}

int kp_dense_tile_users() { return TU; }

// Evaluation (statistics into a.partials [grid][K + 2] and/or x) over
// a.ntiles tiles of kp_dense_tile_users() users; win: the SCD window pass
// (a.st: every knapsack in KS_WINDOW or finished; events staged per block
// into a.stage_*, window corrections into a.st[k].corr, users with a pair
// to walk counted into a.fcount[1] when a.fcount is set).  grid: an upper
// bound (the size of the per-block buffers); *used receives the blocks
// launched (at most the resident ones).
hipError_t kp_launch_dense(const SweepArgs &a, int grid, hipStream_t stream, int *used, bool win) {
  const int M = a.pr.M, K = a.pr.K;
  if (a.pr.fmt != 0 || M < 1 || M > 16 || K < 1 || K > 16 || a.tree.L < 0) return hipErrorInvalidValue;
  if (win && (!a.st || !a.err || !a.stage_v1 || a.stage_cap == 0)) return hipErrorInvalidValue;
  const size_t lds = dn_lds(M, K, a.tree.L, win);
  const int x4 = (((uintptr_t)a.pr.p | (uintptr_t)a.pr.b) & 15) == 0;
  return dispatch_dense(M, K, [&](auto em, auto ek) {
    constexpr int EM = decltype(em)::value, EK = decltype(ek)::value;
    if (M == EM) {
      if (K == 10)
        return win ? launch_dense_t<EM, EK, true, true, 10>(a, lds, grid, x4, stream, used)
                   : launch_dense_t<EM, EK, false, true, 10>(a, lds, grid, x4, stream, used);
      if (K == 2)
        return win ? launch_dense_t<EM, EK, true, true, 2>(a, lds, grid, x4, stream, used)
                   : launch_dense_t<EM, EK, false, true, 2>(a, lds, grid, x4, stream, used);
      return win ? launch_dense_t<EM, EK, true, true>(a, lds, grid, x4, stream, used)
                 : launch_dense_t<EM, EK, false, true>(a, lds, grid, x4, stream, used);
    }
    return win ? launch_dense_t<EM, EK, true, false>(a, lds, grid, x4, stream, used)
               : launch_dense_t<EM, EK, false, false>(a, lds, grid, x4, stream, used);
  });
}

// Blocks of the dense evaluation (win: the window pass) that can be resident
// at once; 0 when the shape is outside the kernel's range or the query fails.
int kp_dense_resident_grid(int M, int K, int L, bool win) {
  if (M < 1 || M > 16 || K < 1 || K > 16) return 0;
  const size_t lds = dn_lds(M, K, L, win);
  return dispatch_dense(M, K, [&](auto em, auto ek) {
    constexpr int EM = decltype(em)::value, EK = decltype(ek)::value;
    if (M == EM) {
      if (K == 10) return win ? resident_dense_t<EM, EK, true, true, 10>(lds) : resident_dense_t<EM, EK, false, true, 10>(lds);
      if (K == 2) return win ? resident_dense_t<EM, EK, true, true, 2>(lds) : resident_dense_t<EM, EK, false, true, 2>(lds);
      return win ? resident_dense_t<EM, EK, true, true>(lds) : resident_dense_t<EM, EK, false, true>(lds);
    }
    return win ? resident_dense_t<EM, EK, true, false>(lds) : resident_dense_t<EM, EK, false, false>(lds);
  });
}
