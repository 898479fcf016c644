// Lean sweep kernel for per-item CSR costs whose item rows all hold the same
// number D of stored entries (row r's entries at [r*D, r*D + D)), M <= 16.
//
// One wave owns a tile of 64 users, one lane per user; waves never wait for
// each other inside the tile loop.  The tile's profits and entries are staged
// with coalesced direct-to-LDS loads and then moved into the lane's registers;
// the staging area is reused as per-lane scratch for the rest of the tile.
// Per lane: cost-adjusted profits (FP64, stored columns ascending, no FMA),
// ranks by (p~ desc, index asc), the laminar greedy (Alg.1 as the matroid
// greedy), its consumption / profit / dual sums, and for SCD every knapsack's
// breakpoints: a knapsack moving one item of the user has at most one, at the
// item's threshold element; knapsacks moving several items of the user are
// queued, and once the one-item cases are done the wave's (user, knapsack)
// pairs are walked exactly, dealt over all 64 lanes.  R, g and P are summed
// in a fixed order (per-lane LDS columns, fixed-order row sums, waves added
// in order per block, blocks added in order by a second kernel); the
// threshold search's sums are exact two-limb integers (order-free atomics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include "kp_device.h"

#define EW 4                 // waves per block (the full-search pass: 8 when its LDS allows)

// wave-wide sum in a fixed butterfly order; every lane gets lane 0's value
__device__ __forceinline__ double wave_sum(double v) {
  #pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, 64);
  return __shfl(v, 0, 64);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Cache policy of the staging loads: nontemporal (every input byte is read
// once per pass, so keeping it in the caches only evicts other data).
#define KP_STAGE_NT 2

// Copy n dwords from global src to LDS dst (coalesced; lanes past the end
// reload the last dword into the padded tail of dst).
__device__ __forceinline__ void stage_dwords(const void *src, int n, void *dst, int lane) {
  const uint32_t *s = (const uint32_t *)src;
  uint32_t *d = (uint32_t *)dst;
  for (int c = 0; c * 64 < n; ++c) {
    int i = c * 64 + lane;
    i = i < n ? i : n - 1;
    __builtin_amdgcn_global_load_lds((const void *)(s + i), (lds_void_t *)(d + c * 64), 4, 0, KP_STAGE_NT);
  }
}

// Copy nbytes (a multiple of 256) from 16-byte aligned global src to LDS dst
// with 16-byte direct-to-LDS loads: lane i carries bytes [16 i, 16 i + 16) of
// each 1 KB chunk; in the last, partial chunk the lanes past the end stay idle.
__device__ __forceinline__ void stage_x4(const void *src, int nbytes, void *dst, int lane) {
  const unsigned char *s = (const unsigned char *)src + lane * 16;
  unsigned char *d = (unsigned char *)dst;
  int c = 0;
  for (; c + 1024 <= nbytes; c += 1024)
    __builtin_amdgcn_global_load_lds((const void *)(s + c), (lds_void_t *)(d + c), 16, 0, KP_STAGE_NT);
  if (c < nbytes && lane * 16 < nbytes - c)
    __builtin_amdgcn_global_load_lds((const void *)(s + c), (lds_void_t *)(d + c), 16, 0, KP_STAGE_NT);
}

// Sum of the entries 0, ST, 2 ST, ... of a 64-entry statistics row in four
// interleaved chains combined in a fixed order.  The stride is a constant,
// so the reads carry immediate offsets and are issued back to back.
template <int ST>
__device__ __forceinline__ double row_part_sum(const double *row) {
  constexpr int LEN = 64 / ST;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  #pragma unroll
  for (int u = 0; u < LEN; ++u) c[u & 3] = c[u & 3] + row[u * ST];
  return (c[0] + c[1]) + (c[2] + c[3]);
}

// lambda_k and the window bound wA_k (fp32, rounded up) of the window main pass
struct LamW {
  double lam;
  float w;
  float pad;
};

// Per-wave scratch of the breakpoint phase (byte offsets in the wave's region).
struct EllScratch {
  int pt, bt, kt, msk, end;
};
__host__ __device__ inline EllScratch ell_scratch(int M, int D, int K) {
  auto r16 = [](int b) { return (b + 15) & ~15; };
  EllScratch x;
  x.pt = 0;
  x.bt = x.pt + r16(M * 64 * 8);
  x.kt = x.bt + r16(M * D * 64 * 4);
  x.msk = x.kt + r16(M * D * 64);
  x.end = x.msk + r16(K * 64 * 2);
  return x;
}

struct EllGeom {
  int M, K, region;   // region: bytes of per-wave LDS
  int rows;           // statistics rows (of 65 doubles) per chunk
  int x4;             // p, col and val are 16-byte aligned: full tiles use 16-byte loads
  int compact;        // at most KP_SEL_MAX items can be selected (the matroid's rank)
  int waves;          // waves per block of the launch
};

// One (user, knapsack) pair of a lane-per-user breakpoint phase, run by
// any lane of the wave for the user of lane col.  In a window pass the
// user's greedy set at lambda^t is kept when it stays optimal at both edges
// of the window; otherwise the pair is walked exactly from above every
// breakpoint: the next breakpoint below is the highest crossing of an item
// outside the current set with zero (a free item) or with a member of the
// innermost full set holding it (Alg.1's exchange), fma-residual comparisons
// deciding which is highest.  Breakpoints inside the window are emitted
// (other search modes: binned or emitted by record_event), those above it
// add up to C_ik(whi+), and C_ik(whi+) - v_ik goes into the window
// correction.  A: the items moving with k; bkc(j, c): the cost in k of item
// j of lane c's user (j in A); ptl: the lanes' p~ columns [M][64]; Sc, posc,
// permc: the user's greedy set, positive items and rank order.
template <class BKC>
__device__ __forceinline__ void lane_walk_pair(const SweepArgs &a, int M, int L, int col, int k, uint64_t A,
                                               uint64_t Sc, uint64_t posc, uint64_t permc, BKC bkc,
                                               const double *ptl, const double *lam, const KState *kst,
                                               const int *kmode, const uint64_t *tmask, const int *tcap,
                                               XSum *kcorr, XSum *hs, uint32_t *hc, unsigned long long *hmin,
                                               unsigned long long *hmax, uint32_t *kcnt, uint32_t *kovf,
                                               uint32_t *nstage) {
  const int mode = kmode[k];
  const double lk = lam[k];
  if (mode == KS_WINDOW) {
    const double whi = kst[k].whi, wlo = kst[k].wlo;
    auto line = [&](int j, double &c, double &b) {
      b = (A >> j & 1) ? bkc(j, col) : 0.0;
      const double add = lk * b;
      c = ptl[j * 64 + col] + add;
    };
    if (window_keeps(Sc, A, posc & ~Sc, line, tmask, tcap, L, whi, 1) &&
        window_keeps(Sc, A, posc & ~Sc, line, tmask, tcap, L, wlo, wlo > 0.0 ? -1 : 1))
      return;
  }
  // start: only horizontal positive lines, in p~ order
  uint64_t Sw = 0;
  {
    uint64_t blocked = 0;
    const uint64_t elig = posc & ~A;
    for (int r = 0; r < M; ++r) {
      const int j = (int)((permc >> (4 * r)) & 15);
      const uint64_t bit = 1ull << j;
      if ((elig & bit) && !(blocked & bit)) {
        Sw |= bit;
        for (int l = 0; l < L; ++l) {
          const uint64_t m = tmask[l];
          if ((m & bit) && popc64(Sw & m) >= tcap[l]) blocked |= m;
        }
      }
    }
  }
  double above = 0.0;
  const int maxev = M * M + M + 8;
  for (int ev = 0;; ++ev) {
    if (ev >= maxev) { atomicAdd(a.err, 1ull); break; }
    double best = 0.0;
    int bo = -1, bs = -1;
    uint64_t cand = A & ~Sw;
    while (cand) {
      const int o = __ffsll((long long)cand) - 1;
      cand &= cand - 1;
      const double bo_d = bkc(o, col);
      const double add_o = lk * bo_d;
      const double co = ptl[o * 64 + col] + add_o;
      uint64_t circ = 0;
      bool tight = false;
      for (int l = 0; l < L; ++l) {
        const uint64_t m = tmask[l];
        if ((m >> o & 1) && popc64(Sw & m) >= tcap[l]) { circ = Sw & m; tight = true; break; }
      }
      // compared with the running maximum through cr_gt: a division only
      // for a crossing that beats it
      if (!tight) {
        if (co > 0.0 && cr_gt(co, bo_d, best)) { best = co / bo_d; bo = o; bs = -1; }
      } else {
        while (circ) {
          const int s2 = __ffsll((long long)circ) - 1;
          circ &= circ - 1;
          const double bs_d = (A >> s2 & 1) ? bkc(s2, col) : 0.0;
          if (bs_d < bo_d) {
            const double add_s = lk * bs_d;
            const double cs = ptl[s2 * 64 + col] + add_s;
            const double num = co - cs;
            const double den = bo_d - bs_d;
            if (cr_gt(num, den, best)) { best = num / den; bo = o; bs = s2; }
          }
        }
      }
    }
    if (bo < 0) break;
    const double bo_d = bkc(bo, col);
    const double bsv = (bs >= 0 && (A >> bs & 1)) ? bkc(bs, col) : 0.0;
    const double v2 = bs >= 0 ? bo_d - bsv : bo_d;
    if (mode == KS_WINDOW) {
      const uint64_t key = dkey(best);
      if (key < kst[k].klo) break;          // every later breakpoint is lower
      if (key > kst[k].khi) above = above + v2;
      else record_event(a, kst[k], k, best, v2, mode, hs, hc, hmin, hmax, kcnt, kovf, nstage, blockIdx.x);
    } else {
      record_event(a, kst[k], k, best, v2, mode, hs, hc, hmin, hmax, kcnt, kovf, nstage, blockIdx.x);
    }
    Sw = (Sw | (1ull << bo)) & ~(bs >= 0 ? (1ull << bs) : 0ull);
  }
  if (mode == KS_WINDOW) {
    double now = 0.0;
    for (uint64_t m = Sc & A; m; m &= m - 1) now = now + bkc(__ffsll((long long)m) - 1, col);
    if (above != now) {
      xs_atomic_add_sum(&kcorr[k], xs_minus(xs_of(above), xs_of(now)));
    }
  }
}

// The wave's (user, knapsack) pairs (bit k of a lane's `pending`) are
// numbered in lane order and dealt out 64 at a time over all lanes, so a
// wave runs about (its pairs) / 64 rounds instead of its busiest lane's
// count; walk(col, k, S, pos, perm) works on lane col's user with the greedy
// set, positive items and ranks read from that lane's registers.  Every lane
// of the wave calls this.
template <class W>
__device__ __forceinline__ void lane_deal_pairs(int lane, uint64_t pending, uint64_t S, uint64_t pos,
                                                uint64_t perm, W walk) {
  const int cnt = __popcll(pending);
  int incl = cnt;
  #pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int excl = incl - cnt;
  const int total = __shfl(incl, 63, 64);
  for (int base = 0; base < total; base += 64) {
    const int idx = base + lane;
    // the pair's owner: the last lane whose first pair is at or before idx
    int lo = 0, hi = 63;
    #pragma unroll
    for (int st = 0; st < 6; ++st) {
      const int mid = (lo + hi + 1) >> 1;
      if (__shfl(excl, mid, 64) <= idx) lo = mid;
      else hi = mid - 1;
    }
    uint64_t po = (uint64_t)__shfl((long long)pending, lo, 64);
    const int nth = idx - __shfl(excl, lo, 64);
    const uint64_t So = (uint64_t)__shfl((long long)S, lo, 64);
    const uint64_t poso = (uint64_t)__shfl((long long)pos, lo, 64);
    const uint64_t permo = (uint64_t)__shfl((long long)perm, lo, 64);
    if (idx >= total) continue;
    for (int q = 0; q < nth; ++q) po &= po - 1;
    walk(lo, __ffsll((long long)po) - 1, So, poso, permo);
  }
}

// Breakpoint phase of one user (one lane) from its per-lane LDS scratch:
// p~ (ptl), stored costs (btl) and their knapsacks (ktl), and the items
// moving with each knapsack (mskl).  S is the greedy set at lambda^t, pos the
// items with p~ > 0, perm the items ranked by (p~ desc, index asc).
template <int D>
__device__ __forceinline__ void scd_user(const SweepArgs &a, int M, int K, int L, int lane, bool act,
                                         int alg5q, int64_t uidx,
                                         uint64_t S, uint64_t pos, uint64_t perm, double bmax,
                                         const double *ptl, const float *btl, const uint8_t *ktl,
                                         const uint16_t *mskl, const double *lam, const uint64_t *tmask,
                                         const int *tcap, const KState *kst, const int *kmode,
                                         const double *hwin, XSum *kcorr, XSum *hs, uint32_t *hc,
                                         unsigned long long *hmin, unsigned long long *hmax,
                                         uint32_t *kcnt, uint32_t *kovf, uint32_t *nstage) {
  // (every lane of the wave runs this function: inactive lanes skip their
  // own user's work but take part in the walks of the others')
  // cost of item j in knapsack k (j moves with k), from lane c's column
  auto bkc = [&](int j, int k, int c) -> double {
    if (D == 1) return (double)btl[j * 64 + c];
    const int t = ktl[(j * D) * 64 + c] == k ? 0 : 1;
    return (double)btl[(j * D + t) * 64 + c];
  };
  auto bk = [&](int j, int k) -> double { return bkc(j, k, lane); };
  // Window filter per (user, knapsack): over knapsack k's window (within h of
  // lambda_k^t) item a's line moves by at most h b_ak against the fixed lines
  // of the items that do not move with k, and by at most h max(b_ak, b_bk)
  // against another moving item b.  So no crossing with another line (or
  // with zero) lies in the window when every moving item's distance to its
  // nearest neighbour in rank order (and to zero) exceeds h b_ak plus a
  // rounding margin.  Lines below -H (H: the widest window times the
  // largest cost) never turn positive in any window and never matter.
  double H = 0.0, gscale = 0.0;
  uint64_t rinv = 0;   // rank of every item, 4 bits each
  if (hwin[K] > 0.0) {
    H = hwin[K] * bmax * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + bmax * hwin[K]);
    for (int r = 0; r < M; ++r) rinv |= (uint64_t)r << (4 * ((perm >> (4 * r)) & 15));
    gscale = fabs(ptl[(int)(perm & 15) * 64 + lane]) + H;
  }
  // distance from item j's line to its rank neighbours above -H and to zero
  auto gap = [&](int j) -> double {
    const double v = ptl[j * 64 + lane];
    if (!(v > -H)) return 1e300;
    const int r = (int)((rinv >> (4 * j)) & 15);
    double d = fabs(v);
    if (r > 0) d = fmin(d, ptl[(int)((perm >> (4 * (r - 1))) & 15) * 64 + lane] - v);
    if (r + 1 < M) {
      const double w = ptl[(int)((perm >> (4 * (r + 1))) & 15) * 64 + lane];
      if (w > -H) d = fmin(d, v - w);
    }
    return d;
  };
  // true when no breakpoint of this user lies in knapsack k's window (A: the
  // items moving with k)
  auto calm = [&](int k, uint32_t A) -> bool {
    const double h = hwin[k], lk = lam[k];
    for (uint32_t m = A; m; m &= m - 1) {
      const int o = __ffs((int)m) - 1;
      const double b = bk(o, k);
      const double need = h * b * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + gscale + lk * b + h * b);
      if (!(gap(o) > need)) return false;
    }
    return true;
  };
  // threshold element of every item against the greedy solution of the other
  // items (valid when it is the only item that moves with lambda_k): the
  // lowest member of the innermost full set holding a non-member, or for a
  // member the best positive non-member whose innermost full set holds it;
  // zlev marks items whose only competitor is zero
  uint64_t tau = 0, zlev = 0;
  {
    uint64_t assigned = S;
    for (int l = 0; l < L; ++l) {
      const uint64_t m = tmask[l];
      if (popc64(S & m) < tcap[l]) continue;
      uint64_t pend = m & ~assigned;
      if (!pend) continue;
      int low = 0;
      for (int r = M - 1; r >= 0; --r) {
        const int j = (int)((perm >> (4 * r)) & 15);
        if ((S & m) >> j & 1) { low = j; break; }
      }
      assigned |= pend;
      while (pend) {
        const int o = __ffsll((long long)pend) - 1;
        pend &= pend - 1;
        tau |= (uint64_t)low << (4 * o);
      }
    }
    const uint64_t all = (M == 64) ? ~0ull : ((1ull << M) - 1);
    zlev |= ~assigned & all;
    uint64_t resolved = 0;
    for (int r = 0; r < M && resolved != S; ++r) {
      const int e = (int)((perm >> (4 * r)) & 15);
      if ((S >> e & 1) || !(pos >> e & 1)) continue;
      uint64_t lm = 0;
      for (int l = 0; l < L; ++l) {
        const uint64_t m = tmask[l];
        if ((m >> e & 1) && popc64(S & m) >= tcap[l]) { lm = m; break; }
      }
      uint64_t nw = S & lm & ~resolved;
      resolved |= nw;
      while (nw) {
        const int o = __ffsll((long long)nw) - 1;
        nw &= nw - 1;
        tau |= (uint64_t)e << (4 * o);
      }
    }
    zlev |= S & ~resolved;
  }
  // Alg.5 (Sec. 5.1; a user whose item j consumes only knapsack j, M = K,
  // one top-Q set): the Q-th and (Q+1)-th largest adjusted profits
  // max(p~, 0) are read off the rank order Alg.1 already holds (0 past the
  // last item); item k's only breakpoint is where its line p_k - lambda b_kk
  // meets the (Q+1)-th when k is in the top Q (ties with the Q-th count as
  // in it), else the Q-th
  double qth = 0.0, q1th = 0.0;
  if (alg5q > 0) {
    if (alg5q <= M) qth = fmax(ptl[(int)((perm >> (4 * (alg5q - 1))) & 15) * 64 + lane], 0.0);
    if (alg5q + 1 <= M) q1th = fmax(ptl[(int)((perm >> (4 * alg5q)) & 15) * 64 + lane], 0.0);
  }
  // one breakpoint per (item, knapsack) that moves alone; queue the others
  uint64_t pending = 0;
  for (int j = 0; act && j < M; ++j) {
    for (int t = 0; t < D; ++t) {
      const int k = ktl[(j * D + t) * 64 + lane];
      if (k >= K) continue;
      const int mode = kmode[k];
      if (!walk_mode(mode)) continue;
      const uint32_t A = mskl[k * 64 + lane];
      if (A != (1u << j)) {
        if (j == __ffs((int)A) - 1 && !(mode == KS_WINDOW && calm(k, A))) pending |= 1ull << k;
        continue;
      }
      if (mode == KS_WINDOW && calm(k, A)) continue;
      const double lk = lam[k];
      const double bo_d = (double)btl[(j * D + t) * 64 + lane];
      const double add_o = lk * bo_d;
      const double co = ptl[j * 64 + lane] + add_o;
      double best = 0.0;
      if (alg5q > 0) {
        const double pk = (double)a.pr.p[uidx * M + j];
        const double adj = fmax(ptl[j * 64 + lane], 0.0);
        const double pbar = adj >= qth ? q1th : qth;
        if (pk > pbar && bo_d > 0.0) {
          const double num = pk - pbar;
          best = num / bo_d;
        }
      } else if (zlev >> j & 1) {
        if (co > 0.0) best = co / bo_d;
      } else {
        const int th = (int)((tau >> (4 * j)) & 15);
        const double bs_d = 0.0;
        const double add_s = lk * bs_d;
        const double cs = ptl[th * 64 + lane] + add_s;
        const double num = co - cs;
        const double den = bo_d - bs_d;
        const double val = num / den;
        if (val > 0.0) best = val;
      }
      if (best > 0.0)
        record_event(a, kst[k], k, best, bo_d, mode, hs, hc, hmin, hmax, kcnt, kovf, nstage, blockIdx.x);
      if (mode == KS_WINDOW) {
        // consumption just above the window against the one at lambda^t
        const double above = (best > 0.0 && dkey(best) > kst[k].khi) ? bo_d : 0.0;
        const double now = (S >> j & 1) ? bo_d : 0.0;
        if (above != now) xs_atomic_add(&kcorr[k], above - now);
      }
    }
  }
  // Knapsacks moving several items of a user: dealt over the wave (see
  // lane_deal_pairs) and walked through the owner's LDS column
  __builtin_amdgcn_s_waitcnt(0);   // every lane's scratch column is written before any lane reads another's
  __builtin_amdgcn_wave_barrier();
  __asm__ volatile("" ::: "memory");
  lane_deal_pairs(lane, pending, S, pos, perm, [&](int col, int k, uint64_t So, uint64_t poso, uint64_t permo) {
    lane_walk_pair(a, M, L, col, k, (uint64_t)mskl[k * 64 + col], So, poso, permo,
                   [&](int j, int c) { return bkc(j, k, c); }, ptl, lam, kst, kmode, tmask, tcap, kcorr, hs, hc,
                   hmin, hmax, kcnt, kovf, nstage);
  });
}

// Kernel modes: evaluation (and its post-processing variant); full SCD pass
// (every search mode); the window pass split in two -- the main kernel
// evaluates every user and lists the
// users whose lines may cross inside some knapsack's window, the second kernel
// gathers the listed users 64 per wave and runs their breakpoint phase with
// every lane busy.
enum { KM_EVAL = 0, KM_SCD = 1, KM_WMAIN = 2, KM_WFAIL = 3, KM_FIX = 4 };
// KM_FIX: the evaluation plus the post-processing's per-user bins (its own
// instantiation, so the plain evaluation keeps its registers).

// Waves per block (WPB): 4; the full-search pass keeps K x 64 exact
// histogram bins per block in LDS, so when its LDS allows it runs 8 waves per
// block (one block per compute unit, two waves per SIMD) rather than 4 (which
// its LDS would hold to one block).

// The window main pass of the exact kernels up to 10 items is held to 3
// waves per SIMD, the occupancy its LDS allows (without the hint it compiles
// just above the register limit).  The larger ones would spill registers
// under that limit; a build of one of them that spilled gave wrong
// multipliers after a window pass where the same source without the limit
// did not, so they keep every register they need.
template <int MODE, int EM, bool EXACT> struct EllWaves {
  static constexpr int value = (MODE == 2 && EXACT && EM <= 10) ? 3 : 1;
};

// EM: the item-count class (8, 10, 12, 16); EXACT: M equals EM, so every
// test of an item index against M folds away.  KX: the knapsack count when
// it is fixed at compile time (10 or 20 with M = 10, and every statistics
// row in one chunk), else 0: the loops over the knapsacks and the rows then
// have constant trip counts (c3 window pass 4.51 -> 4.27 ms, evaluation
// 3.35 -> 3.20 ms).
template <int D, int MODE, int EM, bool EXACT, int WPB, bool CMP, int KX>
__global__ void __launch_bounds__(WPB * 64)
__attribute__((amdgpu_waves_per_eu(EllWaves<MODE, EM, EXACT>::value, 8)))
k_ell(const SweepArgs a, const EllGeom g) {
  constexpr int EWM = WPB;
  constexpr int ENT = EWM * 64;
  constexpr bool BREAK = (MODE == KM_SCD || MODE == KM_WFAIL);   // breakpoint phase
  constexpr bool STAGED = (MODE != KM_WFAIL);                    // contiguous tiles
  constexpr bool EV = (MODE == KM_EVAL || MODE == KM_FIX);       // evaluation only
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int M = EXACT ? EM : g.M, K = KX ? KX : g.K;
  const int grows = KX ? KX + 2 : g.rows;   // statistics rows per chunk
  // g.compact, fixed at compile time for the kernels instantiated for one
  // item count: the other path's arrays then need no registers
  const bool compact = EXACT ? CMP : g.compact != 0;
  size_t off = 0;
  auto carve = [&](size_t bytes) { unsigned char *p = smem + off; off += (bytes + 15) & ~(size_t)15; return p; };
  double *lam = (double *)carve((size_t)(K + 1) * 8);   // [K] = 0 for the clamped reads
  uint64_t *tmask = (uint64_t *)carve((size_t)a.tree.L * 8 + 8);
  int *tcap = (int *)carve((size_t)a.tree.L * 4 + 4);
  double *wacc = (double *)carve((size_t)EWM * (K + 2) * 8);
  KState *kst = BREAK ? (KState *)carve((size_t)K * sizeof(KState)) : nullptr;
  XSum *hs = nullptr;
  uint32_t *hc = nullptr, *kcnt = nullptr, *kpos = nullptr, *kovf = nullptr, *nstage = nullptr;
  int *kmode = nullptr;
  unsigned long long *hmin = nullptr, *hmax = nullptr;
  XSum *kcorr = nullptr;
  double *hwin = nullptr;
  if (!EV) {
    kmode = (int *)carve((size_t)K * 4);
    hwin = (double *)carve((size_t)K * 8 + 16);  // [K] window half-widths (0: no window), [K] their max,
                                                 // [K+1] the largest multiplier with a window
  }
  // window main pass: (lambda_k, wA_k) pairs read together by the scoring,
  // [K] = (0, 0) for the clamped reads
  LamW *lw = MODE == KM_WMAIN ? (LamW *)carve((size_t)(K + 1) * sizeof(LamW)) : nullptr;
  if (BREAK) {
    kcorr = (XSum *)carve((size_t)K * sizeof(XSum));
    if (MODE == KM_SCD) {   // the listed users' pass runs only when every search has a window
      hs = (XSum *)carve((size_t)K * KP_NB * sizeof(XSum));
      hc = (uint32_t *)carve((size_t)K * KP_NB * 4);
    }
    kcnt = (uint32_t *)carve((size_t)K * 4);
    kpos = (uint32_t *)carve((size_t)K * 4);
    kovf = (uint32_t *)carve((size_t)K * 4);
    hmin = (unsigned long long *)carve((size_t)K * 8);
    hmax = (unsigned long long *)carve((size_t)K * 8);
    nstage = (uint32_t *)carve(16);
  }
  // post-processing bins: violated-slot map, splitters, the block's bin sums
  int *fkv = nullptr;
  uint64_t *fsp = nullptr;
  XSum *fhs = nullptr;
  uint32_t *fhc = nullptr;
  if (MODE == KM_FIX) {
    fkv = (int *)carve((size_t)K * 4);
    fsp = (uint64_t *)carve((size_t)a.fx.nb * 8);
    fhs = (XSum *)carve((size_t)a.fx.nb * a.fx.nv * sizeof(XSum));
    fhc = (uint32_t *)carve((size_t)a.fx.nb * 4);
    for (int t = tid; t < K; t += ENT) fkv[t] = a.fx.kv[t];
    for (int t = tid; t < a.fx.nb - 1; t += ENT) fsp[t] = a.fx.split[t];
    for (int t = tid; t < a.fx.nb * a.fx.nv; t += ENT) fhs[t] = xs_zero();
    for (int t = tid; t < a.fx.nb; t += ENT) fhc[t] = 0u;
  }
  unsigned char *wreg = smem + off + (size_t)wv * g.region;   // this wave's region
  for (int t = tid; t <= K; t += ENT) lam[t] = t < K ? a.lam[t] : 0.0;
  if (MODE == KM_WMAIN && tid == 0) lw[K] = LamW{0.0, 0.0f, 0.0f};
  for (int t = tid; t < a.tree.L; t += ENT) { tmask[t] = a.tree.mask[t]; tcap[t] = a.tree.cap[t]; }
  for (int t = tid; t < EWM * (K + 2); t += ENT) wacc[t] = 0.0;
  if (!EV) {
    for (int t = tid; t < K; t += ENT) {
      kmode[t] = a.st[t].mode;
      hwin[t] = a.st[t].mode == KS_WINDOW ? a.st[t].hw : 0.0;
      if (MODE == KM_WMAIN) {
        const double h = hwin[t];
        // wA_k, widened by 2^-20 before rounding to fp32 so that the fp32
        // product with a cost still bounds the exact one from above
        const double w = h > 0.0 ? h * (1.0 + 0x1p-30) + 0x1p-36 * (a.lam[t] + h) : 0.0;
        lw[t] = LamW{a.lam[t], (float)(w * (1.0 + 0x1p-20)), 0.0f};
      }
    }
  }
  if (BREAK) {
    for (int t = tid; t < K; t += ENT) {
      kst[t] = a.st[t];
      kcnt[t] = 0u; kpos[t] = 0u; kovf[t] = 0u;
      hmin[t] = ~0ull; hmax[t] = 0ull;
      kcorr[t] = xs_zero();
    }
    for (int t = tid; hs && t < K * KP_NB; t += ENT) { hs[t] = xs_zero(); hc[t] = 0u; }
    if (tid == 0) *nstage = 0u;
  }
  __syncthreads();
  if (!EV && tid == 0) {
    double m = 0.0, l = 0.0;
    for (int k = 0; k < K; ++k) {
      m = hwin[k] > m ? hwin[k] : m;
      if (hwin[k] > 0.0) l = lam[k] > l ? lam[k] : l;
    }
    hwin[K] = m;
    hwin[K + 1] = l;
  }
  uint32_t nlisted = 0;
  if (MODE == KM_WFAIL) {
    const uint32_t cnt = *a.fcount;
    nlisted = cnt < a.fcap ? cnt : a.fcap;
    // a list that overflowed cannot be processed whole: full search instead
    if (blockIdx.x == 0 && tid < K && cnt > a.fcap && a.st[tid].mode == KS_WINDOW)
      atomicOr(&a.st[tid].overflow, 1);
  }
  __syncthreads();
  const int L = a.tree.L;
  const int64_t N = a.pr.N;
  const int64_t W = (int64_t)gridDim.x * EWM;
  const int64_t ntiles = MODE == KM_WFAIL ? ((int64_t)nlisted + 63) / 64 : a.ntiles;

  // staging area of the wave (contiguous tiles); the statistics rows reuse it
  float *sp = (float *)wreg;
  int32_t *sc = (int32_t *)(wreg + (size_t)64 * M * 4);
  float *sv = (float *)(wreg + (size_t)64 * M * 4 + (size_t)64 * M * D * 4);
  double *rowbuf = (double *)wreg;

  uint32_t ch_pos = 0, ch_end = 0;   // the wave's reserved list chunk (window main pass)
  uint32_t nlist = 0;                 // users the wave listed
  // tile indices fit 32 bits (the launcher rejects more than 2^31 - 1 tiles)
  for (int tile = (int)blockIdx.x * EWM + wv; tile < (int)ntiles; tile += (int)W) {
    const int64_t u0 = (int64_t)tile * 64;
    float pv[EM];
    int cl[EM * D];
    float vl[EM * D];
    bool act;
    if (STAGED) {
      // ---- stage the tile (coalesced) and move the lane's user into registers ----
      const int nu = (int)((N - u0) < 64 ? (N - u0) : 64);
      act = lane < nu;
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      if (nu == 64 && g.x4) {
        stage_x4(a.pr.p + u0 * M, 256 * M, sp, lane);
        stage_x4(a.pr.col + u0 * M * D, 256 * M * D, sc, lane);
        stage_x4(a.pr.val + u0 * M * D, 256 * M * D, sv, lane);
      } else {
        stage_dwords(a.pr.p + u0 * M, nu * M, sp, lane);
        stage_dwords(a.pr.col + u0 * M * D, nu * M * D, sc, lane);
        stage_dwords(a.pr.val + u0 * M * D, nu * M * D, sv, lane);
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
      // unconditional reads of EM items (the region has slack past the last
      // lane's row), no selects: the padding items (j >= M) are cleared, and
      // lanes past the end of the last tile keep whatever the staging area
      // holds (they select nothing, emit nothing and are never listed).
      // With M known and the rows 16-byte aligned (M * D a multiple of 4),
      // costs are read 16 bytes at a time, which keeps the lanes (80 bytes
      // apart for M = 10, D = 2) on distinct LDS banks.
      const float *spl = sp + lane * M;
      const int32_t *scl = sc + lane * M * D;
      const float *svl = sv + lane * M * D;
      if (EXACT && (EM * D) % 4 == 0) {
        #pragma unroll
        for (int q = 0; q < EM * D / 4; ++q) {
          const int4 c4 = ((const int4 *)scl)[q];
          const float4 v4 = ((const float4 *)svl)[q];
          cl[4 * q] = c4.x; cl[4 * q + 1] = c4.y; cl[4 * q + 2] = c4.z; cl[4 * q + 3] = c4.w;
          vl[4 * q] = v4.x; vl[4 * q + 1] = v4.y; vl[4 * q + 2] = v4.z; vl[4 * q + 3] = v4.w;
        }
      } else {
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          #pragma unroll
          for (int t = 0; t < D; ++t) {
            const int32_t c0 = scl[j * D + t];
            const float v0 = svl[j * D + t];
            cl[j * D + t] = j < M ? c0 : -1;
            vl[j * D + t] = j < M ? v0 : 0.0f;
          }
        }
      }
      if (EXACT && EM % 2 == 0) {
        #pragma unroll
        for (int q = 0; q < EM / 2; ++q) {
          const float2 p2 = ((const float2 *)spl)[q];
          pv[2 * q] = p2.x; pv[2 * q + 1] = p2.y;
        }
      } else {
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          const float p0 = spl[j];
          pv[j] = j < M ? p0 : 0.0f;
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
    } else {
      // ---- gather the listed user into registers ----
      const int64_t idx = u0 + lane;
      const uint32_t entry = idx < (int64_t)nlisted ? a.flist[idx] : KP_LIST_HOLE;
      act = entry != KP_LIST_HOLE;
      const int64_t u = act ? (int64_t)entry : 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (j < M) {
          pv[j] = act ? a.pr.p[u * M + j] : 0.0f;
          #pragma unroll
          for (int t = 0; t < D; ++t) {
            cl[j * D + t] = act ? a.pr.col[(u * M + j) * D + t] : -1;
            vl[j * D + t] = act ? a.pr.val[(u * M + j) * D + t] : 0.0f;
          }
        } else {
          pv[j] = 0.0f;
          #pragma unroll
          for (int t = 0; t < D; ++t) { cl[j * D + t] = -1; vl[j * D + t] = 0.0f; }
        }
      }
    }
    // ---- cost-adjusted profits ----
    double pt[EM];
    // window main pass: nd[j] = item j's largest b_jk wA_k over its knapsacks
    // (0 when none has a window), an fp32 upper bound
    float nd[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      double acc = (double)pv[j];
      nd[j] = 0.0f;
      #pragma unroll
      for (int t = 0; t < D; ++t) {
        // every lane reads: entries outside [0, K) (and the padding) read
        // the zero slot lam[K], and subtracting 0 * v (v finite) leaves acc
        // unchanged bit for bit, so no branch or select is needed
        const unsigned k = (unsigned)cl[j * D + t];
        const unsigned kc = k < (unsigned)K ? k : (unsigned)K;
        double lk;
        if (MODE == KM_WMAIN) {
          const LamW e = lw[kc];
          lk = e.lam;
          nd[j] = fmaxf(nd[j], e.w * vl[j * D + t]);
          __asm__ volatile("" : "+v"(nd[j]));   // fold now: e.w dies here
        } else {
          lk = lam[kc];
        }
        const double prod = lk * (double)vl[j * D + t];
        acc = acc - prod;
      }
      pt[j] = acc;
    }
    // ---- ranks by (p~ desc, index asc), packed permutation ----
    int rk[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) rk[j] = j;   // rank = j + (later items ahead) - (earlier items behind)
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
    uint64_t perm = 0, pos = 0;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      if (j < M) {
        perm |= (uint64_t)j << (4 * rk[j]);
        if (pt[j] > 0.0) pos |= 1ull << j;
      }
    }
    if (!act) pos = 0;
    // ---- Alg.1's cap pass, in rank space (M <= 16: 32-bit masks) ----
    // Bit r of `alive` stands for the item of rank r; starting from the
    // items with p~ > 0, every laminar set (subsets first) keeps its cap
    // best live members.  The sets are uniform: their masks and caps come
    // from the kernel arguments into scalar registers.
    uint64_t S = 0;
    uint32_t rbit[EM];   // 1 << rank (the rank itself is its lowest set bit)
    {
      uint32_t alive = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        rbit[j] = j < M ? 1u << rk[j] : 0u;
        if (pt[j] > 0.0) alive |= rbit[j];
      }
      if (!act) alive = 0;
      for (int l = 0; l < L; ++l) {
        const uint32_t m = (uint32_t)a.tree.mask[l];
        const int cap = a.tree.cap[l];
        uint32_t mr = 0;
        #pragma unroll
        for (int j = 0; j < EM; ++j)
          if (m >> j & 1u) mr |= rbit[j];
        uint32_t x = alive & mr;
        for (int c = 0; c < cap; ++c) x &= x - 1u;   // drop the cap best: x = the rest
        alive &= ~x;
      }
      uint32_t S32 = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j)
        if (alive & rbit[j]) S32 |= 1u << j;
      S = S32;
    }
    double bmax = 0.0;
    if (!EV) {
      // largest stored cost (exact in fp32; widened once)
      float bm = 0.0f;
      #pragma unroll
      for (int j = 0; j < EM * D; ++j) bm = fmaxf(bm, vl[j]);
      bmax = (double)bm;
    }
    // ---- statistics: profit, group dual value, consumption ----
    double Pi = 0.0, Gi = 0.0;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      if (S >> j & 1) { Pi = Pi + (double)pv[j]; Gi = Gi + pt[j]; }
    }
    // At most KP_SEL_MAX items can be selected (the laminar matroid's rank,
    // g.compact): their stored entries are gathered from the staged tile
    // (still intact) in item order, so the consumption sums below visit
    // KP_SEL_MAX * D entries instead of M * D.  Unused slots hold (-1, 0).
    int sk[KP_SEL_MAX * D];
    float sv_[KP_SEL_MAX * D];
    if (STAGED && compact) {
      uint32_t sm = (uint32_t)S;
      const int32_t *scl = sc + lane * M * D;
      const float *svl = sv + lane * M * D;
      #pragma unroll
      for (int r = 0; r < KP_SEL_MAX; ++r) {
        const int j = sm ? __ffs((int)sm) - 1 : 0;
        const bool ok = sm != 0;
        sm &= sm - 1u;
        #pragma unroll
        for (int t = 0; t < D; ++t) {
          const int32_t c0 = scl[j * D + t];
          const float v0 = svl[j * D + t];
          sk[r * D + t] = ok ? c0 : -1;
          sv_[r * D + t] = ok ? v0 : 0.0f;
        }
      }
    }
    // Last read of the staged tile: the statistics rows and the breakpoint
    // phase's scratch are written over it (as other types, which the
    // compiler would otherwise take for separate memory), and another
    // lane's reads must not move below those writes.  LDS operations of a
    // wave run in program order, so keeping the compiler's order suffices.
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    // ---- post-processing bins (Sec. 5.4): a candidate's bin by G_i and its
    // costs on the violated knapsacks into the bin's exact sums ----
    if (MODE == KM_FIX && act) {
      const int nv = a.fx.nv;
      const int b = fx_bin_of(fsp, a.fx.nb, dkey(Gi + 0.0));
      XSum *row = fhs + (size_t)b * nv;
      bool cand = false;
      auto add = [&](int k, float c) {
        if ((unsigned)k >= (unsigned)K || !(c > 0.0f)) return;
        const int v = fkv[k];
        if (v < 0) return;
        cand = true;
        xs_atomic_add(&row[v], (double)c);
      };
      if (compact) {
        #pragma unroll
        for (int e = 0; e < KP_SEL_MAX * D; ++e) add(sk[e], sv_[e]);
      } else {
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          if (!(S >> j & 1)) continue;
          #pragma unroll
          for (int t = 0; t < D; ++t) add(cl[j * D + t], vl[j * D + t]);
        }
      }
      if (cand) atomicAdd(&fhc[b], 1u);
      a.fx.bin[u0 + lane] = cand ? (uint8_t)b : (uint8_t)0xFF;
    }
    // ---- window filter (main window pass), before the arrays die ----
    bool listed = false;
    if (MODE == KM_WMAIN) {
      // The breakpoint phase's test for all knapsacks at once: over the
      // windows, item a's line moves against any other line by at most
      // max_k b_ak wA_k (wA_k = h_k (1 + 2^-30) + 2^-36 (lambda_k + h_k), the
      // other item's own bound covering the pairs where its cost is the
      // larger), so the user is calm when every item with a window knapsack
      // is farther than that (plus 2^-36 (1 + gscale)) from its rank
      // neighbours above -H and from zero.  Lines below -H never turn
      // positive.  p~ and the bounds by rank go into the dead staging area.
      const double H = hwin[K] * bmax * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + bmax * hwin[K]);
      // The test runs in fp32: every p~ rounded to fp32 is within 2^-24 of
      // S = |top p~| + H of its FP64 value (lines below -H are cut), and a
      // difference of two such values within 2^-23 S plus its own rounding,
      // so requiring a margin of 2^-20 (1 + S) instead of the FP64 test's
      // 2^-36 (1 + S) keeps every decision on the safe side (a user is at
      // worst listed when it need not be; round-to-nearest keeps the rank
      // order, so the gaps stay >= 0).  The cut is widened by the margin.
      float *srt = (float *)wreg;
      float *srn = srt + (size_t)M * 64;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (j < M) {
          const int r = __builtin_ctz(rbit[j]);
          srt[r * 64 + lane] = (float)pt[j];
          srn[r * 64 + lane] = nd[j];
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
      const float S = fabsf(srt[lane]) + (float)H;
      const float marg = 0x1p-20f * (1.0f + S);
      const float Hc = (float)H + marg;
      // item r - 1 is decided once its lower neighbour is known
      bool fail = false, have = false;
      float pv0 = 0.0f, pd = 0.0f, pn = 0.0f;   // previous item: p~, gap so far, bound
      for (int r = 0; r < M; ++r) {
        const float v = srt[r * 64 + lane];
        if (!(v > -Hc)) break;
        const float n = srn[r * 64 + lane];
        float d = fabsf(v);
        if (have) {
          const float gg = pv0 - v;
          d = fminf(d, gg);
          pd = fminf(pd, gg);
          fail = fail || (pn > 0.0f && !(pd > pn + marg));
        }
        pv0 = v; pd = d; pn = n; have = true;
      }
      if (have) fail = fail || (pn > 0.0f && !(pd > pn + marg));
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
      __asm__ volatile("" ::: "memory");
      listed = act && fail;
    }
    if (STAGED && MODE != KM_FIX) {   // (the bin pass needs neither x nor the statistics)
      if (a.x_out && act) {
        uint8_t *xo = a.x_out + (u0 + lane) * M;
        for (int j = 0; j < M; ++j) xo[j] = (uint8_t)(S >> j & 1);
      }
      if (a.want_stats) {
        // per-lane rows [K + 2][65] (consumption per knapsack, G_i, P_i) over
        // the dead staging area, grows of them at a time.  Each lane adds its
        // selected costs into its own column with LDS atomic adds (one lane
        // per address, so the adds happen in program order and the sums are
        // the plain sequential ones); then lpr lanes per row sum contiguous
        // parts of it and combine them in a fixed butterfly (fixed order; the
        // odd row stride keeps the lanes on distinct banks)
        double *rows = rowbuf;
        const int KT = K + 2;
        for (int c0 = 0; c0 < KT; c0 += grows) {
          const int nq = KT - c0 < grows ? KT - c0 : grows;
          for (int q = 0; q < nq; ++q) rows[q * 65 + lane] = 0.0;
          if ((unsigned)(K - c0) < (unsigned)nq) rows[(K - c0) * 65 + lane] = Gi;
          if ((unsigned)(K + 1 - c0) < (unsigned)nq) rows[(K + 1 - c0) * 65 + lane] = Pi;
          if (compact) {
            #pragma unroll
            for (int e = 0; e < KP_SEL_MAX * D; ++e) {
              const int q = sk[e] - c0;
              const bool ok = (unsigned)q < (unsigned)nq && q < K - c0;
              __hip_atomic_fetch_add(&rows[(ok ? q : 0) * 65 + lane], ok ? (double)sv_[e] : 0.0,
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
          } else {
            #pragma unroll
            for (int j = 0; j < EM; ++j) {
              #pragma unroll
              for (int t = 0; t < D; ++t) {
                const int q = cl[j * D + t] - c0;
                // widened again here (an opaque copy): keeping the scoring's
                // widened costs alive until now would cost 2 registers each
                float v = vl[j * D + t];
                __asm__("" : "+v"(v));
                // unselected or foreign entries add +0 to row 0 (a consumption
                // row, never -0): no branch
                const bool ok = (S >> j & 1) && (unsigned)q < (unsigned)nq && q < K - c0;
                __hip_atomic_fetch_add(&rows[(ok ? q : 0) * 65 + lane], ok ? (double)v : 0.0,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
              }
            }
          }
          __builtin_amdgcn_s_waitcnt(0);
          __builtin_amdgcn_wave_barrier();
          __asm__ volatile("" ::: "memory");
          int lg = 0;
          while ((2 << lg) * nq <= 64) ++lg;
          const int q = lane >> lg, step = 1 << lg;
          double sum = 0.0;
          if (q < nq) {
            // part i sums the entries i, i + step, ... of the row (parts on
            // distinct banks)
            const double *row = rows + q * 65 + (lane & (step - 1));
            switch (lg) {
              case 0: sum = row_part_sum<1>(row); break;
              case 1: sum = row_part_sum<2>(row); break;
              case 2: sum = row_part_sum<4>(row); break;
              case 3: sum = row_part_sum<8>(row); break;
              case 4: sum = row_part_sum<16>(row); break;
              case 5: sum = row_part_sum<32>(row); break;
              default: sum = row_part_sum<64>(row); break;
            }
          }
          for (int o = 1; o < (1 << lg); o <<= 1) sum = sum + __shfl_xor(sum, o, 64);
          if (q < nq && (lane & ((1 << lg) - 1)) == 0)
            wacc[wv * KT + c0 + q] = wacc[wv * KT + c0 + q] + sum;
          __builtin_amdgcn_s_waitcnt(0);
          __builtin_amdgcn_wave_barrier();
          __asm__ volatile("" ::: "memory");
        }
      }
    }
    if (MODE == KM_WMAIN) {
      // append to the wave's reserved chunk of the list (one counter atomic
      // per KP_LIST_CHUNK entries instead of one per tile)
      const uint64_t mask = __ballot(listed);
      if (mask) {
        const uint32_t cnt = (uint32_t)__popcll(mask);
        nlist += cnt;
        const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
        // entries that still fit the current chunk, the rest opens a new one
        const uint32_t room = ch_end - ch_pos;
        uint32_t slot = ch_pos + rank;
        if (cnt > room) {
          uint32_t nb = 0;
          if (lane == 0) nb = atomicAdd(a.fcount, (uint32_t)KP_LIST_CHUNK);
          nb = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl(nb, 0, 64));
          if (rank >= room) slot = nb + (rank - room);
          ch_pos = nb + (cnt - room);
          ch_end = nb + KP_LIST_CHUNK;
        } else {
          ch_pos += cnt;
        }
        if (listed && slot < a.fcap) a.flist[slot] = (uint32_t)(u0 + lane);
      }
    }
    if (BREAK) {
      // per-lane scratch over the dead staging area: p~ [M][64], the stored
      // costs and their knapsacks [M*D][64], moving-item masks [K][64]
      const EllScratch sl = ell_scratch(M, D, K);
      double *ptl = (double *)(wreg + sl.pt);
      float *btl = (float *)(wreg + sl.bt);
      uint8_t *ktl = (uint8_t *)(wreg + sl.kt);
      uint16_t *mskl = (uint16_t *)(wreg + sl.msk);
      for (int k = 0; k < K; ++k) mskl[k * 64 + lane] = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        if (j < M) {
          ptl[j * 64 + lane] = pt[j];
          #pragma unroll
          for (int t = 0; t < D; ++t) {
            const int k = cl[j * D + t];
            const bool ok = (unsigned)k < (unsigned)K;
            btl[(j * D + t) * 64 + lane] = vl[j * D + t];
            ktl[(j * D + t) * 64 + lane] = (uint8_t)(ok ? k : 255);
            if (ok) mskl[k * 64 + lane] = (uint16_t)(mskl[k * 64 + lane] | (1u << j));
          }
        }
      }
      // Alg.5's setting for this user: item j's only entry is knapsack j
      bool diag = D == 1 && a.alg5_q > 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j)
        if (j < M) diag = diag && cl[j * D] == j;
      const int64_t uidx = STAGED ? u0 + lane : (act ? (int64_t)a.flist[u0 + lane] : 0);
      scd_user<D>(a, M, K, L, lane, act, diag ? a.alg5_q : 0, uidx, S, pos, perm, bmax, ptl, btl, ktl, mskl,
                  lam, tmask, tcap, kst,
                  kmode, hwin, kcorr, hs, hc, hmin, hmax, kcnt, kovf, nstage);
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (MODE == KM_WMAIN) {
    // mark the unused tail of the wave's last chunk
    for (uint32_t e = ch_pos + lane; e < ch_end; e += 64)
      if (e < a.fcap) a.flist[e] = KP_LIST_HOLE;
    if (lane == 0 && nlist) atomicAdd(a.fcount + 1, nlist);
  }
  __syncthreads();
  if (MODE == KM_FIX) {
    for (int t = tid; t < a.fx.nb * a.fx.nv; t += ENT)
      if (xs_nonzero(fhs[t])) xs_atomic_add_sum(&a.fx.hsum[t], fhs[t]);
    for (int t = tid; t < a.fx.nb; t += ENT)
      if (fhc[t]) atomicAdd(&a.fx.hcnt[t], fhc[t]);
  }
  if (a.want_stats && STAGED && MODE != KM_FIX) {
    for (int c = tid; c < K + 2; c += ENT) {
      double s = 0.0;
      for (int w = 0; w < EWM; ++w) s = s + wacc[w * (K + 2) + c];
      a.partials[(size_t)blockIdx.x * (K + 2) + c] = s;
    }
  }
  if (BREAK) publish_block(a, K, hs, hc, hmin, hmax, kcnt, kpos, kovf, nstage, tid, ENT, blockIdx.x, kcorr);
}

size_t kp_ell_lds_bytes(int M, int K, int D, int L, int mode, int *region_out);

// Persistent launch: never more blocks than can be resident at once (the
// tile loop strides over the rest), so no block waits for another to finish
// and every CU stays busy to the end.  grid <= 0 asks for exactly that many.
template <int D, int MODE, int EM, bool EXACT, int WPB, bool CMP = false, int KX = 0>
static hipError_t launch_ell_t(const SweepArgs &a, const EllGeom &g, size_t lds, int grid,
                               hipStream_t stream, int *used) {
  const void *fn = (const void *)k_ell<D, MODE, EM, EXACT, WPB, CMP, KX>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WPB * 64, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int resident = cus * per_cu;
  if (grid <= 0 || grid > resident) grid = resident;
  if (used) *used = grid;
  hipLaunchKernelGGL((k_ell<D, MODE, EM, EXACT, WPB, CMP, KX>), dim3(grid), dim3(WPB * 64), lds, stream, a, g);
  return hipGetLastError();
}

// The kernels for one item count, with the statistics path of g.compact
// (the listed users' pass keeps no statistics: one kernel)
template <int D, int MODE, int EM, int WPB, int KX>
static hipError_t launch_ell_c(const SweepArgs &a, const EllGeom &g, size_t lds, int grid,
                               hipStream_t stream, int *used) {
  if constexpr (MODE != KM_WFAIL) {
    if (g.compact) return launch_ell_t<D, MODE, EM, true, WPB, true, KX>(a, g, lds, grid, stream, used);
  }
  return launch_ell_t<D, MODE, EM, true, WPB, false, KX>(a, g, lds, grid, stream, used);
}

// ... and for M = 10 with 10 or 20 knapsacks whose statistics rows fit one
// chunk, the kernels with the knapsack count compiled in
template <int D, int MODE, int EM, int WPB>
static hipError_t launch_ell_x(const SweepArgs &a, const EllGeom &g, size_t lds, int grid,
                               hipStream_t stream, int *used) {
  if constexpr (EM == 10) {
    if (g.rows >= g.K + 2) {
      if (g.K == 20) return launch_ell_c<D, MODE, EM, WPB, 20>(a, g, lds, grid, stream, used);
      if (g.K == 10) return launch_ell_c<D, MODE, EM, WPB, 10>(a, g, lds, grid, stream, used);
    }
  }
  return launch_ell_c<D, MODE, EM, WPB, 0>(a, g, lds, grid, stream, used);
}

template <int D, int MODE, int WPB>
static hipError_t launch_ell_mw(const SweepArgs &a, const EllGeom &g, size_t lds, int grid,
                                hipStream_t stream, int *used) {
  switch (g.M) {
    case 8: return launch_ell_x<D, MODE, 8, WPB>(a, g, lds, grid, stream, used);
    case 10: return launch_ell_x<D, MODE, 10, WPB>(a, g, lds, grid, stream, used);
    case 12: return launch_ell_x<D, MODE, 12, WPB>(a, g, lds, grid, stream, used);
    case 16: return launch_ell_x<D, MODE, 16, WPB>(a, g, lds, grid, stream, used);
    default: break;
  }
  if constexpr (WPB != EW) {
    return hipErrorInvalidValue;   // 8-wave blocks are launched only for the exact item counts
  } else {
    if (g.M <= 8) return launch_ell_t<D, MODE, 8, false, WPB>(a, g, lds, grid, stream, used);
    if (g.M <= 10) return launch_ell_t<D, MODE, 10, false, WPB>(a, g, lds, grid, stream, used);
    if (g.M <= 12) return launch_ell_t<D, MODE, 12, false, WPB>(a, g, lds, grid, stream, used);
    return launch_ell_t<D, MODE, 16, false, WPB>(a, g, lds, grid, stream, used);
  }
}

template <int D, int MODE>
static hipError_t launch_ell_m(const SweepArgs &a, const EllGeom &g, size_t lds, int grid,
                               hipStream_t stream, int *used) {
  if constexpr (MODE == KM_SCD) {
    if (g.waves == 8) return launch_ell_mw<D, MODE, 8>(a, g, lds, grid, stream, used);
  }
  return launch_ell_mw<D, MODE, EW>(a, g, lds, grid, stream, used);
}

template <int D, int MODE, int EM, bool EXACT, int WPB, bool CMP = false, int KX = 0>
static int resident_blocks_t(size_t lds) {
  const void *fn = (const void *)k_ell<D, MODE, EM, EXACT, WPB, CMP, KX>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WPB * 64, lds) != hipSuccess) return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// the largest count over the kernels of one item count (an upper bound
// for the per-block buffers; a launch never exceeds its own kernel's count)
template <int D, int MODE, int EM, int WPB, int KX>
static int resident_blocks_c(size_t lds) {
  const int r = resident_blocks_t<D, MODE, EM, true, WPB, false, KX>(lds);
  if constexpr (MODE != KM_WFAIL) {
    const int c = resident_blocks_t<D, MODE, EM, true, WPB, true, KX>(lds);
    return c > r ? c : r;
  }
  return r;
}
template <int D, int MODE, int EM, int WPB>
static int resident_blocks_x(size_t lds) {
  int r = resident_blocks_c<D, MODE, EM, WPB, 0>(lds);
  if constexpr (EM == 10) {
    const int r20 = resident_blocks_c<D, MODE, EM, WPB, 20>(lds);
    const int r10 = resident_blocks_c<D, MODE, EM, WPB, 10>(lds);
    r = r20 > r ? r20 : r;
    r = r10 > r ? r10 : r;
  }
  return r;
}

template <int D, int MODE, int WPB>
static int resident_blocks_mw(int M, size_t lds) {
  switch (M) {
    case 8: return resident_blocks_x<D, MODE, 8, WPB>(lds);
    case 10: return resident_blocks_x<D, MODE, 10, WPB>(lds);
    case 12: return resident_blocks_x<D, MODE, 12, WPB>(lds);
    case 16: return resident_blocks_x<D, MODE, 16, WPB>(lds);
    default: break;
  }
  if constexpr (WPB != EW) {
    return 0;
  } else {
    if (M <= 8) return resident_blocks_t<D, MODE, 8, false, WPB>(lds);
    if (M <= 10) return resident_blocks_t<D, MODE, 10, false, WPB>(lds);
    if (M <= 12) return resident_blocks_t<D, MODE, 12, false, WPB>(lds);
    return resident_blocks_t<D, MODE, 16, false, WPB>(lds);
  }
}

template <int D, int MODE>
static int resident_blocks_m(int M, size_t lds, int waves) {
  if constexpr (MODE == KM_SCD) {
    if (waves == 8) return resident_blocks_mw<D, MODE, 8>(M, lds);
  }
  return resident_blocks_mw<D, MODE, EW>(M, lds);
}

// one translation unit per mode instantiates these (kp_ell_m<mode>.hip)
template <int MODE>
hipError_t kp_launch_ell_mode(const SweepArgs &a, const EllGeom &g, size_t lds, int grid, int D,
                              hipStream_t stream, int *used);
template <int MODE>
int kp_ell_resident_mode(int D, int M, size_t lds, int waves);
