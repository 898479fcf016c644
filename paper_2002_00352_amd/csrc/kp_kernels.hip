// gfx950 kernels of the per-user subproblem sweep.
//
// One block (256 threads, four wave64s) processes tiles of U users at a time:
//   phase 0  the tile's costs b are staged in LDS as a dense [U][M][K] tile
//            (coalesced 16-byte loads for dense b, a per-row scatter for CSR),
//   phase A  one thread per item row computes the cost-adjusted profit
//            p~ = p - sum_k lambda_k b_k  (FP64, k ascending, no FMA),
//   phase B1 one thread per user ranks its items by (p~ desc, index asc) and
//            runs the hierarchical greedy (Alg.1, as the equivalent laminar
//            matroid greedy on bitmasks),
//   phase B2 one thread per (user, knapsack) reduces consumption and, for SCD,
//            walks the user's consumption step function in lambda_k (the
//            breakpoints of Alg.3/4) and bins / emits them.
// R, g and P are summed in a fixed order: per (user,k) values go to LDS and
// are added in user order, per block into a private slot, and slots are
// added in block order by a second kernel.  The threshold search's sums
// (histogram bins, window corrections) are exact two-limb integers added
// with integer atomics, so their order does not matter.  This file also
// holds the threshold search's state machine, the post-processing, the
// batched plan's helpers and the input checks.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <algorithm>
#include <functional>
#include "kp_internal.h"

#define NT 256

#include "kp_device.h"

// ---------------------------------------------------------------------------
// the sweep kernel
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
#define CH 8      // prefetched 16-byte chunks of dense costs per thread and tile
#define PCH 4     // prefetched profits (and CSR row offsets) per thread and tile
#define ECH 8     // prefetched CSR entries per thread and tile

// Register-resident copy of one tile's inputs, loaded one tile ahead so the
// loads overlap the previous tile's compute.
struct Prefetch {
  v4f b4[CH];
  float pv[PCH];
  int64_t rp[PCH];      // CSR: rowptr of the rows this thread scores
  int64_t rp_end;       // CSR: rowptr one past the tile (valid in thread 0)
  int32_t ec[ECH];      // CSR entries of the tile, cooperative layout
  float ev[ECH];
};

template <int FMT>
__device__ __forceinline__ void issue_rows(Prefetch &f, const ProbDev &pr, int64_t u0, int nr, int K,
                                           int tid, int aligned) {
  // profits (all formats) and, for CSR, the row offsets
  #pragma unroll
  for (int i = 0; i < PCH; ++i) {
    const int r = tid + i * NT;
    if (r < nr) {
      f.pv[i] = __builtin_nontemporal_load(pr.p + u0 * pr.M + r);
      if (FMT == 1) f.rp[i] = pr.rowptr[u0 * pr.M + r];
    }
  }
  if (FMT == 1 && tid == 0) f.rp_end = pr.rowptr[u0 * pr.M + nr];
  if (FMT == 0 && aligned) {
    const float *src = pr.b + u0 * (int64_t)pr.M * K;
    const int n4 = (nr * K) >> 2;
    const v4f *s4 = (const v4f *)src;
    #pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int t = tid + i * NT;
      if (t < n4) f.b4[i] = __builtin_nontemporal_load(s4 + t);
    }
  }
}

__device__ __forceinline__ void issue_entries(Prefetch &f, const ProbDev &pr, int64_t e0, int64_t e1,
                                              int tid) {
  #pragma unroll
  for (int i = 0; i < ECH; ++i) {
    const int64_t e = e0 + tid + (int64_t)i * NT;
    if (e < e1) {
      f.ec[i] = __builtin_nontemporal_load(pr.col + e);
      f.ev[i] = __builtin_nontemporal_load(pr.val + e);
    }
  }
}

// The far-window test for at most one binding set (far_window_single) in
// two parts.  First pass: zmax, the selection outside the set (whose moving
// members must keep their sign: the smallest |z'| among those that may be
// positive is checked against the bound), and the set's positive members
// with their smallest z' and the best other members (all of them; moving
// ones).  Lines at or below -Hs
// never turn positive in the window (Hs may be an upper bound of the
// window's reach: the tests only grow more cautious).
struct FarPass {
  double zmax = 0.0, nearz = INFINITY;
  bool anyn = false;
  uint64_t sel = 0, posm = 0;
  double minpos = INFINITY, bestneg = -INFINITY, bestnegA = -INFINITY;
};
__device__ __forceinline__ void far_item(FarPass &f, double z, int j, bool moving, bool member, double Hs) {
  if (z > -Hs) f.zmax = fmax(f.zmax, fabs(z));
  if (member) {
    if (z > 0.0) {
      f.posm |= 1ull << j;
      f.minpos = fmin(f.minpos, z);
    } else {
      f.bestneg = fmax(f.bestneg, z);
      if (moving) f.bestnegA = fmax(f.bestnegA, z);
    }
  } else {
    if (moving && z > -Hs) { f.nearz = fmin(f.nearz, fabs(z)); f.anyn = true; }
    if (z > 0.0) f.sel |= 1ull << j;
  }
}
// The rest of the test from its first pass (Hs: the exact reach r bmk plus
// margin): at most c1 positive members -- T is all of them, the best member
// left out the best of the others; more -- T by passes over the set.
__device__ __forceinline__ bool far_finish(const FarPass &f, const double *zu, const float *bu, int M, int K,
                                           int k, uint64_t A, double lk, double dl, double r, double bmk,
                                           double Hs, uint64_t m1, int c1, double *cw) {
  const double bound = r * bmk * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + f.zmax + Hs + (lk + fabs(dl) + r) * bmk);
  if (f.anyn && !(f.nearz > bound)) return false;   // may change sign
  auto moved = [&](int j) -> double {
    const double b = (A >> j & 1) ? (double)bu[j * K + k] : 0.0;
    const double s = dl * b;
    return zu[j] - s;
  };
  uint64_t sel = f.sel;
  const int npos = popc64(f.posm);
  if (npos <= c1) {
    // at most c1 positive members: T is all of them, the best member left
    // out the best of the others (the same tests as below, no more passes)
    if (npos == c1 && f.bestneg > -Hs && !(f.minpos - f.bestneg > bound)) return false;
    if (npos > 0 && !(f.minpos > bound)) return false;
    if (npos < c1 && !(f.bestnegA < -bound)) return false;
    sel |= f.posm;
    double sum = 0.0;
    for (uint64_t m = sel & A; m; m &= m - 1) {
      const int j = __ffsll((long long)m) - 1;
      sum = sum + (double)bu[j * K + k];
    }
    *cw = sum;
    return true;
  }
  // more: T, the c1 best positive members (z' desc, index asc), taken two
  // per pass over the set (the second best of a pass is the best once the
  // first has joined T)
  uint64_t inT = 0;
  int nt = 0;
  double minT = INFINITY;
  for (;;) {
    double v1 = -INFINITY, v2 = -INFINITY;
    int j1 = -1, j2 = -1;
    #pragma unroll 4
    for (int j = 0; j < M; ++j) {
      if (!(m1 >> j & 1) || (inT >> j & 1)) continue;
      const double z = moved(j);
      if (z > v1) { v2 = v1; j2 = j1; v1 = z; j1 = j; }
      else if (z > v2) { v2 = z; j2 = j; }
    }
    bool done = false;
    for (int h = 0; h < 2 && !done; ++h) {
      const double best = h == 0 ? v1 : v2;
      const int bj = h == 0 ? j1 : j2;
      if (bj < 0) { done = true; break; }
      if (nt < c1 && best > 0.0) {
        inT |= 1ull << bj;
        minT = best;
        ++nt;
        continue;
      }
      // bj: the best member outside T
      if (nt == c1 && best > -Hs && !(minT - best > bound)) return false;
      done = true;
    }
    if (done) break;
  }
  if (nt > 0 && !(minT > bound)) return false;
  if (nt < c1) {
    // room is left: no moving member outside T may turn positive
    #pragma unroll 4
    for (int j = 0; j < M; ++j) {
      if (!(m1 >> j & 1) || (inT >> j & 1) || !(A >> j & 1)) continue;
      if (!(moved(j) < -bound)) return false;
    }
  }
  sel |= inT;
  double sum = 0.0;
  for (uint64_t m = sel & A; m; m &= m - 1) {
    const int j = __ffsll((long long)m) - 1;
    sum = sum + (double)bu[j * K + k];
  }
  *cw = sum;
  return true;
}

// The same test for at most one binding set (top-Q and the like: set mask
// m1 with cap c1, or no set), for any M, in O(M c1) with no per-item
// state: items outside the set are selected when positive, so a moving one
// must keep its sign over the window; inside the set the selection at c is
// the c1 best positive members T (picked by repeated maxima, two per pass
// over the set, ties to the lower index), and it stays the same when T
// stays positive and the best other member stays below T (one gap: every
// pair across it moves against each other by at most r bmax), or, when
// fewer than c1 members are positive, when no moving member outside T can
// turn positive.  Returns false when the test does not apply or fails; else
// true with *cw = the selection's consumption of k.
__device__ __forceinline__ bool far_window_single(const double *zu, const float *bu, int M, int K, int k,
                                                  uint64_t A, double lk, double wlo, double whi, double bmk,
                                                  uint64_t m1, int c1, double *cw) {
  const double c = 0.5 * (wlo + whi);
  const double r = fmax(whi - c, c - wlo);
  const double dl = c - lk;
  if (!(fabs(dl) > r)) return false;
  const double Hs = r * bmk * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (lk + fabs(dl) + r) * bmk);
  FarPass f;
  #pragma unroll 4
  for (int j = 0; j < M; ++j) {
    const double b = (A >> j & 1) ? (double)bu[j * K + k] : 0.0;
    const double s = dl * b;
    far_item(f, zu[j] - s, j, (A >> j & 1) != 0, (m1 >> j & 1) != 0, Hs);
  }
  return far_finish(f, zu, bu, M, K, k, A, lk, dl, r, bmk, Hs, m1, c1, cw);
}

// A window that does not contain lambda_k^t (an alternation window around
// lambda_k^{t-1}): move the user's lines to the window's centre c,
// z'_j = p~_j - (c - lambda_k^t) b_jk.  Over the window (radius r around c)
// a moving line moves by at most r b_jk, so no two lines cross in it (nor a
// moving line and zero) when every such gap between lines that can turn
// positive there exceeds r bmax plus a rounding margin; then the greedy set
// is the same over the whole window, and it is Alg.1 on the moved lines (in
// rank space, as a mask of ranks).  Returns false when the test does not
// apply or fails; else true with *cw = the set's consumption of k, in item
// order.  zu: p~ of the user's items, bu: its costs [M][K]; A: the items
// moving with k.  M <= 16.
__device__ __forceinline__ bool far_window_set(const double *zu, const float *bu, int M, int K, int k,
                                               uint64_t A, double lk, double wlo, double whi, double bmk,
                                               const TreeDev &T, double *cw) {
  const double c = 0.5 * (wlo + whi);
  const double r = fmax(whi - c, c - wlo);
  const double dl = c - lk;
  if (M > 16 || !(fabs(dl) > r)) return false;
  const double Hs = r * bmk * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (lk + fabs(dl) + r) * bmk);
  auto moved = [&](int j) -> double {
    const double b = (A >> j & 1) ? (double)bu[j * K + k] : 0.0;
    const double s = dl * b;
    return zu[j] - s;
  };
  uint64_t rk = 0;   // rank of every item by (z' desc, index asc), 4 bits each
  for (int j = 0; j < M; ++j) rk |= (uint64_t)j << (4 * j);
  uint64_t posc = 0;
  double gmin = 1e300, zmax = 0.0;
  for (int x = 0; x < M; ++x) {
    const double zx = moved(x);
    const bool mx = A >> x & 1, rx = zx > -Hs;
    if (zx > 0.0) posc |= 1ull << x;
    if (rx) zmax = fmax(zmax, fabs(zx));
    if (rx && mx) gmin = fmin(gmin, fabs(zx));
    for (int y = x + 1; y < M; ++y) {
      const double zy = moved(y);
      if (zy > zx) { rk += 1ull << (4 * x); rk -= 1ull << (4 * y); }
      // pairs that can cross: at least one moves, and not two equal lines
      // with equal costs in k (they coincide over the whole window)
      const bool my = A >> y & 1;
      if (rx && zy > -Hs && (mx || my) && !(zx == zy && bu[x * K + k] == bu[y * K + k]))
        gmin = fmin(gmin, fabs(zx - zy));
    }
  }
  const double need = r * bmk * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + zmax + Hs + (lk + fabs(dl) + r) * bmk);
  if (!(gmin > need)) return false;
  uint32_t alive = 0;
  for (int j = 0; j < M; ++j)
    if (posc >> j & 1) alive |= 1u << ((rk >> (4 * j)) & 15);
  for (int l = 0; l < T.L; ++l) {
    const uint64_t m = T.mask[l];
    uint32_t mr = 0;
    for (int j = 0; j < M; ++j)
      if (m >> j & 1) mr |= 1u << ((rk >> (4 * j)) & 15);
    uint32_t x = alive & mr;
    for (int q = 0; q < T.cap[l]; ++q) x &= x - 1u;
    alive &= ~x;
  }
  double sum = 0.0;
  for (int j = 0; j < M; ++j)
    if ((A >> j & 1) && (alive >> ((rk >> (4 * j)) & 15) & 1)) sum = sum + (double)bu[j * K + k];
  *cw = sum;
  return true;
}

// MX, KX: the item and knapsack counts when they are fixed at compile time
// (dense costs with M = K = 10, or M = 20 and K = 50), else 0: the loops
// over the items and the knapsacks then have constant trip counts (c2 SCD
// step 3.50 -> 3.25 ms; c4 SCD 28.4 -> 27.6 ms, DD 9.02 -> 8.58 ms).
template <int FMT, bool SCD, int MX = 0, int KX = 0>
__device__ __forceinline__ void sweep_body(const SweepArgs &a, const TileGeom &g, const int bid,
                                           const int nblk, unsigned char *smem) {
  const int tid = threadIdx.x;
  const int M = MX ? MX : g.M, K = KX ? KX : g.K, U = g.U;
  const int R = U * M;             // item rows per tile
  const int Q = U * K;             // (user, knapsack) pairs per tile
  // ---- LDS carve-up (byte offsets are multiples of 16) ----
  size_t off = 0;
  auto carve = [&](size_t bytes) { unsigned char *p = smem + off; off += (bytes + 15) & ~(size_t)15; return p; };
  float *bt = (float *)carve((size_t)R * K * 4);          // [U][M][K]
  double *pt = (double *)carve((size_t)R * 8);            // [U][M]
  uint8_t *perm = (uint8_t *)carve((size_t)R);            // [U][M] rank -> item
  uint64_t *Sm = (uint64_t *)carve((size_t)U * 8);        // greedy set at lambda^t
  uint64_t *Pm = (uint64_t *)carve((size_t)U * 8);        // items with p~ > 0
  int8_t *tau = (int8_t *)carve(SCD ? (size_t)R : 0);     // per item: threshold element (-1 = zero level)
  double *vk = (double *)carve((size_t)Q * 8);            // per (user,k) consumption
  double *uPG = (double *)carve((size_t)U * 16);          // per user P_i, G_i
  double *acc = (double *)carve((size_t)(K + 2) * 8);     // block running sums
  double *lam = (double *)carve((size_t)K * 8);           // lambda^t staged once per block
  float *pl = (float *)carve((size_t)R * 4);              // staged profits
  int32_t *rpl = (int32_t *)carve((size_t)(R + 1) * 4);   // CSR: row offsets relative to the tile
  int32_t *ecl = (int32_t *)carve(FMT == 1 ? (size_t)NT * ECH * 4 : 0);  // CSR: staged entries
  float *evl = (float *)carve(FMT == 1 ? (size_t)NT * ECH * 4 : 0);
  int64_t *ebase = (int64_t *)carve(16);                  // CSR: first entry of the next tile
  KState *kst = SCD ? (KState *)carve((size_t)K * sizeof(KState)) : nullptr;
  XSum *hs = nullptr;
  uint32_t *hc = nullptr;
  const bool hist = !a.no_hist;   // histograms (exponential buckets, refinement bins) in LDS
  int *kmode = nullptr;
  uint32_t *kcnt = nullptr, *kpos = nullptr, *kovf = nullptr, *nstage = nullptr;
  unsigned long long *hmin = nullptr, *hmax = nullptr;
  double *kwide = nullptr, *ugap = nullptr;
  XSum *kxs = nullptr;
  if (SCD) {
    kwide = (double *)carve(16);                   // the widest window
    kxs = (XSum *)carve((size_t)K * sizeof(XSum)); // window corrections
    ugap = (double *)carve((size_t)U * 16);        // per user: gap and scale of the window filter
    if (hist) {
      hs = (XSum *)carve((size_t)K * KP_NB * sizeof(XSum));
      hc = (uint32_t *)carve((size_t)K * KP_NB * 4);
    }
    kmode = (int *)carve((size_t)K * 4);
    kcnt = (uint32_t *)carve((size_t)K * 4);
    kpos = (uint32_t *)carve((size_t)K * 4);
    kovf = (uint32_t *)carve((size_t)K * 4);
    hmin = (unsigned long long *)carve((size_t)K * 8);
    hmax = (unsigned long long *)carve((size_t)K * 8);
    nstage = (uint32_t *)carve(16);
  }
  for (int t = tid; t < K + 2; t += NT) acc[t] = 0.0;
  for (int t = tid; t < K; t += NT) lam[t] = a.lam[t];
  if (SCD) {
    for (int t = tid; t < K; t += NT) kst[t] = a.st[t];
    if (hist)
      for (int t = tid; t < K * KP_NB; t += NT) { hs[t] = xs_zero(); hc[t] = 0u; }
    for (int t = tid; t < K; t += NT) {
      kmode[t] = a.st[t].mode;
      kcnt[t] = 0u;
      kpos[t] = 0u;
      kovf[t] = 0u;
      hmin[t] = ~0ull;
      hmax[t] = 0ull;
      kxs[t] = xs_zero();
    }
    if (tid == 0) {
      *nstage = 0u;
      double m = 0.0;
      for (int k = 0; k < K; ++k)
        if (a.st[k].mode == KS_WINDOW) m = a.st[k].hw > m ? a.st[k].hw : m;
      kwide[0] = m;
    }
  }
  const int64_t N = a.pr.N;
  if (SCD && !a.want_stats) {
    __syncthreads();
    __shared__ int busy;
    if (tid == 0) busy = 0;
    __syncthreads();
    for (int t = tid; t < K; t += NT)
      if (walk_mode(kmode[t])) busy = 1;
    __syncthreads();
    if (!busy) return;
  }

  // ---- software pipeline: prefetch tile bid ----
  Prefetch f;
  int64_t tile = bid;
  if (tile < a.ntiles) {
    const int64_t u0 = tile * (int64_t)U;
    const int nu = (int)((N - u0) < U ? (N - u0) : U);
    issue_rows<FMT>(f, a.pr, u0, nu * M, K, tid, g.aligned);
    if (FMT == 1) {
      if (tid == 0) { ebase[0] = a.pr.rowptr[u0 * M]; ebase[1] = f.rp_end; }
      __syncthreads();
      issue_entries(f, a.pr, ebase[0], ebase[1], tid);
    }
  }

  for (; tile < a.ntiles; tile += nblk) {
    const int64_t u0 = tile * (int64_t)U;
    const int nu = (int)((N - u0) < U ? (N - u0) : U);     // users in this tile
    const int nr = nu * M;
    __syncthreads();   // previous tile's readers are done with the LDS tile
    // ---- store the prefetched tile into LDS ----
    int64_t e_first = 0;
    int n_ent = 0;
    #pragma unroll
    for (int i = 0; i < PCH; ++i) {
      const int r = tid + i * NT;
      if (r < nr) pl[r] = f.pv[i];
    }
    if (FMT == 0) {
      const float *src = a.pr.b + u0 * (int64_t)M * K;
      const int nf = nr * K;
      if (g.aligned) {
        const int n4 = nf >> 2;
        v4f *d4 = (v4f *)bt;
        #pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int t = tid + i * NT;
          if (t < n4) d4[t] = f.b4[i];
        }
        // beyond the prefetched chunks, and the ragged tail: direct loads
        const v4f *s4 = (const v4f *)src;
        for (int t = tid + CH * NT; t < n4; t += NT) d4[t] = s4[t];
        for (int t = (n4 << 2) + tid; t < nf; t += NT) bt[t] = src[t];
      } else {
        for (int t = tid; t < nf; t += NT) bt[t] = src[t];
      }
    } else {
      e_first = ebase[0];
      n_ent = (int)(ebase[1] - ebase[0]);
      #pragma unroll
      for (int i = 0; i < PCH; ++i) {
        const int r = tid + i * NT;
        if (r < nr) rpl[r] = (int32_t)(f.rp[i] - e_first);
      }
      if (tid == 0) rpl[nr] = n_ent;
      #pragma unroll
      for (int i = 0; i < ECH; ++i) {
        const int t = tid + i * NT;
        if (t < n_ent && t < NT * ECH) { ecl[t] = f.ec[i]; evl[t] = f.ev[i]; }
      }
      for (int t = tid; t < R * K; t += NT) bt[t] = 0.0f;
    }
    // ---- issue the next tile's loads (they land during this tile's compute) ----
    const int64_t ntile = tile + nblk;
    int64_t nu0 = 0;
    int nnr = 0;
    if (ntile < a.ntiles) {
      nu0 = ntile * (int64_t)U;
      nnr = (int)((N - nu0) < U ? (N - nu0) : U) * M;
      issue_rows<FMT>(f, a.pr, nu0, nnr, K, tid, g.aligned);
    }
    // at most one (pruned) set, e.g. top-Q: every row decides its own
    // selection in the rank phase; the users' masks start empty
    const bool fastsel = a.tree.L <= 1;
    if (fastsel && tid < nu) Sm[tid] = 0ull;
    // with at most one set the threshold elements follow from two items per
    // user, found by the rank phase: [0] the set's lowest selected member
    // (set full) and [1] its best positive member left out
    const bool fastau = SCD && fastsel && M >= 2;
    if (fastau && tid < nu) { tau[tid * M] = -1; tau[tid * M + 1] = -1; }
    // window filter, per user: [0] the smallest gap (a minimum over the
    // rows, taken on the bits of non-negative doubles), [1] the largest cost
    // (a maximum over the rows, on the bits of a non-negative float)
    if (SCD && tid < nu) {
      ((unsigned long long *)ugap)[2 * tid] = (unsigned long long)__double_as_longlong(1e300);
      ((unsigned int *)ugap)[4 * tid + 2] = 0u;
    }
    __syncthreads();
    // ---- phase A: scores ----
    if (FMT == 0) {
      for (int r = tid; r < nr; r += NT) {
        double accp = (double)pl[r];
        const float *br = bt + (size_t)r * K;
        #pragma unroll 4
        for (int k = 0; k < K; ++k) {
          const double prod = lam[k] * (double)br[k];
          accp = accp - prod;
        }
        pt[r] = accp;
      }
    } else {
      // CSR: scatter each row's stored entries into the dense tile and score
      // over the stored columns in ascending order (skipping zeros is
      // bit-identical: acc - lambda*0 == acc)
      for (int r = tid; r < nr; r += NT) {
        const int e0 = rpl[r], e1 = rpl[r + 1];
        double accp = (double)pl[r];
        for (int e = e0; e < e1; ++e) {
          int k;
          float v;
          if (e < NT * ECH) { k = ecl[e]; v = evl[e]; }
          else { k = a.pr.col[e_first + e]; v = a.pr.val[e_first + e]; }   // tile beyond the staging
          if ((unsigned)k >= (unsigned)K) continue;   // malformed column: ignored (kp_validate_inputs reports it)
          bt[(size_t)r * K + k] = v;
          const double prod = lam[k] * (double)v;
          accp = accp - prod;
        }
        pt[r] = accp;
      }
    }
    __syncthreads();
    // ---- phase B1a: rank of every item of every user (one thread per row) ----
    const uint64_t m1 = a.tree.L == 1 ? a.tree.mask[0] : 0ull;
    const int c1 = a.tree.L == 1 ? a.tree.cap[0] : 0;
    for (int r = tid; r < nr; r += NT) {
      const int u = r / M, j = r - u * M;
      const double *z = pt + u * M;
      const double zj = z[j];
      int rank = 0, rank1 = 0;
      #pragma unroll 4
      for (int jj = 0; jj < M; ++jj) {
        const double zz = z[jj];
        const int beats = (zz > zj) || (zz == zj && jj < j);
        rank += beats;
        rank1 += beats & (int)(m1 >> jj & 1);
      }
      perm[u * M + rank] = (uint8_t)j;
      if (SCD && kwide[0] > 0.0) {
        // largest positive cost of the row (0 if none): the maximum below
        // is taken over the users' rows as unsigned bits, which order like
        // the floats for positive values
        const float *br = bt + (size_t)r * K;
        float mx = 0.0f;
        #pragma unroll 4
        for (int k = 0; k < K; ++k) mx = br[k] > mx ? br[k] : mx;
        if (mx > 0.0f) atomicMax((unsigned int *)ugap + 4 * u + 2, __float_as_uint(mx));
      }
      // Alg.1 with at most one set: a positive item is kept unless it is in
      // the set behind cap better members of it (those are positive too)
      if (fastsel && zj > 0.0 && (!(m1 >> j & 1) || rank1 < c1))
        atomicOr((unsigned long long *)&Sm[u], 1ull << j);
      if (fastau && zj > 0.0 && (m1 >> j & 1)) {
        if (rank1 == c1 - 1) tau[u * M] = (int8_t)j;
        else if (rank1 == c1) tau[u * M + 1] = (int8_t)j;
      }
    }
    // CSR: the next tile's entry range is known now that its row offsets have
    // landed; start those loads too
    if (FMT == 1 && ntile < a.ntiles) {
      if (tid == 0) { ebase[0] = f.rp[0]; ebase[1] = f.rp_end; }
    }
    __syncthreads();
    if (FMT == 1 && ntile < a.ntiles) issue_entries(f, a.pr, ebase[0], ebase[1], tid);
    // ---- phase B1b: the greedy, one thread per user ----
    if (tid < nu) {
      const int u = tid;
      const double *z = pt + u * M;
      uint64_t pos = 0;
      #pragma unroll 4
      for (int j = 0; j < M; ++j) if (z[j] > 0.0) pos |= 1ull << j;
      const uint64_t S = fastsel ? Sm[u] : greedy_mask(perm + u * M, M, pos, a.tree);
      Sm[u] = S;
      Pm[u] = pos;
      if (SCD && !fastau) {
        // Threshold element of every item o against the greedy solution G_o of
        // the other items (their order does not depend on lambda_k when o is
        // the only item that moves with it): o is selected exactly when its
        // line beats that element (or is positive, for the zero level -1).
        //   o not in S: G_o = S; the lowest-ranked member of S in the smallest
        //     full set containing o, or the zero level if no set containing o
        //     is full.
        //   o in S: G_o = S - o + r(o) with r(o) the best positive item outside
        //     S whose smallest full set contains o; the threshold is r(o), or
        //     the zero level when there is none.
        const uint8_t *pu = perm + u * M;
        int8_t *tu = tau + u * M;
        uint64_t assigned = S;   // items outside S get their value below
        for (int l = 0; l < a.tree.L; ++l) {
          const uint64_t m = a.tree.mask[l];
          if (popc64(S & m) < a.tree.cap[l]) continue;
          uint64_t pend = m & ~assigned;
          if (!pend) continue;
          int low = -1;
          for (int r = M - 1; r >= 0; --r) {
            const int j = pu[r];
            if ((S & m) >> j & 1) { low = j; break; }
          }
          assigned |= pend;
          while (pend) {
            const int o = __ffsll((long long)pend) - 1;
            pend &= pend - 1;
            tu[o] = (int8_t)low;
          }
        }
        uint64_t rest = ~assigned & ((M == 64) ? ~0ull : ((1ull << M) - 1));
        while (rest) {
          const int o = __ffsll((long long)rest) - 1;
          rest &= rest - 1;
          tu[o] = -1;
        }
        uint64_t resolved = 0;
        for (int r = 0; r < M && resolved != S; ++r) {
          const int e = pu[r];
          if ((S >> e & 1) || !(pos >> e & 1)) continue;
          uint64_t lm = 0;
          for (int l = 0; l < a.tree.L; ++l) {
            const uint64_t m = a.tree.mask[l];
            if ((m >> e & 1) && popc64(S & m) >= a.tree.cap[l]) { lm = m; break; }
          }
          uint64_t nw = S & lm & ~resolved;
          resolved |= nw;
          while (nw) {
            const int o = __ffsll((long long)nw) - 1;
            nw &= nw - 1;
            tu[o] = (int8_t)e;
          }
        }
        uint64_t left = S & ~resolved;
        while (left) {
          const int o = __ffsll((long long)left) - 1;
          left &= left - 1;
          tu[o] = -1;
        }
      }
      // sums over the selected items in ascending index order
      double Pi = 0.0, Gi = 0.0;
      const float *pp = pl + u * M;
      for (uint64_t m = S; m; m &= m - 1) {
        const int j = __ffsll((long long)m) - 1;
        Pi = Pi + (double)pp[j];
        Gi = Gi + z[j];
      }
      uPG[2 * u] = Pi;
      uPG[2 * u + 1] = Gi;
      if (a.x_out) {
        uint8_t *xo = a.x_out + (u0 + u) * M;
        for (int j = 0; j < M; ++j) xo[j] = (uint8_t)(S >> j & 1);
      }
    }
    if (SCD && kwide[0] > 0.0) {
      // window filter, one thread per rank position: the smallest gap
      // between a user's p~ in rank order and between them and zero, over
      // the lines that can turn positive inside the widest window (ranks
      // descend, so those are a prefix of the ranks); two identical lines
      // (equal p~ and equal costs in every knapsack, e.g. the copies of a
      // categorical item) never cross
      const double hm = kwide[0];
      for (int q = tid; q < nr; q += NT) {
        const int u = q / M, rr = q - u * M;
        const float bm = __uint_as_float(((const unsigned int *)ugap)[4 * u + 2]);
        const double H = hm * (double)bm * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (double)bm * hm);
        const double *z = pt + u * M;
        const int jv = perm[u * M + rr];
        const double v = z[jv];
        if (!(v > -H)) continue;
        double c = fabs(v);
        if (rr > 0) {
          const int jp = perm[u * M + rr - 1];
          const double prev = z[jp];
          bool same = prev == v;
          const float *ba = bt + ((size_t)u * M + jp) * K, *bb = bt + ((size_t)u * M + jv) * K;
          for (int k = 0; same && k < K; ++k) same = ba[k] == bb[k];
          if (!same) c = prev - v < c ? prev - v : c;
        }
        atomicMin((unsigned long long *)ugap + 2 * u, (unsigned long long)__double_as_longlong(c));
      }
    }
    __syncthreads();
    // ---- phase B2: one thread per (user, knapsack) ----
    for (int q = tid; q < nu * K; q += NT) {
      const int u = q / K, k = q - u * K;
      const uint64_t S0 = Sm[u];
      const float *bu = bt + (size_t)u * M * K;
      double v = 0.0;
      uint64_t A = 0;     // SCD: moving lines, b_jk > 0
      float bmk = 0.0f;   // SCD: their largest cost
      // a window away from lambda_k^t with at most one binding set: the
      // far-window test's first pass runs in the same pass over the items
      // (its cut at -Hs taken with the user's largest cost over every
      // knapsack, an upper bound of bmk: only more cautious)
      bool fused = false, fused_ok = false;
      double fused_cw = 0.0;
      // a user with no line above -H (its gap record untouched) is calm in
      // every window: only its consumption is needed (A stays empty, so no
      // test or walk follows)
      const bool settled = SCD && kmode[k] == KS_WINDOW && kwide[0] > 0.0 && !(ugap[2 * u] < 1e300);
      if (settled) {
        for (uint64_t m = S0; m; m &= m - 1) v = v + (double)bu[(__ffsll((long long)m) - 1) * K + k];
      } else if (SCD) {
        double fr = 0.0, fdl = 0.0;
        if (kmode[k] == KS_WINDOW && a.tree.L <= 1 && kwide[0] > 0.0) {
          const double wlo = kst[k].wlo, whi = kst[k].whi;
          const double c = 0.5 * (wlo + whi);
          fr = fmax(whi - c, c - wlo);
          fdl = c - lam[k];
          fused = fabs(fdl) > fr;
        }
        if (fused) {
          const double *zu = pt + u * M;
          const double lk = lam[k];
          const uint64_t m1 = a.tree.L == 1 ? a.tree.mask[0] : 0ull;
          const double bmu = (double)__uint_as_float(((const unsigned int *)ugap)[4 * u + 2]);
          const double Hup = fr * bmu * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (lk + fabs(fdl) + fr) * bmu);
          FarPass f;
          #pragma unroll 4
          for (int j = 0; j < M; ++j) {
            const float bj = bu[j * K + k];
            if (S0 >> j & 1) v = v + (double)bj;
            const bool mov = bj > 0.0f;
            if (mov) A |= 1ull << j;
            bmk = bj > bmk ? bj : bmk;
            const double b = mov ? (double)bj : 0.0;
            const double sh = fdl * b;
            far_item(f, zu[j] - sh, j, mov, (m1 >> j & 1) != 0, Hup);
          }
          const double Hs = fr * (double)bmk * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (lk + fabs(fdl) + fr) * (double)bmk);
          fused_ok = far_finish(f, zu, bu, M, K, k, A, lk, fdl, fr, (double)bmk, Hs, m1,
                                a.tree.L == 1 ? a.tree.cap[0] : 0, &fused_cw);
        } else {
          #pragma unroll 4
          for (int j = 0; j < M; ++j) {
            const float bj = bu[j * K + k];
            if (S0 >> j & 1) v = v + (double)bj;
            if (bj > 0.0f) A |= 1ull << j;
            bmk = bj > bmk ? bj : bmk;
          }
        }
      } else {
        // the selected items only, in ascending index order
        for (uint64_t m = S0; m; m &= m - 1) v = v + (double)bu[(__ffsll((long long)m) - 1) * K + k];
      }
      vk[q] = v;
      if (SCD) {
        const int mode = kmode[k];
        if (walk_mode(mode)) {
          const double lk = lam[k];
          const double *zu = pt + u * M;
          bool walk = A != 0;
          if (walk && !hist && (mode == KS_EXP || mode == KS_REFINE)) {
            atomicAdd(a.err, 1ull);   // launched without the histograms these modes need
            walk = false;
          }
          if (walk && mode == KS_WINDOW) {
            // no breakpoint of this user inside the window: nothing to emit
            // and its consumption just above the window is v_ik (no correction)
            double cw = fused_cw;
            // the filter's scale: |top p~| + H, with H from the user's
            // largest cost and the widest window
            const float bmu = __uint_as_float(((const unsigned int *)ugap)[4 * u + 2]);
            const double hm = kwide[0];
            const double Hu = hm * (double)bmu * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + (double)bmu * hm);
            const double gscale = fabs(zu[perm[u * M]]) + Hu;
            if (window_calm(ugap[2 * u], gscale, kst[k].hw, (double)bmk, lk)) {
              walk = false;
            } else if (fused ? fused_ok
                             : a.tree.L <= 1
                                 ? far_window_single(zu, bu, M, K, k, A, lk, kst[k].wlo, kst[k].whi, (double)bmk,
                                                     a.tree.L == 1 ? a.tree.mask[0] : 0ull,
                                                     a.tree.L == 1 ? a.tree.cap[0] : 0, &cw)
                                 : far_window_set(zu, bu, M, K, k, A, lk, kst[k].wlo, kst[k].whi, (double)bmk,
                                                  a.tree, &cw)) {
              // no breakpoint inside the window: its consumption just above
              // the window is the window's set's
              walk = false;
              if (cw != v) {
                xs_atomic_add_sum(&kxs[k], xs_minus(xs_of(cw), xs_of(v)));
              }
            } else {
              auto line = [&](int j, double &c, double &b) {
                b = (A >> j & 1) ? (double)bu[j * K + k] : 0.0;
                const double add = lk * b;
                c = zu[j] + add;
              };
              const double whi = kst[k].whi, wlo = kst[k].wlo;
              if (window_keeps(S0, A, Pm[u] & ~S0, line, a.tree.mask, a.tree.cap, a.tree.L, whi, 1) &&
                  window_keeps(S0, A, Pm[u] & ~S0, line, a.tree.mask, a.tree.cap, a.tree.L, wlo,
                               wlo > 0.0 ? -1 : 1))
                walk = false;
            }
          }
          if (walk) {
            double above = 0.0;   // window: increments of the breakpoints above it
            const KState &ks = kst[k];
            const double center = ks.center, delta = ks.delta;
            const int bstar = ks.bstar;
            const uint64_t klo = ks.klo, khi = ks.khi;
            const int shift = ks.shift;
            const int maxev = M * M + M + 8;
            const bool single = (A & (A - 1)) == 0;
            // start above every breakpoint: only horizontal positive lines,
            // ranked by p~ (their lines are c_j = p~_j exactly)
            uint64_t S = single ? 0ull : greedy_mask(perm + u * M, M, Pm[u] & ~A, a.tree);
            for (int ev = 0; ; ++ev) {
              if (ev >= maxev) { atomicAdd(a.err, 1ull); break; }
              if (single && ev > 0) break;
              double best = 0.0;
              int bo = -1, bs = -1;
              uint64_t cand = single ? 0ull : (A & ~S);
              if (single) {
                // one moving line: its only breakpoint is where it crosses its
                // threshold element (a horizontal line) or the zero level
                const int o = __ffsll((long long)A) - 1;
                // with one set: the lowest selected member when o is out,
                // the best member left out when o is in (set full), else zero
                const int th = !fastau ? (int)tau[u * M + o]
                               : (!(m1 >> o & 1) || tau[u * M] < 0) ? -1
                               : (int)tau[u * M + ((S0 >> o & 1) ? 1 : 0)];
                const double bo_d = (double)bu[o * K + k];
                const double add_o = lk * bo_d;
                const double co = zu[o] + add_o;
                if (th < 0) {
                  if (co > 0.0) { best = co / bo_d; bo = o; bs = -1; }
                } else {
                  const double bs_d = 0.0;
                  const double add_s = lk * bs_d;
                  const double cs = zu[th] + add_s;
                  const double num = co - cs;
                  const double den = bo_d - bs_d;
                  const double val = num / den;
                  if (val > 0.0) { best = val; bo = o; bs = th; }
                }
              }
              while (cand) {
                const int o = __ffsll((long long)cand) - 1;
                cand &= cand - 1;
                const double bo_d = (double)bu[o * K + k];
                const double add_o = lk * bo_d;
                const double co = zu[o] + add_o;
                // lowest full node containing o (nodes are ordered subsets first)
                uint64_t circ = 0;
                bool tight = false;
                for (int l = 0; l < a.tree.L; ++l) {
                  const uint64_t m = a.tree.mask[l];
                  if ((m >> o & 1) && popc64(S & m) >= a.tree.cap[l]) { circ = S & m; tight = true; break; }
                }
                // candidates are compared with the running maximum through
                // cr_gt (fma residuals), so a division is only taken for a
                // crossing that beats it: the same decisions as comparing
                // the divided crossings
                if (!tight) {
                  if (co > 0.0 && cr_gt(co, bo_d, best)) { best = co / bo_d; bo = o; bs = -1; }
                } else {
                  while (circ) {
                    const int s = __ffsll((long long)circ) - 1;
                    circ &= circ - 1;
                    const float bsf = bu[s * K + k];
                    if ((double)bsf < bo_d) {
                      const double bs_d = (double)bsf;
                      const double add_s = lk * bs_d;
                      const double cs = zu[s] + add_s;
                      const double num = co - cs;
                      const double den = bo_d - bs_d;
                      if (cr_gt(num, den, best)) { best = num / den; bo = o; bs = s; }
                    }
                  }
                }
              }
              if (bo < 0) break;
              const double bo_d = (double)bu[bo * K + k];
              const double v2 = bs >= 0 ? bo_d - (double)bu[bs * K + k] : bo_d;
              S = (S | (1ull << bo)) & ~(bs >= 0 ? (1ull << bs) : 0ull);
              if (mode == KS_WINDOW) {
                const uint64_t key = dkey(best);
                if (key < klo) break;                 // every later breakpoint is lower
                if (key > khi) { above = above + v2; continue; }
              }
              record_event(a, ks, k, best, v2, mode, hs, hc, hmin, hmax, kcnt, kovf, nstage, bid);
            }
            if (mode == KS_WINDOW && above != v) {
              xs_atomic_add_sum(&kxs[k], xs_minus(xs_of(above), xs_of(v)));
            }
          }
        }
      }
    }
    __syncthreads();
    // ---- fixed-order sums of the tile into the block accumulators ----
    if (a.want_stats) {
      for (int k = tid; k < K; k += NT) {
        double s = 0.0;
        #pragma unroll 4
        for (int u = 0; u < nu; ++u) s = s + vk[u * K + k];
        acc[k] = acc[k] + s;
      }
      if (tid == NT - 1) {
        double sp = 0.0, sg = 0.0;
        for (int u = 0; u < nu; ++u) { sp = sp + uPG[2 * u]; sg = sg + uPG[2 * u + 1]; }
        acc[K] = acc[K] + sg;
        acc[K + 1] = acc[K + 1] + sp;
      }
    }
  }
  __syncthreads();
  if (a.want_stats) {
    for (int t = tid; t < K + 2; t += NT) a.partials[(size_t)bid * (K + 2) + t] = acc[t];
  }
  if (SCD) publish_block(a, K, hs, hc, hmin, hmax, kcnt, kpos, kovf, nstage, tid, NT, bid, kxs);
}


template <int FMT, bool SCD, int MX = 0, int KX = 0>
__global__ void __launch_bounds__(NT) k_sweep(const SweepArgs a, const TileGeom g) {
  extern __shared__ __align__(16) unsigned char smem[];
  sweep_body<FMT, SCD, MX, KX>(a, g, blockIdx.x, gridDim.x, smem);
}

// the general kernel for a shape (dense costs with M = K = 10, or M = 20
// and K = 50: the counts compiled in)
static const void *sweep_fn(int fmt, bool scd, int M, int K) {
  if (fmt == 0 && M == 10 && K == 10)
    return scd ? (const void *)k_sweep<0, true, 10, 10> : (const void *)k_sweep<0, false, 10, 10>;
  if (fmt == 0 && M == 20 && K == 50)
    return scd ? (const void *)k_sweep<0, true, 20, 50> : (const void *)k_sweep<0, false, 20, 50>;
  if (fmt == 0) return scd ? (const void *)k_sweep<0, true> : (const void *)k_sweep<0, false>;
  return scd ? (const void *)k_sweep<1, true> : (const void *)k_sweep<1, false>;
}

// Batched: blocks [block_off[s], block_off[s+1]) work on instance s, whose
// arguments are copied into LDS; one launch covers every instance.  n_dev:
// the instance count read from the device (a split made there; blocks past
// the last instance's range exit at once), else n_inst.
// at most 168 VGPRs: three waves per SIMD
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3, 8))) k_sweep_batched(const SweepArgs *descs, const TileGeom *geoms,
                                                      const int *block_off, int n_inst, const int *n_dev) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ SweepArgs sa;
  __shared__ TileGeom sg;
  __shared__ int inst;
  if (n_dev) {
    n_inst = *n_dev;
    if (n_inst <= 0 || (int)blockIdx.x >= block_off[n_inst]) return;
  }
  if (threadIdx.x == 0) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {   // last s with block_off[s] <= blockIdx.x
      const int mid = (lo + hi + 1) >> 1;
      if (block_off[mid] <= (int)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    inst = lo;
  }
  __syncthreads();
  const int s = inst;
  {
    const int *src = (const int *)(descs + s);
    int *dst = (int *)&sa;
    for (int t = threadIdx.x; t < (int)(sizeof(SweepArgs) / 4); t += NT) dst[t] = src[t];
    if (threadIdx.x == 0) sg = geoms[s];
  }
  __syncthreads();
  const int bid = blockIdx.x - block_off[s];
  const int nblk = block_off[s + 1] - block_off[s];
  if (sa.pr.fmt == 0) sweep_body<0, true>(sa, sg, bid, nblk, smem);
  else sweep_body<1, true>(sa, sg, bid, nblk, smem);
}

// ---------------------------------------------------------------------------
// second-level reduction of the block partials (fixed order), dual value
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_reduce_stats(const double *partials, int nblk, int K,
                                                      const double *lam, const double *B,
                                                      double *R, double *g, double *P) {
  // one block per output column (K consumptions, then sum G_i, then sum P_i);
  // every thread adds a fixed strided subset, then a fixed tree: deterministic
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < nblk; b += 256) s = s + partials[(size_t)b * (K + 2) + c];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = red[t] + red[t + w];
    __syncthreads();
  }
  if (t != 0) return;
  s = red[0];
  if (c < K) {
    if (R) R[c] = s;
  } else if (c == K) {
    // g = sum_i G_i + sum_k lambda_k B_k
    double tt = s;
    for (int k = 0; k < K; ++k) { const double lb = lam[k] * B[k]; tt = tt + lb; }
    if (g) *g = tt;
  } else {
    if (P) *P = s;
  }
}

// ---------------------------------------------------------------------------
// SCD threshold search
// ---------------------------------------------------------------------------
// The window a search starts with, from the multiplier's history: around
// lambda_k^t, 1.25x the last step wide, when that step was small against
// lambda_k^t; else, when the multiplier alternates (it returns close to
// lambda_k^{t-1}: the drift |lambda^t - lambda^{t-2}| is under 1/8 of the
// last step), around lambda_k^{t-1}, 1.25x the drift wide.  hw is the
// farthest window edge from lambda_k^t (the filters bound the lines'
// movement by it).  step, prev, drift < 0 or NaN: unknown.
// Half-widths are at least 2^-20 of the centre: near convergence a
// multiplier's step or its 2-cycle drift can shrink to almost nothing and
// then move by more than that once, and a window that misses costs a full
// pass, while a few hundred more listed users cost little.
__device__ __forceinline__ void choose_window(KState &s, double step, double prev, double drift) {
  double c = 0.0, h = 0.0;
  if (step > 0.0 && KP_WIN_MULT * step <= KP_WIN_MAX_REL * s.center) {
    c = s.center;
    h = fmax(KP_WIN_MULT * step, s.center * 0x1p-20);
  } else if (step > 0.0 && drift >= 0.0 && prev >= 0.0 && drift * 8.0 <= step) {
    const double floor_ = (prev > 0x1p-20 ? prev : 0x1p-20) * 0x1p-20;
    c = prev;
    h = KP_WIN_MULT * (drift > floor_ ? drift : floor_);
  } else {
    return;
  }
  s.mode = KS_WINDOW;
  s.whi = c + h;
  s.wlo = c - h > 0.0 ? c - h : 0.0;
  const double up = s.whi - s.center, dn = s.center - s.wlo;
  s.hw = fmax(fabs(up), fabs(dn));
  s.klo = dkey(s.wlo);
  s.khi = dkey(s.whi);
}

__global__ void k_scd_init(KState *st, int K, const double *lam_in, const uint8_t *kmask,
                           double *hist, int hinted_in, int window, int interp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  KState s;
  s.mode = (kmask && !kmask[k]) ? KS_DONE : KS_EXP;
  s.bstar = 0;
  s.shift = 0;
  s.overflow = 0;
  s.n_emit = 0;
  s.flags = 0;
  s.center = lam_in[k];
  // hist: [K] bucket widths and [K] last steps (valid when hinted_in), then
  // [K] lambda^{t-1} and [K] lambda^{t-2} (NaN while unknown), shifted here
  // once per iteration
  const double *delta_hint = (hist && hinted_in) ? hist : nullptr;
  double d = delta_hint ? delta_hint[k] : 0.0;
  const bool hinted = d > 0.0;
  double prev = -1.0, drift = -1.0;
  if (hist) {
    prev = hist[2 * K + k];
    const double prev2 = hist[3 * K + k];
    drift = fabs(lam_in[k] - prev2);   // NaN while unknown
    hist[3 * K + k] = prev;
    hist[2 * K + k] = lam_in[k];
  }
  if (interp) {
    // interpolated reduce: a fixed fine central bucket, 2^-20 of the
    // multiplier (of 2^-20 when it is smaller), a power of two
    const double base = lam_in[k] > 0x1p-20 ? lam_in[k] : 0x1p-20;
    d = ldexp(1.0, ilogb(base) - 20);
  } else if (!hinted) {
    // no history: 2^-10 of the multiplier, a power of two; at a multiplier
    // of 0 (or below 2^-20) 2^-20, so that the base-2 buckets around 0 reach
    // 2^11 before they are capped
    d = lam_in[k] > 0x1p-20 ? ldexp(1.0, ilogb(lam_in[k]) - 10) : 0x1p-20;
  }
  s.delta = d;
  s.fab = xs_zero();
  s.result = lam_in[k];
  s.klo = 0;
  s.khi = ~0ull;
  s.hull_lo = ~0ull;
  s.hull_hi = 0;
  s.wlo = 0.0;
  s.whi = 0.0;
  s.hw = 0.0;
  s.corr = xs_zero();
  s.eoff = 0;
  s.ecap = 0;
  s.pad2 = 0;
  if (interp) s.flags = KS_FLAG_INTERP;
  else if (window && hinted && s.mode == KS_EXP) choose_window(s, delta_hint[K + k], prev, drift);
  st[k] = s;
}

__device__ __forceinline__ int bits_needed(uint64_t x) { return x ? 64 - __clzll((long long)x) : 0; }

// Full search of the next pass: exponential buckets over every breakpoint.
__device__ __forceinline__ void restart_full(KState &s) {
  s.mode = KS_EXP;
  s.flags = 0;
  s.n_emit = 0;
  s.overflow = 0;
  s.fab = xs_zero();
  s.klo = 0;
  s.khi = ~0ull;
  s.hull_lo = ~0ull;
  s.hull_hi = 0;
}

__device__ __forceinline__ void set_refine(KState &s, uint64_t lo, uint64_t hi) {
  s.klo = lo;
  s.khi = hi;
  const int nb = bits_needed(hi - lo);
  s.shift = nb > 6 ? nb - 6 : 0;   // (hi - lo) >> shift < 64
  s.mode = KS_REFINE;
}

// After a pass: pick the bin holding the threshold and choose the next step.
__global__ void k_scd_locate(KState *st, int K, const double *B, const double *R, const int *rinst,
                             XSum *hist_sum, uint32_t *hist_cnt, uint32_t emit_cap, unsigned int *win) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  KState s = st[k];
  if (s.ecap) emit_cap = s.ecap;   // batched: this knapsack's own buffer
  const double Bk = B[k];
  const XSum *hsum = hist_sum + (size_t)k * KP_NB;
  const uint32_t *hcnt = hist_cnt + (size_t)k * KP_NB;
  // sums and comparisons with B_k are exact (XSum): the bin that holds the
  // threshold does not depend on the order of any addition
  if (s.mode == KS_EXP) {
    XSum total = xs_zero();
    for (int b = 0; b < KP_NB; ++b) total = xs_plus(total, hsum[b]);
    if (!xs_gt(total, Bk)) {
      s.mode = KS_DONE;
      s.result = 0.0;
    } else {
      XSum cum = xs_zero();
      int bin = 1;
      for (int b = KP_NB - 1; b >= 1; --b) {
        if (hcnt[b] && xs_gt(xs_plus(cum, hsum[b]), Bk)) { bin = b; break; }
        cum = xs_plus(cum, hsum[b]);
      }
      s.bstar = bin - 32;
      s.fab = cum;
      if (s.flags & KS_FLAG_INTERP) {
        // Sec. 5.2's approximate reduce: the bucket's increments spread
        // linearly over its interval [lo, hi] (lo clamped at 0)
        const int id = bin - 32;
        const double c = s.center, d = s.delta;
        double lo, hi;
        if (id == 0) { lo = c - d; hi = c + d; }
        else if (id > 0) { lo = c + ldexp(d, id - 1); hi = c + ldexp(d, id); }
        else { lo = c - ldexp(d, -id); hi = c - ldexp(d, -id - 1); }
        lo = fmax(lo, 0.0);
        const double frac = (Bk - xs_to_double(cum)) / xs_to_double(hsum[bin]);
        const double width = hi - lo;
        const double prod = frac * width;
        const double v = hi - prod;
        s.mode = KS_DONE;
        s.result = fmax(v, lo);
        st[k] = s;
        for (int b = 0; b < KP_NB; ++b) { hist_sum[(size_t)k * KP_NB + b] = xs_zero(); hist_cnt[(size_t)k * KP_NB + b] = 0u; }
        return;
      }
      const bool central = s.bstar >= -KP_CENTRAL_W && s.bstar <= KP_CENTRAL_W;
      if (central && !s.overflow) {
        s.mode = KS_SELECT_BUCKET;
      } else {
        s.mode = hcnt[bin] <= emit_cap / 2 ? KS_EMIT_BUCKET : KS_HULL_BUCKET;
        s.n_emit = 0;
        s.overflow = 0;
        s.hull_lo = ~0ull;
        s.hull_hi = 0;
      }
    }
  } else if (s.mode == KS_EMIT_BUCKET || s.mode == KS_HULL_BUCKET) {
    if (s.mode == KS_EMIT_BUCKET && !s.overflow) {
      s.mode = KS_SELECT_BUCKET;
    } else {
      set_refine(s, s.hull_lo, s.hull_hi);
    }
  } else if (s.mode == KS_REFINE) {
    XSum cum = s.fab;
    int bin = -1;
    for (int b = KP_NB - 1; b >= 0; --b) {
      if (hcnt[b] && xs_gt(xs_plus(cum, hsum[b]), Bk)) { bin = b; break; }
      cum = xs_plus(cum, hsum[b]);
    }
    if (bin < 0) {  // cannot happen with exact sums; fall back to the lowest bin
      bin = 0;
      cum = s.fab;
      for (int b = KP_NB - 1; b >= 1; --b) cum = xs_plus(cum, hsum[b]);
    }
    s.fab = cum;
    const uint64_t lo = s.klo + ((uint64_t)bin << s.shift);
    const uint64_t hi0 = lo + ((((uint64_t)1) << s.shift) - 1);
    const uint64_t hi = hi0 < s.khi ? hi0 : s.khi;
    if (lo == hi) {
      s.mode = KS_DONE;
      s.result = kdbl(lo);
    } else if (hcnt[bin] <= emit_cap / 2) {
      s.klo = lo;
      s.khi = hi;
      s.mode = KS_EMIT_RANGE;
      s.n_emit = 0;
      s.overflow = 0;
    } else {
      set_refine(s, lo, hi);
    }
  } else if (s.mode == KS_EMIT_RANGE) {
    if (!s.overflow) s.mode = KS_SELECT_RANGE;
    else set_refine(s, s.klo, s.khi);
  } else if (s.mode == KS_WINDOW) {
    // consumption just above the window, summed over users
    // consumption of knapsack k (batched: R of instance rinst[k] sits after
    // the R, g, P columns of the instances before it)
    const double Rk = rinst ? R[k + 2 * rinst[k]] : R[k];
    const XSum above = xs_plus(xs_of(Rk), s.corr);
    if (win) { atomicAdd(&win[0], 1u); atomicAdd(&win[3], s.n_emit); }
    if (s.overflow || xs_gt(above, Bk)) {
      if (win) atomicAdd(&win[1], 1u);
      restart_full(s);                  // the threshold lies above the window
    } else {
      s.mode = KS_SELECT_RANGE;         // [klo, khi] is the window
      s.fab = above;
      s.flags |= KS_FLAG_WINDOW;
    }
  }
  st[k] = s;
  for (int b = 0; b < KP_NB; ++b) { hist_sum[(size_t)k * KP_NB + b] = xs_zero(); hist_cnt[(size_t)k * KP_NB + b] = 0u; }
}

// Exact threshold among the emitted events of one knapsack (one block per k):
// narrow the key range with LDS histograms until at most KP_SORT_MAX events
// remain, sort them (bitonic, descending), scan the increments and return the
// first distinct breakpoint whose cumulative increment exceeds B_k.
#define SEL_NT 1024
__global__ void __launch_bounds__(SEL_NT) k_scd_select(KState *st, const double *B,
                                                       const double *emit_v1, const double *emit_v2,
                                                       uint32_t emit_cap, unsigned int *win) {
  const int k = blockIdx.x;
  __shared__ KState s;
  __shared__ XSum hsum[256];
  __shared__ uint32_t hcnt[256];
  __shared__ uint64_t skey[KP_SORT_MAX];
  __shared__ double sval[KP_SORT_MAX];
  __shared__ uint64_t lo, hi;
  __shared__ XSum Fab;
  __shared__ uint32_t nsel;
  __shared__ int done;
  __shared__ double result;
  const int tid = threadIdx.x;
  if (tid == 0) s = st[k];
  __syncthreads();
  if (s.mode != KS_SELECT_BUCKET && s.mode != KS_SELECT_RANGE) return;
  const size_t eo = s.ecap ? (size_t)s.eoff : (size_t)k * emit_cap;
  if (s.ecap) emit_cap = s.ecap;
  const uint32_t n = s.n_emit < emit_cap ? s.n_emit : emit_cap;
  const double *V1 = emit_v1 + eo;
  const double *V2 = emit_v2 + eo;
  const bool bucket = s.mode == KS_SELECT_BUCKET;
  const double Bk = B[k];
  if (tid == 0) {
    lo = bucket ? 0ull : s.klo;
    hi = bucket ? ~0ull : s.khi;
    Fab = s.fab;
    done = 0;
  }
  __syncthreads();
  if (s.flags & KS_FLAG_WINDOW) {
    // the threshold lies in the window iff the window's increments take the
    // running sum past B_k
    __shared__ XSum part[SEL_NT / 64];
    XSum v = xs_zero();
    for (uint32_t e = tid; e < n; e += SEL_NT) xs_add(v, V2[e]);
    for (int off = 32; off > 0; off >>= 1) {
      v.hi = v.hi + __shfl_xor(v.hi, off, 64);
      v.lo = v.lo + __shfl_xor(v.lo, off, 64);
    }
    if ((tid & 63) == 0) part[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      XSum tot = Fab;
      for (int w = 0; w < SEL_NT / 64; ++w) tot = xs_plus(tot, part[w]);
      if (!xs_gt(tot, Bk)) {
        if (s.wlo == 0.0) {             // every breakpoint is in the window
          st[k].result = 0.0;
          st[k].mode = KS_DONE;
        } else {
          KState r = s;                 // below the window: full search
          restart_full(r);
          st[k] = r;
          if (win) atomicAdd(&win[2], 1u);
        }
        done = 2;
      }
    }
    __syncthreads();
    if (done == 2) return;
  }
  // narrowing loop
  for (int it = 0; it < 80; ++it) {
    if (tid == 0) nsel = 0;
    if (tid < 256) { hsum[tid] = xs_zero(); hcnt[tid] = 0u; }
    __syncthreads();
    const uint64_t L0 = lo, H0 = hi;
    for (uint32_t e = tid; e < n; e += SEL_NT) {
      const double v = V1[e];
      if (bucket && exp_bucket(v, s.center, s.delta) != s.bstar) continue;
      const uint64_t key = dkey(v);
      if (key < L0 || key > H0) continue;
      atomicAdd(&nsel, 1u);
    }
    __syncthreads();
    if (nsel <= KP_SORT_MAX) break;
    const int nb = bits_needed(H0 - L0);
    const int shift = nb > 8 ? nb - 8 : 0;
    for (uint32_t e = tid; e < n; e += SEL_NT) {
      const double v = V1[e];
      if (bucket && exp_bucket(v, s.center, s.delta) != s.bstar) continue;
      const uint64_t key = dkey(v);
      if (key < L0 || key > H0) continue;
      const int bin = (int)((key - L0) >> shift);
      xs_atomic_add(&hsum[bin], V2[e]);
      atomicAdd(&hcnt[bin], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      XSum cum = Fab;
      int bin = -1;
      for (int b = 255; b >= 0; --b) {
        if (hcnt[b] && xs_gt(xs_plus(cum, hsum[b]), Bk)) { bin = b; break; }
        cum = xs_plus(cum, hsum[b]);
      }
      if (bin < 0) { bin = 0; }
      Fab = cum;
      const uint64_t nlo = L0 + ((uint64_t)bin << shift);
      const uint64_t nhi0 = nlo + ((((uint64_t)1) << shift) - 1);
      lo = nlo;
      hi = nhi0 < H0 ? nhi0 : H0;
      if (lo == hi) { done = 1; result = kdbl(lo); }
    }
    __syncthreads();
    if (done) break;
  }
  if (!done) {
    // gather the surviving events
    if (tid == 0) nsel = 0;
    __syncthreads();
    const uint64_t L0 = lo, H0 = hi;
    for (uint32_t e = tid; e < n; e += SEL_NT) {
      const double v = V1[e];
      if (bucket && exp_bucket(v, s.center, s.delta) != s.bstar) continue;
      const uint64_t key = dkey(v);
      if (key < L0 || key > H0) continue;
      const uint32_t slot = atomicAdd(&nsel, 1u);
      if (slot < KP_SORT_MAX) { skey[slot] = key; sval[slot] = V2[e]; }
    }
    __syncthreads();
    const uint32_t m = nsel < KP_SORT_MAX ? nsel : KP_SORT_MAX;
    int P2 = 1;
    while (P2 < (int)m) P2 <<= 1;
    for (int t = m + tid; t < P2; t += SEL_NT) { skey[t] = 0ull; sval[t] = 0.0; }
    __syncthreads();
    // bitonic sort, descending by key (ties: any order -- equal keys are grouped)
    for (int size = 2; size <= P2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int t = tid; t < P2; t += SEL_NT) {
          const int pt2 = t ^ stride;
          if (pt2 > t) {
            const bool desc = ((t & size) == 0);
            const uint64_t ka = skey[t], kb = skey[pt2];
            if (desc ? (ka < kb) : (ka > kb)) {
              skey[t] = kb; skey[pt2] = ka;
              const double va = sval[t]; sval[t] = sval[pt2]; sval[pt2] = va;
            }
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      XSum cum = Fab;
      double ans = m ? kdbl(skey[m - 1]) : kdbl(lo);
      uint32_t e = 0;
      while (e < m) {
        const uint64_t key = skey[e];
        while (e < m && skey[e] == key) { xs_add(cum, sval[e]); ++e; }
        if (xs_gt(cum, Bk)) { ans = kdbl(key); break; }
      }
      result = ans;
    }
    __syncthreads();
  }
  if (tid == 0) {
    st[k].result = result;
    st[k].mode = KS_DONE;
  }
}

__global__ void k_scd_finish(const KState *st, int K, const double *lam_in, double *lam_out,
                             double *delta_next, int *pending) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double nl = st[k].result;
  lam_out[k] = nl;
  if (delta_next) {
    // next search: the bucket width, a power of two above this step, and the
    // step itself (bounded below) for the window
    const double step = fabs(nl - lam_in[k]);
    const double floor_ = (nl > 0x1p-20 ? nl : 0x1p-20) * 0x1p-30;
    const double w = step > floor_ ? step : floor_;
    delta_next[k] = ldexp(1.0, ilogb(w) + 1);
    delta_next[K + k] = w;
  }
}

// A full search (no window) centres its buckets on the threshold of a
// sample of users (lam_hat, from the same search on the sample with its
// budgets scaled): buckets of half-width 2^-8 of it around it, so the central
// buckets emitted by the first pass usually hold the threshold.  With
// windows enabled, and lambda_k^t within a quarter of lam_hat, the search
// starts instead with a window over those central buckets (4 bucket widths
// either side of lam_hat): the walks stop below the window and nothing is
// binned (c3 cold iterations 95 -> 45-55 ms); from further away (a start
// from lambda = 0) the window pass costs more than the buckets.  A miss
// falls back to the full search around lam_hat.  Exactness does not depend
// on either (the threshold is located by exact sums over all users).
__global__ void k_scd_recenter(KState *st, int K, const double *lam_hat, const double *lam_in, int window) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double c = lam_hat[k];
  if (st[k].mode != KS_EXP || !(c > 0x1p-20)) return;
  KState s = st[k];
  s.center = c;
  s.delta = ldexp(1.0, ilogb(c) - 8);
  if (window && fabs(lam_in[k] - c) <= 0.25 * c) {
    const double h = 4.0 * s.delta;
    s.mode = KS_WINDOW;
    s.whi = c + h;
    s.wlo = c - h > 0.0 ? c - h : 0.0;
    s.klo = dkey(s.wlo);
    s.khi = dkey(s.whi);
    const double l = lam_in[k];
    s.hw = fmax(fabs(s.whi - l), fabs(l - s.wlo));
  }
  st[k] = s;
}

// users[s] = s * stride + off (a strided sample)
__global__ void k_strided_users(int64_t *users, int64_t n, int64_t stride, int64_t off) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x)
    users[s] = s * stride + off;
}

// rowptr of a sample whose rows all hold D entries: r * D
__global__ void k_uniform_rowptr(int64_t *rowptr, int64_t nrows, int D) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= nrows; r += (int64_t)gridDim.x * blockDim.x)
    rowptr[r] = r * D;
}

// Knapsacks starting with a window and those needing another search mode.
// out[0]: knapsacks searching with a window, out[1]: with another search
// mode, out[2]: windows that do not contain lambda_k^t (alternation windows);
// out[3] is cleared (the dense window pass's probe counts into it)
__global__ void k_count_modes(const KState *st, int K, int *out) {
  __shared__ int c[3];
  if (threadIdx.x < 3) c[threadIdx.x] = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const KState &s = st[k];
    if (s.mode == KS_WINDOW) {
      atomicAdd(&c[0], 1);
      const double cen = 0.5 * (s.wlo + s.whi);
      if (!(fabs(cen - s.center) <= fmax(s.whi - cen, cen - s.wlo))) atomicAdd(&c[2], 1);
    } else if (s.mode != KS_DONE) {
      atomicAdd(&c[1], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) out[threadIdx.x] = c[threadIdx.x];
  if (threadIdx.x == 3) out[3] = 0;
}

__global__ void k_count_pending(const KState *st, int K, int *pending) {
  __shared__ int c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    if (st[k].mode != KS_DONE) atomicAdd(&c, 1);
  __syncthreads();
  if (threadIdx.x == 0) *pending = c;
}

// ---------------------------------------------------------------------------
// Pre-solving by sampling (Sec. 5.3): the sub-instance of the sampled users
// ---------------------------------------------------------------------------
// dst[s * rowlen + c] = src[users[s] * rowlen + c]
__global__ void k_gather_rows(const float *src, float *dst, const int64_t *users, int64_t n,
                              int64_t rowlen) {
  const int64_t total = n * rowlen;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / rowlen, c = e - s * rowlen;
    dst[e] = src[users[s] * rowlen + c];
  }
}

// stored entries of every sampled item row
__global__ void k_gather_len(const int64_t *rowptr, const int64_t *users, int64_t n, int M,
                             int64_t *len) {
  const int64_t total = n * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / M, j = e - s * M;
    const int64_t r = users[s] * M + j;
    len[e] = rowptr[r + 1] - rowptr[r];
  }
}

// out[0] = 0, out[i + 1] = len[0] + ... + len[i]  (one block; chunk per thread,
// then a scan of the chunk sums in LDS)
__global__ void __launch_bounds__(1024) k_scan_i64(const int64_t *len, int64_t *out, int64_t n) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = t * chunk < n ? t * chunk : n;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  int64_t sum = 0;
  for (int64_t i = lo; i < hi; ++i) sum += len[i];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;
  if (t == 0) out[0] = 0;
  for (int64_t i = lo; i < hi; ++i) { run += len[i]; out[i + 1] = run; }
}

// copy the sampled item rows' entries (rows are short: one thread per row)
__global__ void k_gather_csr(const int64_t *rowptr, const int32_t *col, const float *val,
                             const int64_t *users, int64_t n, int M, const int64_t *subptr,
                             int32_t *scol, float *sval) {
  const int64_t total = n * M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / M, j = e - s * M;
    const int64_t r = users[s] * M + j;
    int64_t o = subptr[e];
    for (int64_t q = rowptr[r]; q < rowptr[r + 1]; ++q, ++o) {
      scol[o] = col[q];
      sval[o] = val[q];
    }
  }
}

// ---------------------------------------------------------------------------
// DD step (Eq.14) and the dual gradient
// ---------------------------------------------------------------------------
__global__ void k_dd_update(int K, double alpha, const double *R, const double *B, double *lam) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double d = R[k] - B[k];
  const double stp = alpha * d;
  const double nl = lam[k] + stp;
  lam[k] = nl > 0.0 ? nl : 0.0;
}

__global__ void k_dual_backward(int K, const double *R, const double *B, const double *gout,
                                double *glam) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double d = B[k] - R[k];
  glam[k] = gout[0] * d;
}

// ---------------------------------------------------------------------------
// input validation pass
// ---------------------------------------------------------------------------
__global__ void k_validate(const float *v, int64_t n, unsigned int *flags) {
  // flags[0]: non-finite seen, flags[1]: negative seen
  unsigned int nf = 0, ng = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const float x = v[t];
    nf |= !isfinite(x);
    ng |= (x < 0.0f);
  }
  if (nf) atomicOr(&flags[0], 1u);
  if (ng) atomicOr(&flags[1], 1u);
}

__global__ void k_validate_csr(const int64_t *rowptr, const int32_t *col, int64_t nrows, int K,
                               unsigned int *flags) {
  unsigned int bad = 0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e0 = rowptr[r], e1 = rowptr[r + 1];
    if (e1 < e0) { bad = 1; continue; }
    int prev = -1;
    for (int64_t e = e0; e < e1; ++e) {
      const int c = col[e];
      if (c <= prev || c >= K) bad = 1;
      prev = c;
    }
  }
  if (bad) atomicOr(&flags[2], 1u);
}

// ---------------------------------------------------------------------------
// post-processing for feasibility (Sec. 5.4): the candidates (users whose
// solution consumes a violated knapsack) are taken in (G_i asc, i asc) order
// and the shortest prefix whose reset covers every violated knapsack is
// reset.  No candidate list is sorted whole: splitters drawn from a strided
// sample of the candidates' G values cut the key range into nb bins; one pass
// over the users adds every candidate's costs on the violated knapsacks into
// per-bin exact sums; the bin in which the last knapsack becomes covered is
// found from the bins' prefix sums; only that bin's users are sorted (stable
// LSD radix sort of G's bits over a list compacted in user order) and
// scanned; then the users of the earlier bins and the scanned prefix are
// reset.  Coverage compares exact sums (two-limb fixed point) with B_k:
// the consumption a reset leaves is a real sum, so the reset set does not
// depend on any summation order.
// ---------------------------------------------------------------------------
#define FX_NT 256
#define FX_IPT 16                       // items per thread in the sort / scan kernels
#define FX_CHUNK (FX_NT * FX_IPT)
#define FX_NONE 0xFFu                   // bin byte of a user that is not a candidate
#define FX_LDS_MAX (48 * 1024)          // per-block accumulators above this live in global memory

struct FixState {
  int bstar;          // bin in which the last violated knapsack is covered (-1: none violated)
  uint32_t nbefore;   // candidates in the bins before it
  uint32_t nstar;     // candidates in it
  uint32_t tstar;     // users of its sorted list that are reset
};

struct FixArgs {
  ProbDev pr;
  uint8_t *x;             // [N*M] selection at lambda; the reset clears rows
  const double *lam;      // [K]
  const int *kv;          // [K] slot of a violated knapsack, or -1
  const int *vk;          // [nv] knapsack of each slot
  const double *Bv;       // [nv] their budgets
  int nv, nb;
  int d;                  // CSR: entries in every row (row r's start at r * d), or 0
  const uint64_t *split;  // [nb - 1] ascending splitter keys
  uint8_t *bin;           // [N] bin of every user (FX_NONE: not a candidate)
  XSum *hsum;             // [nb][nv] exact consumption per bin
  uint32_t *hcnt;         // [nb] candidates per bin
  FixState *fs;
  XSum *cthr;             // [nv] consumption of the bins before the one covering the slot
  int *vb;                // [nv] bin covering the slot (-1: covered with no reset)
  XSum *rem;              // [K + 1] removed consumption and profit
};

// exclusive scan of n counts in one block (n up to a few million; sequential
// chunks per thread, then a block scan of the chunk totals)
__global__ void __launch_bounds__(1024) k_scan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                                                   uint32_t *total) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b0 = t * per, b1 = (b0 + per < n) ? b0 + per : n;
  uint64_t s = 0;
  for (int64_t i = b0; i < b1; ++i) s += in[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    uint64_t run = 0;
    for (int i = 0; i < 1024; ++i) { const uint64_t v = part[i]; part[i] = run; run += v; }
    if (total) *total = (uint32_t)run;
  }
  __syncthreads();
  uint64_t run = part[t];
  for (int64_t i = b0; i < b1; ++i) { const uint32_t v = in[i]; out[i] = (uint32_t)run; run += v; }
}

// one 4-bit digit of a stable LSD radix sort: per-block digit counts
__global__ void __launch_bounds__(FX_NT) k_rs_hist(const uint64_t *key, uint32_t n, int shift,
                                                   uint32_t *hist, uint32_t nblk) {
  __shared__ uint32_t h[16];
  if (threadIdx.x < 16) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t base = blockIdx.x * FX_CHUNK;
  for (int t = 0; t < FX_IPT; ++t) {
    const uint32_t i = base + threadIdx.x * FX_IPT + t;
    if (i >= n) break;
    atomicAdd(&h[(key[i] >> shift) & 15], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 16) hist[(size_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// stable scatter: each thread owns FX_IPT consecutive items; ranks come from
// per-thread digit counts scanned across the block in thread order
__global__ void __launch_bounds__(FX_NT) k_rs_scatter(const uint64_t *key, const uint32_t *val,
                                                      uint32_t n, int shift, const uint32_t *hoff,
                                                      uint32_t nblk, uint64_t *okey,
                                                      uint32_t *oval) {
  __shared__ uint32_t cnt[16][FX_NT + 1];
  const int t = threadIdx.x;
  const uint32_t base = blockIdx.x * FX_CHUNK + t * FX_IPT;
  uint32_t c[16];
  for (int d = 0; d < 16; ++d) c[d] = 0;
  for (int q = 0; q < FX_IPT; ++q) {
    const uint32_t i = base + q;
    if (i >= n) break;
    c[(key[i] >> shift) & 15]++;
  }
  for (int d = 0; d < 16; ++d) cnt[d][t] = c[d];
  __syncthreads();
  if (t < 16) {
    uint32_t run = hoff[(size_t)t * nblk + blockIdx.x];
    for (int q = 0; q < FX_NT; ++q) { const uint32_t v = cnt[t][q]; cnt[t][q] = run; run += v; }
  }
  __syncthreads();
  for (int d = 0; d < 16; ++d) c[d] = cnt[d][t];
  for (int q = 0; q < FX_IPT; ++q) {
    const uint32_t i = base + q;
    if (i >= n) break;
    const uint64_t kk = key[i];
    const int d = (int)((kk >> shift) & 15);
    const uint32_t dst = c[d]++;
    okey[dst] = kk;
    oval[dst] = val[i];
  }
}

// the cost entries (k, b) of item row r in storage order (d > 0: every CSR
// row holds d entries)
template <class F>
__device__ __forceinline__ void fx_row(const ProbDev &pr, int d, int64_t r, F f) {
  if (pr.fmt == 0) {   // dense rows
    const float *bb = pr.b + r * pr.K;
    for (int k = 0; k < pr.K; ++k) f(k, bb[k]);
  } else if (d > 0) {
    const int64_t e0 = r * d;
    for (int t = 0; t < d; ++t) f((int)pr.col[e0 + t], pr.val[e0 + t]);
  } else {
    const int64_t e1 = pr.rowptr[r + 1];
    for (int64_t e = pr.rowptr[r]; e < e1; ++e) f((int)pr.col[e], pr.val[e]);
  }
}

// G_i, the sum of p~ over the selected items in ascending index order (p~ as
// the sweep forms it: the stored costs in order, a product then a
// subtraction), and whether user i consumes a violated knapsack
__device__ __forceinline__ bool fx_user(const FixArgs &f, int64_t i, double &G) {
  const int M = f.pr.M, K = f.pr.K;
  bool cand = false;
  double g = 0.0;
  for (int j = 0; j < M; ++j) {
    const int64_t r = i * M + j;
    if (!f.x[r]) continue;
    double acc = (double)f.pr.p[r];
    fx_row(f.pr, f.d, r, [&](int k, float c) {
      if ((unsigned)k >= (unsigned)K) return;
      const double prod = f.lam[k] * (double)c;
      acc = acc - prod;
      cand = cand || (c > 0.0f && f.kv[k] >= 0);
    });
    g = g + acc;
  }
  G = g;
  return cand;
}

// exact consumption of knapsack k by user i's selection
__device__ __forceinline__ XSum fx_use(const FixArgs &f, int64_t i, int k) {
  XSum s = xs_zero();
  for (int j = 0; j < f.pr.M; ++j) {
    const int64_t r = i * f.pr.M + j;
    if (!f.x[r]) continue;
    fx_row(f.pr, f.d, r, [&](int kk, float c) {
      if (kk == k) s = xs_plus(s, xs_of((double)c));
    });
  }
  return s;
}

// sampled users i = s * stride that are candidates: their keys
__global__ void __launch_bounds__(FX_NT) k_fix_sample(FixArgs f, int64_t stride, uint32_t ns,
                                                      uint64_t *keys, uint32_t *idx, uint32_t *count) {
  const uint32_t s = blockIdx.x * FX_NT + threadIdx.x;
  if (s >= ns) return;
  double G;
  if (!fx_user(f, (int64_t)s * stride, G)) return;
  const uint32_t slot = atomicAdd(count, 1u);
  keys[slot] = dkey(G + 0.0);
  idx[slot] = slot;
}

// splitters at the sample's quantiles q / nb (all keys in bin 0 when the
// sample holds no candidate)
__global__ void k_fix_split(const uint64_t *sorted, const uint32_t *count, int nb, uint64_t *split) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb - 1) return;
  const uint32_t n = *count;
  split[q] = n ? sorted[((uint64_t)(q + 1) * n) / nb] : ~0ull;
}

// every user: bin byte, per-bin candidate counts and exact consumption of the
// violated knapsacks (block accumulators in LDS when they fit, added to the
// global ones at the end; the grid strides over 4096-user chunks)
__global__ void __launch_bounds__(FX_NT) k_fix_bins(FixArgs f, int lds) {
  extern __shared__ __align__(16) unsigned char fsm[];
  const int nb = f.nb, nv = f.nv, K = f.pr.K, M = f.pr.M;
  XSum *hs = lds ? (XSum *)fsm : f.hsum;
  uint32_t *hc = lds ? (uint32_t *)(fsm + (size_t)nb * nv * sizeof(XSum)) : f.hcnt;
  uint64_t *sp = (uint64_t *)(fsm + (lds ? (size_t)nb * nv * sizeof(XSum) + (size_t)nb * 4 + 8 : 0));
  if (lds) {
    for (int t = threadIdx.x; t < nb * nv; t += FX_NT) hs[t] = xs_zero();
    for (int t = threadIdx.x; t < nb; t += FX_NT) hc[t] = 0u;
  }
  for (int t = threadIdx.x; t < nb - 1; t += FX_NT) sp[t] = f.split[t];
  __syncthreads();
  const int64_t N = f.pr.N;
  const int64_t nch = (N + FX_CHUNK - 1) / FX_CHUNK;
  for (int64_t ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    for (int q = 0; q < FX_IPT; ++q) {
      const int64_t i = ch * FX_CHUNK + (int64_t)q * FX_NT + threadIdx.x;
      if (i >= N) break;
      double G;
      uint8_t bb = (uint8_t)FX_NONE;
      if (fx_user(f, i, G)) {
        const int b = fx_bin_of(sp, nb, dkey(G + 0.0));
        bb = (uint8_t)b;
        atomicAdd(&hc[b], 1u);
        XSum *row = hs + (size_t)b * nv;
        for (int j = 0; j < M; ++j) {
          const int64_t r = i * M + j;
          if (!f.x[r]) continue;
          fx_row(f.pr, f.d, r, [&](int k, float c) {
            if ((unsigned)k >= (unsigned)K || !(c > 0.0f)) return;
            const int v = f.kv[k];
            if (v >= 0) xs_atomic_add(&row[v], (double)c);
          });
        }
      }
      f.bin[i] = bb;
    }
  }
  if (!lds) return;
  __syncthreads();
  for (int t = threadIdx.x; t < nb * nv; t += FX_NT)
    if (xs_nonzero(hs[t])) xs_atomic_add_sum(&f.hsum[t], hs[t]);
  for (int t = threadIdx.x; t < nb; t += FX_NT)
    if (hc[t]) atomicAdd(&f.hcnt[t], hc[t]);
}

// per violated knapsack: the first bin whose prefix covers it, exactly
// (covered: total - removed <= B); the threshold bin is the largest
__global__ void __launch_bounds__(256) k_fix_locate(FixArgs f) {
  __shared__ int bst;
  if (threadIdx.x == 0) bst = -1;
  __syncthreads();
  for (int v = threadIdx.x; v < f.nv; v += 256) {
    XSum T = xs_zero();
    for (int b = 0; b < f.nb; ++b) T = xs_plus(T, f.hsum[(size_t)b * f.nv + v]);
    const double Bk = f.Bv[v];
    int vb = -1;
    XSum S = xs_zero();
    if (xs_gt(T, Bk)) {
      vb = f.nb - 1;
      for (int b = 0; b < f.nb; ++b) {
        const XSum S2 = xs_plus(S, f.hsum[(size_t)b * f.nv + v]);
        if (!xs_gt(xs_minus(T, S2), Bk)) { vb = b; break; }
        S = S2;
      }
    }
    f.vb[v] = vb;
    f.cthr[v] = S;
    atomicMax(&bst, vb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t before = 0;
    for (int b = 0; b < bst; ++b) before += f.hcnt[b];
    f.fs->bstar = bst;
    f.fs->nbefore = before;
    f.fs->nstar = bst >= 0 ? f.hcnt[bst] : 0u;
    f.fs->tstar = 0u;
  }
}

// the bin bytes of FX_IPT consecutive users from user i0 on (fewer at the end)
__device__ __forceinline__ void fx_bins16(const uint8_t *bin, int64_t i0, int64_t N, uint8_t out[FX_IPT]) {
  if (i0 + FX_IPT <= N) {
    const uint4 w = *(const uint4 *)(bin + i0);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    for (int q = 0; q < FX_IPT; ++q) out[q] = (uint8_t)(ws[q >> 2] >> (8 * (q & 3)));
  } else {
    for (int q = 0; q < FX_IPT; ++q) out[q] = i0 + q < N ? bin[i0 + q] : (uint8_t)FX_NONE;
  }
}

// users of the threshold bin per chunk
__global__ void __launch_bounds__(FX_NT) k_fix_bcount(FixArgs f, uint32_t *bcnt) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  const int bst = f.fs->bstar;
  uint8_t bb[FX_IPT];
  fx_bins16(f.bin, (int64_t)blockIdx.x * FX_CHUNK + (int64_t)threadIdx.x * FX_IPT, f.pr.N, bb);
  uint32_t mine = 0;
  for (int q = 0; q < FX_IPT; ++q) mine += (int)bb[q] == bst;
  atomicAdd(&c, mine);
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = c;
}

// stable compaction of the threshold bin's users in user order, with keys
__global__ void __launch_bounds__(FX_NT) k_fix_collect(FixArgs f, const uint32_t *boff, uint64_t *ckey,
                                                       uint32_t *cidx) {
  __shared__ uint32_t tcnt[FX_NT];
  const int bst = f.fs->bstar;
  const int64_t i0 = (int64_t)blockIdx.x * FX_CHUNK + (int64_t)threadIdx.x * FX_IPT;
  uint8_t bb[FX_IPT];
  fx_bins16(f.bin, i0, f.pr.N, bb);
  uint32_t mine = 0;
  for (int q = 0; q < FX_IPT; ++q) mine += (int)bb[q] == bst;
  tcnt[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int t = 0; t < FX_NT; ++t) { const uint32_t v = tcnt[t]; tcnt[t] = run; run += v; }
  }
  __syncthreads();
  uint32_t pos = boff[blockIdx.x] + tcnt[threadIdx.x];
  for (int q = 0; q < FX_IPT; ++q) {
    if ((int)bb[q] != bst) continue;
    double G;
    fx_user(f, i0 + q, G);
    ckey[pos] = dkey(G + 0.0);
    cidx[pos] = (uint32_t)(i0 + q);
    ++pos;
  }
}

// per chunk of the sorted threshold-bin list: exact consumption of every
// slot covered inside that bin
__global__ void __launch_bounds__(FX_NT) k_fix_chunk(FixArgs f, const uint32_t *sidx, XSum *csum, int lds) {
  extern __shared__ __align__(16) unsigned char fsm[];
  const int nv = f.nv, K = f.pr.K, M = f.pr.M;
  XSum *cs = lds ? (XSum *)fsm : csum + (size_t)blockIdx.x * nv;
  if (lds)
    for (int t = threadIdx.x; t < nv; t += FX_NT) cs[t] = xs_zero();
  __syncthreads();
  const int bst = f.fs->bstar;
  const uint32_t n = f.fs->nstar;
  for (int q = 0; q < FX_IPT; ++q) {
    const uint32_t e = blockIdx.x * FX_CHUNK + q * FX_NT + threadIdx.x;
    if (e >= n) break;
    const int64_t i = sidx[e];
    for (int j = 0; j < M; ++j) {
      const int64_t r = i * M + j;
      if (!f.x[r]) continue;
      fx_row(f.pr, f.d, r, [&](int k, float c) {
        if ((unsigned)k >= (unsigned)K || !(c > 0.0f)) return;
        const int v = f.kv[k];
        if (v >= 0 && f.vb[v] == bst) xs_atomic_add(&cs[v], (double)c);
      });
    }
  }
  if (!lds) return;
  __syncthreads();
  for (int t = threadIdx.x; t < nv; t += FX_NT) csum[(size_t)blockIdx.x * nv + t] = cs[t];
}

// one block per slot covered in the threshold bin: the shortest prefix of the
// sorted list that covers it; tstar is the largest over the slots
__global__ void __launch_bounds__(FX_NT) k_fix_prefix(FixArgs f, const uint32_t *sidx, const XSum *csum,
                                                      uint32_t nchunks) {
  const int v = blockIdx.x;
  const int bst = f.fs->bstar;
  if (bst < 0 || f.vb[v] != bst) return;
  const uint32_t n = f.fs->nstar;
  const int k = f.vk[v];
  const double Bk = f.Bv[v];
  __shared__ uint32_t chunk, first;
  __shared__ XSum tsum[FX_NT];
  __shared__ XSum Tsh;
  if (threadIdx.x == 0) {
    XSum T = xs_zero();
    for (int b = 0; b < f.nb; ++b) T = xs_plus(T, f.hsum[(size_t)b * f.nv + v]);
    XSum S = f.cthr[v];
    uint32_t c = nchunks - 1;
    for (uint32_t q = 0; q < nchunks; ++q) {
      const XSum S2 = xs_plus(S, csum[(size_t)q * f.nv + v]);
      if (!xs_gt(xs_minus(T, S2), Bk)) { c = q; break; }
      S = S2;
    }
    chunk = c;
    first = 0xFFFFFFFFu;
    Tsh = T;
    tsum[0] = S;   // consumption before the chunk (the scan below adds the rest)
  }
  __syncthreads();
  const XSum before = tsum[0];
  __syncthreads();
  const uint32_t e0 = chunk * FX_CHUNK + threadIdx.x * FX_IPT;
  XSum mine = xs_zero();
  for (int q = 0; q < FX_IPT; ++q)
    if (e0 + q < n) mine = xs_plus(mine, fx_use(f, sidx[e0 + q], k));
  tsum[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    XSum run = before;
    for (int t = 0; t < FX_NT; ++t) { const XSum w = tsum[t]; tsum[t] = run; run = xs_plus(run, w); }
  }
  __syncthreads();
  XSum S = tsum[threadIdx.x];
  for (int q = 0; q < FX_IPT; ++q) {
    const uint32_t e = e0 + q;
    if (e >= n) break;
    S = xs_plus(S, fx_use(f, sidx[e], k));
    if (!xs_gt(xs_minus(Tsh, S), Bk)) { atomicMin(&first, e); break; }
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&f.fs->tstar, first != 0xFFFFFFFFu ? first + 1 : n);
}

// clear user i's selection; its profit and consumption go to rem
__device__ __forceinline__ void fx_remove(const FixArgs &f, int64_t i, XSum *rem) {
  const int M = f.pr.M, K = f.pr.K;
  for (int j = 0; j < M; ++j) {
    const int64_t r = i * M + j;
    if (!f.x[r]) continue;
    f.x[r] = 0;
    xs_atomic_add(&rem[K], (double)f.pr.p[r]);
    fx_row(f.pr, f.d, r, [&](int k, float c) {
      if ((unsigned)k < (unsigned)K && c != 0.0f) xs_atomic_add(&rem[k], (double)c);
    });
  }
}

// reset the candidates of the bins before the threshold bin (list == null)
// or the first tstar users of the sorted list
__global__ void __launch_bounds__(FX_NT) k_fix_reset(FixArgs f, const uint32_t *sidx, int lds) {
  extern __shared__ __align__(16) unsigned char fsm[];
  const int K = f.pr.K;
  XSum *rem = lds ? (XSum *)fsm : f.rem;
  if (lds)
    for (int t = threadIdx.x; t <= K; t += FX_NT) rem[t] = xs_zero();
  __syncthreads();
  const int bst = f.fs->bstar;
  if (!sidx) {
    const int64_t N = f.pr.N;
    for (int64_t i = (int64_t)blockIdx.x * FX_NT + threadIdx.x; i < N; i += (int64_t)gridDim.x * FX_NT) {
      const int b = f.bin[i];
      if (b != (int)FX_NONE && b < bst) fx_remove(f, i, rem);
    }
  } else {
    const uint32_t ts = f.fs->tstar;
    for (uint32_t e = blockIdx.x * FX_NT + threadIdx.x; e < ts; e += gridDim.x * FX_NT) fx_remove(f, sidx[e], rem);
  }
  if (!lds) return;
  __syncthreads();
  for (int t = threadIdx.x; t <= K; t += FX_NT)
    if (xs_nonzero(rem[t])) xs_atomic_add_sum(&f.rem[t], rem[t]);
}

__global__ void k_fix_final(FixArgs f, const double *R, const double *P, double *R_out, double *P_out,
                            int64_t *n_reset) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int K = f.pr.K;
  if (c > K) return;
  const double s = xs_to_double(f.rem[c]);
  if (c < K) {
    R_out[c] = R[c] - s;
  } else {
    *P_out = *P - s;
    *n_reset = f.fs->bstar < 0 ? 0 : (int64_t)f.fs->nbefore + (int64_t)f.fs->tstar;
  }
}

// stable LSD radix sort of n (key, value) pairs, 4 bits per pass; the result
// ends in (k0, v0) (an even number of passes)
static hipError_t fx_sort(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, uint32_t n,
                          uint32_t *hist, uint32_t *hoff, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t nbs = (n + FX_CHUNK - 1) / FX_CHUNK;
  for (int shift = 0; shift < 64; shift += 4) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nbs), dim3(FX_NT), 0, stream, k0, n, shift, hist, nbs);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, stream, hist, hoff, (int64_t)16 * nbs,
                       (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nbs), dim3(FX_NT), 0, stream, k0, v0, n, shift, hoff, nbs, k1, v1);
    uint64_t *tk = k0; k0 = k1; k1 = tk;
    uint32_t *tv = v0; v0 = v1; v1 = tv;
  }
  return hipGetLastError();
}

// bins of the post-processing: the most (a power of two, at most 128) whose
// sums over nv slots fit in budget bytes
int kp_fixup_bins(int nv, size_t budget) {
  int nb = 128;
  while (nb > 1 && (size_t)nb * nv * sizeof(XSum) > budget) nb >>= 1;
  return nb;
}

namespace {
struct FxLayout {
  size_t bin, skey, tkey, sidx, tidx, scount, split, hsum, hcnt, fs, cthr, vb, rem, ckey, ckey2, cidx, cidx2,
      hist, hoff, bcnt, boff, csum, total;
};
FxLayout fx_layout(int64_t N, int nv, int K) {
  FxLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
  // the bin arrays at their largest (at most 128 bins, at most 40 KB of
  // sums or one row per slot), so that a layout never outgrows the one for
  // more slots
  const uint32_t ns = (uint32_t)(N < 65536 ? N : 65536);
  const size_t nch = (size_t)((N + FX_CHUNK - 1) / FX_CHUNK) + 1;
  L.bin = take((size_t)N + 16);
  L.skey = take((size_t)ns * 8 + 8);
  L.tkey = take((size_t)ns * 8 + 8);
  L.sidx = take((size_t)ns * 4 + 4);
  L.tidx = take((size_t)ns * 4 + 4);
  L.scount = take(8);
  L.split = take(128 * 8);
  L.hsum = take(std::max<size_t>(40 * 1024, (size_t)nv * sizeof(XSum)));
  L.hcnt = take(128 * 4);
  L.fs = take(sizeof(FixState));
  L.cthr = take((size_t)nv * sizeof(XSum));
  L.vb = take((size_t)nv * 4);
  L.rem = take((size_t)(K + 1) * sizeof(XSum));
  L.ckey = take((size_t)N * 8 + 8);
  L.ckey2 = take((size_t)N * 8 + 8);
  L.cidx = take((size_t)N * 4 + 4);
  L.cidx2 = take((size_t)N * 4 + 4);
  L.hist = take(16 * nch * 4);
  L.hoff = take(16 * nch * 4);
  L.bcnt = take(nch * 4);
  L.boff = take(nch * 4);
  L.csum = take(nch * (size_t)nv * sizeof(XSum));
  L.total = off;
  return L;
}
}  // namespace

size_t kp_fixup_scratch_bytes(int64_t N, int nv, int K) { return fx_layout(N, nv, K).total; }

// kv / vk / Bv: device arrays of the violated slots; nb: bins (at most 128,
// nb * nv sums within 40 KB); pinned: 32 bytes of pinned host memory;
// persist: blocks of the user passes; bins_pass: launches the per-user bin
// pass (k_fix_bins when empty).  Synchronizes the stream twice (the
// sample's candidate count, then the threshold bin).
hipError_t kp_launch_fixup_pipeline(ProbDev pr, int row_d, uint8_t *x, const double *lam, const int *kv,
                                    const int *vk, const double *Bv, int nv, int nb, const double *R,
                                    const double *P,
                                    double *R_out, double *P_out, int64_t *n_reset, void *scratch,
                                    hipStream_t stream, uint32_t *pinned, int persist,
                                    const std::function<hipError_t(const FixBins &)> &bins_pass) {
  const int64_t N = pr.N;
  const int K = pr.K;
  const FxLayout L = fx_layout(N, nv, K);
  char *w = (char *)scratch;
  FixArgs f;
  f.pr = pr;
  f.d = pr.fmt == 0 ? 0 : row_d;
  f.x = x;
  f.lam = lam;
  f.kv = kv;
  f.vk = vk;
  f.Bv = Bv;
  f.nv = nv;
  if (nb < 1 || nb > 128 || (nb > 1 && (size_t)nb * nv * sizeof(XSum) > 40 * 1024)) return hipErrorInvalidValue;
  f.nb = nb;
  f.split = (const uint64_t *)(w + L.split);
  f.bin = (uint8_t *)(w + L.bin);
  f.hsum = (XSum *)(w + L.hsum);
  f.hcnt = (uint32_t *)(w + L.hcnt);
  f.fs = (FixState *)(w + L.fs);
  f.cthr = (XSum *)(w + L.cthr);
  f.vb = (int *)(w + L.vb);
  f.rem = (XSum *)(w + L.rem);
  hipError_t e;
  if ((e = hipMemsetAsync(f.hsum, 0, (size_t)f.nb * nv * sizeof(XSum), stream)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(f.hcnt, 0, (size_t)f.nb * 4, stream)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(f.rem, 0, (size_t)(K + 1) * sizeof(XSum), stream)) != hipSuccess) return e;
  uint32_t *scount = (uint32_t *)(w + L.scount);
  if ((e = hipMemsetAsync(scount, 0, 4, stream)) != hipSuccess) return e;
  // splitters from a strided sample
  const uint32_t ns = (uint32_t)(N < 65536 ? N : 65536);
  const int64_t stride = ns ? N / ns : 1;
  uint64_t *skey = (uint64_t *)(w + L.skey), *tkey = (uint64_t *)(w + L.tkey);
  uint32_t *sidx = (uint32_t *)(w + L.sidx), *tidx = (uint32_t *)(w + L.tidx);
  uint32_t *hist = (uint32_t *)(w + L.hist), *hoff = (uint32_t *)(w + L.hoff);
  if (ns)
    hipLaunchKernelGGL(k_fix_sample, dim3((ns + FX_NT - 1) / FX_NT), dim3(FX_NT), 0, stream, f, stride, ns,
                       skey, sidx, scount);
  if ((e = hipMemcpyAsync(pinned, scount, 4, hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  const uint32_t nsc = pinned[0];
  if ((e = fx_sort(skey, sidx, tkey, tidx, nsc, hist, hoff, stream)) != hipSuccess) return e;
  if (f.nb > 1)
    hipLaunchKernelGGL(k_fix_split, dim3(1), dim3(128), 0, stream, skey, scount, f.nb, (uint64_t *)f.split);
  // bins and their exact sums
  if (bins_pass) {
    FixBins fb;
    fb.bin = f.bin;
    fb.kv = kv;
    fb.split = f.split;
    fb.hsum = f.hsum;
    fb.hcnt = f.hcnt;
    fb.nb = f.nb;
    fb.nv = nv;
    if ((e = bins_pass(fb)) != hipSuccess) return e;
  } else {
    const size_t lb = (size_t)f.nb * nv * sizeof(XSum) + (size_t)f.nb * 4 + 8 + (size_t)f.nb * 8;
    const int bins_lds = lb <= FX_LDS_MAX;
    const size_t lb_used = bins_lds ? lb : (size_t)f.nb * 8;
    if (lb_used > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fix_bins, dim3(persist), dim3(FX_NT), lb_used, stream, f, bins_lds);
  }
  hipLaunchKernelGGL(k_fix_locate, dim3(1), dim3(256), 0, stream, f);
  if ((e = hipMemcpyAsync(pinned, f.fs, sizeof(FixState), hipMemcpyDeviceToHost, stream)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(stream)) != hipSuccess) return e;
  FixState hs;
  memcpy(&hs, pinned, sizeof hs);
  const int rem_lds = (size_t)(K + 1) * sizeof(XSum) <= FX_LDS_MAX;
  const size_t lr = rem_lds ? (size_t)(K + 1) * sizeof(XSum) : 0;
  if (hs.bstar >= 0) {
    const uint32_t nch = (uint32_t)((N + FX_CHUNK - 1) / FX_CHUNK);
    uint32_t *bcnt = (uint32_t *)(w + L.bcnt), *boff = (uint32_t *)(w + L.boff);
    uint64_t *ckey = (uint64_t *)(w + L.ckey), *ckey2 = (uint64_t *)(w + L.ckey2);
    uint32_t *cidx = (uint32_t *)(w + L.cidx), *cidx2 = (uint32_t *)(w + L.cidx2);
    XSum *csum = (XSum *)(w + L.csum);
    hipLaunchKernelGGL(k_fix_bcount, dim3(nch), dim3(FX_NT), 0, stream, f, bcnt);
    hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, stream, bcnt, boff, (int64_t)nch, (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_fix_collect, dim3(nch), dim3(FX_NT), 0, stream, f, boff, ckey, cidx);
    if ((e = fx_sort(ckey, cidx, ckey2, cidx2, hs.nstar, hist, hoff, stream)) != hipSuccess) return e;
    const uint32_t nchs = (hs.nstar + FX_CHUNK - 1) / FX_CHUNK;
    if (nchs) {
      const int c_lds = (size_t)nv * sizeof(XSum) <= FX_LDS_MAX;
      if (!c_lds && (e = hipMemsetAsync(csum, 0, (size_t)nchs * nv * sizeof(XSum), stream)) != hipSuccess)
        return e;
      hipLaunchKernelGGL(k_fix_chunk, dim3(nchs), dim3(FX_NT), c_lds ? (size_t)nv * sizeof(XSum) : 0, stream,
                         f, cidx, csum, c_lds);
      hipLaunchKernelGGL(k_fix_prefix, dim3(nv), dim3(FX_NT), 0, stream, f, cidx, csum, nchs);
    }
    hipLaunchKernelGGL(k_fix_reset, dim3(persist), dim3(FX_NT), lr, stream, f, (const uint32_t *)nullptr,
                       rem_lds);
    if (hs.nstar) {
      const uint32_t g = (hs.nstar + FX_NT - 1) / FX_NT;
      hipLaunchKernelGGL(k_fix_reset, dim3(g < (uint32_t)persist ? g : (uint32_t)persist), dim3(FX_NT), lr,
                         stream, f, (const uint32_t *)cidx, rem_lds);
    }
  }
  hipLaunchKernelGGL(k_fix_final, dim3((K + 1 + 255) / 256), dim3(256), 0, stream, f, R, P, R_out, P_out,
                     n_reset);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched helpers: statistics by column table, flat per-(instance, k) init
// and finish
// ---------------------------------------------------------------------------
struct ColDesc {
  const double *partials;  // [nblk][K + 2] of the instance
  const double *lam;       // [K]
  const double *B;         // [K]
  double *out;             // destination of this column
  int nblk, K, col, pad;
};

__global__ void __launch_bounds__(256) k_reduce_stats_tab(const ColDesc *tab) {
  __shared__ double red[256];
  const ColDesc d = tab[blockIdx.x];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < d.nblk; b += 256) s = s + d.partials[(size_t)b * (d.K + 2) + d.col];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = red[t] + red[t + w];
    __syncthreads();
  }
  if (t != 0) return;
  s = red[0];
  if (d.col == d.K) {
    for (int k = 0; k < d.K; ++k) { const double lb = d.lam[k] * d.B[k]; s = s + lb; }
  }
  *d.out = s;
}

__global__ void k_scd_init_flat(KState *st, int Kf, const double *const *lam_in, const int *kinst,
                                const int *klocal, double *hint, int window, const uint64_t *eoff,
                                const uint32_t *ecap) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= Kf) return;
  const double l = lam_in[kinst[f]][klocal[f]];
  KState s;
  s.mode = KS_EXP;
  s.bstar = 0;
  s.shift = 0;
  s.overflow = 0;
  s.n_emit = 0;
  s.flags = 0;
  s.center = l;
  // bucket width: a power of two above the last step when there is one
  s.delta = (hint && hint[f] > 0.0) ? hint[f] : (l > 0x1p-20 ? ldexp(1.0, ilogb(l) - 10) : 0x1p-20);
  s.fab = xs_zero();
  s.result = l;
  s.klo = 0;
  s.khi = ~0ull;
  s.hull_lo = ~0ull;
  s.hull_hi = 0;
  s.wlo = 0.0;
  s.whi = 0.0;
  s.hw = 0.0;
  s.corr = xs_zero();
  s.eoff = eoff ? eoff[f] : 0;
  s.ecap = ecap ? ecap[f] : 0;
  s.pad2 = 0;
  // a window from the multiplier's history (as the single-instance search);
  // the history columns shift once per iteration, here
  if (hint) {
    const double prev = hint[2 * Kf + f];
    const double drift = fabs(l - hint[3 * Kf + f]);
    hint[3 * Kf + f] = prev;
    hint[2 * Kf + f] = l;
    if (window && hint[f] > 0.0) choose_window(s, hint[Kf + f], prev, drift);
  }
  st[f] = s;
}

// Batched: flags[s] = 1 if instance s has a knapsack that needs another
// pass over its users (knapsacks koff[s] .. koff[s+1]-1 of the flat state).
__global__ void k_inst_active(const KState *st, const int *koff, int n, int *flags) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int on = 0;
  for (int f = koff[s]; f < koff[s + 1]; ++f) on |= walk_mode(st[f].mode) ? 1 : 0;
  flags[s] = on;
}

__global__ void k_scd_finish_flat(const KState *st, int Kf, double *const *lam_out, const int *kinst,
                                  const int *klocal, double *hint) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= Kf) return;
  const double nl = st[f].result;
  lam_out[kinst[f]][klocal[f]] = nl;
  if (hint) {
    // the next iteration's bucket width: the power of two above this step
    const double step = fabs(nl - st[f].center);
    const double floor_ = (nl > 0x1p-20 ? nl : 0x1p-20) * 0x1p-30;
    const double w = step > floor_ ? step : floor_;
    hint[f] = ldexp(1.0, ilogb(w) + 1);
    hint[Kf + f] = w;
  }
}

hipError_t kp_launch_sweep_batched(const SweepArgs *descs, const TileGeom *geoms, const int *block_off,
                                   int n_inst, int total_blocks, size_t lds, hipStream_t stream,
                                   const int *n_dev) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)k_sweep_batched,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sweep_batched, dim3(total_blocks), dim3(NT), lds, stream, descs, geoms,
                     block_off, n_inst, n_dev);
  return hipGetLastError();
}

hipError_t kp_launch_batched_aux(int which, const void *tab, int n, KState *st, const void *lam_ptrs,
                                 const int *kinst, const int *klocal, double *hint, const uint64_t *eoff,
                                 const uint32_t *ecap, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (which == 0) {
    hipLaunchKernelGGL(k_reduce_stats_tab, dim3(n), dim3(256), 0, stream, (const ColDesc *)tab);
  } else if (which == 1 || which == 3) {   // 3: with a window where the last step allows
    hipLaunchKernelGGL(k_scd_init_flat, dim3((n + 63) / 64), dim3(64), 0, stream, st, n,
                       (const double *const *)lam_ptrs, kinst, klocal, hint,
                       which == 3 ? 1 : 0, eoff, ecap);
  } else {
    hipLaunchKernelGGL(k_scd_finish_flat, dim3((n + 63) / 64), dim3(64), 0, stream, (const KState *)st,
                       n, (double *const *)lam_ptrs, kinst, klocal, hint);
  }
  return hipGetLastError();
}

hipError_t kp_launch_inst_active(const KState *st, const int *koff, int n, int *flags, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inst_active, dim3((n + 63) / 64), dim3(64), 0, stream, st, koff, n, flags);
  return hipGetLastError();
}

TileGeom kp_tile_geom(const SweepArgs &a, int U) {
  TileGeom g;
  g.U = U;
  g.M = a.pr.M;
  g.K = a.pr.K;
  g.aligned = a.pr.fmt == 0 && ((uintptr_t)a.pr.b & 15) == 0 && (((int64_t)U * g.M * g.K) & 3) == 0;
  return g;
}

size_t kp_coldesc_size() { return sizeof(ColDesc); }
void kp_coldesc_fill(void *dst, const double *partials, const double *lam, const double *B, double *out,
                     int nblk, int K, int col) {
  ColDesc d;
  d.partials = partials; d.lam = lam; d.B = B; d.out = out;
  d.nblk = nblk; d.K = K; d.col = col; d.pad = 0;
  memcpy(dst, &d, sizeof d);
}

// ---------------------------------------------------------------------------
// host-side launch helpers (called from the C ABI)
// ---------------------------------------------------------------------------
size_t kp_sweep_lds_bytes(int U, int M, int K, bool scd, int fmt, bool hist = true) {
  auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  const size_t R = (size_t)U * M, Q = (size_t)U * K;
  size_t s = r16(R * K * 4) + r16(R * 8) + r16(R) + r16((size_t)U * 8) * 2 + r16(Q * 8) +
             r16((size_t)U * 16) + r16((size_t)(K + 2) * 8);
  s += r16((size_t)K * 8);   // lambda
  s += r16(R * 4) + r16((R + 1) * 4) + r16(16);   // staged profits, row offsets, entry base
  if (scd) s += r16(R);                            // per-item threshold elements
  if (fmt == 1) s += 2 * r16((size_t)NT * ECH * 4);  // staged CSR entries
  if (scd)
    s += r16((size_t)K * sizeof(KState)) + (hist ? r16((size_t)K * KP_NB * sizeof(XSum)) + r16((size_t)K * KP_NB * 4) : 0) +
         4 * r16((size_t)K * 4) + 2 * r16((size_t)K * 8) + r16(16) +
         r16(16) + r16((size_t)K * sizeof(XSum)) + r16((size_t)U * 16);   // widest window, corrections, per-user filter
  return s;
}

// Blocks of the batched sweep kernel that can be resident at once (0 if unknown).
int kp_sweep_batched_resident(size_t lds) {
  const void *fn = (const void *)k_sweep_batched;
  if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds) != hipSuccess || per_cu < 1) return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// Blocks of the general sweep kernel that can be resident at once (0 if unknown).
int kp_sweep_resident_grid(int U, int M, int K, bool scd, int fmt, bool hist = true) {
  const size_t lds = kp_sweep_lds_bytes(U, M, K, scd, fmt, hist);
  const void *fn = sweep_fn(fmt, scd, M, K);
  if (lds > 64 * 1024 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds) != hipSuccess || per_cu < 1) return 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

hipError_t kp_launch_sweep(const SweepArgs &a, int U, int grid, bool scd, hipStream_t stream,
                           int *used) {
  TileGeom g;
  g.U = U;
  g.M = a.pr.M;
  g.K = a.pr.K;
  g.aligned = a.pr.fmt == 0 && ((uintptr_t)a.pr.b & 15) == 0 &&
              (((int64_t)U * g.M * g.K) & 3) == 0;
  const size_t lds = kp_sweep_lds_bytes(U, g.M, g.K, scd, a.pr.fmt, !(scd && a.no_hist));
  const void *fn = sweep_fn(a.pr.fmt, scd, g.M, g.K);
  if (lds > 64 * 1024) {
    // shapes with many knapsacks need more than the default 64 KB of LDS
    // (gfx950 has 160 KB per workgroup)
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // persistent launch: at most the blocks that can be resident at once
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, lds) == hipSuccess && per_cu > 0 &&
      hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
    if (grid > per_cu * cus) grid = per_cu * cus;
  }
  if (used) *used = grid;
  if (a.pr.fmt == 0 && g.M == 10 && g.K == 10) {
    if (scd) hipLaunchKernelGGL((k_sweep<0, true, 10, 10>), dim3(grid), dim3(NT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_sweep<0, false, 10, 10>), dim3(grid), dim3(NT), lds, stream, a, g);
  } else if (a.pr.fmt == 0 && g.M == 20 && g.K == 50) {
    if (scd) hipLaunchKernelGGL((k_sweep<0, true, 20, 50>), dim3(grid), dim3(NT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_sweep<0, false, 20, 50>), dim3(grid), dim3(NT), lds, stream, a, g);
  } else if (a.pr.fmt == 0) {
    if (scd) hipLaunchKernelGGL((k_sweep<0, true>), dim3(grid), dim3(NT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_sweep<0, false>), dim3(grid), dim3(NT), lds, stream, a, g);
  } else {
    if (scd) hipLaunchKernelGGL((k_sweep<1, true>), dim3(grid), dim3(NT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_sweep<1, false>), dim3(grid), dim3(NT), lds, stream, a, g);
  }
  return hipGetLastError();
}

hipError_t kp_launch_reduce_stats(const double *partials, int nblk, int K, const double *lam,
                                  const double *B, double *R, double *g, double *P,
                                  hipStream_t stream) {
  hipLaunchKernelGGL(k_reduce_stats, dim3(K + 2), dim3(256), 0, stream, partials, nblk, K, lam, B,
                     R, g, P);
  return hipGetLastError();
}

hipError_t kp_launch_scd_init(KState *st, int K, const double *lam_in, const uint8_t *kmask,
                              double *hist, int hinted, int window, int interp, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_init, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, lam_in, kmask,
                     hist, hinted, window, interp);
  return hipGetLastError();
}

hipError_t kp_launch_scd_locate_select(KState *st, int K, const double *B, const double *R,
                                       const int *rinst, XSum *hist_sum, uint32_t *hist_cnt,
                                       const double *ev1, const double *ev2, uint32_t emit_cap,
                                       int *pending, unsigned int *win, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_locate, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, B, R, rinst, hist_sum,
                     hist_cnt, emit_cap, win);
  hipLaunchKernelGGL(k_scd_select, dim3(K), dim3(SEL_NT), 0, stream, st, B, ev1, ev2, emit_cap, win);
  hipLaunchKernelGGL(k_count_pending, dim3(1), dim3(256), 0, stream, st, K, pending);
  return hipGetLastError();
}

hipError_t kp_launch_count_modes(const KState *st, int K, int *out, hipStream_t stream) {
  hipLaunchKernelGGL(k_count_modes, dim3(1), dim3(256), 0, stream, st, K, out);
  return hipGetLastError();
}

hipError_t kp_launch_scd_finish(const KState *st, int K, const double *lam_in, double *lam_out,
                                double *delta_next, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_finish, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, lam_in,
                     lam_out, delta_next, (int *)nullptr);
  return hipGetLastError();
}

static unsigned gather_blocks(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t kp_launch_gather_dense(const float *p, const float *b, const int64_t *users, int64_t n, int M,
                                  int K, float *sp, float *sb, hipStream_t stream) {
  hipLaunchKernelGGL(k_gather_rows, dim3(gather_blocks(n * M)), dim3(256), 0, stream, p, sp, users, n,
                     (int64_t)M);
  if (b)
    hipLaunchKernelGGL(k_gather_rows, dim3(gather_blocks(n * M * K)), dim3(256), 0, stream, b, sb,
                       users, n, (int64_t)M * K);
  return hipGetLastError();
}

hipError_t kp_launch_gather_csr_ptr(const int64_t *rowptr, const int64_t *users, int64_t n, int M,
                                    int64_t *len, int64_t *subptr, hipStream_t stream) {
  hipLaunchKernelGGL(k_gather_len, dim3(gather_blocks(n * M)), dim3(256), 0, stream, rowptr, users, n,
                     M, len);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, stream, len, subptr, n * M);
  return hipGetLastError();
}

hipError_t kp_launch_gather_csr(const int64_t *rowptr, const int32_t *col, const float *val,
                                const int64_t *users, int64_t n, int M, const int64_t *subptr,
                                int32_t *scol, float *sval, hipStream_t stream) {
  hipLaunchKernelGGL(k_gather_csr, dim3(gather_blocks(n * M)), dim3(256), 0, stream, rowptr, col, val,
                     users, n, M, subptr, scol, sval);
  return hipGetLastError();
}

hipError_t kp_launch_recenter(KState *st, int K, const double *lam_hat, const double *lam_in, int window,
                              hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_recenter, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, lam_hat, lam_in, window);
  return hipGetLastError();
}

hipError_t kp_launch_strided_users(int64_t *users, int64_t n, int64_t stride, int64_t off, hipStream_t stream) {
  hipLaunchKernelGGL(k_strided_users, dim3(gather_blocks(n)), dim3(256), 0, stream, users, n, stride, off);
  return hipGetLastError();
}

hipError_t kp_launch_uniform_rowptr(int64_t *rowptr, int64_t nrows, int D, hipStream_t stream) {
  hipLaunchKernelGGL(k_uniform_rowptr, dim3(gather_blocks(nrows + 1)), dim3(256), 0, stream, rowptr, nrows, D);
  return hipGetLastError();
}

hipError_t kp_launch_dd_update(int K, double alpha, const double *R, const double *B, double *lam,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_dd_update, dim3((K + 63) / 64), dim3(64), 0, stream, K, alpha, R, B, lam);
  return hipGetLastError();
}

hipError_t kp_launch_dual_backward(int K, const double *R, const double *B, const double *gout,
                                   double *glam, hipStream_t stream) {
  hipLaunchKernelGGL(k_dual_backward, dim3((K + 63) / 64), dim3(64), 0, stream, K, R, B, gout,
                     glam);
  return hipGetLastError();
}

hipError_t kp_launch_validate(const float *v, int64_t n, unsigned int *flags, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)blocks), dim3(256), 0, stream, v, n, flags);
  return hipGetLastError();
}

hipError_t kp_launch_validate_csr(const int64_t *rowptr, const int32_t *col, int64_t nrows, int K,
                                  unsigned int *flags, hipStream_t stream) {
  if (nrows <= 0) return hipSuccess;
  int64_t blocks = (nrows + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate_csr, dim3((unsigned)blocks), dim3(256), 0, stream, rowptr, col,
                     nrows, K, flags);
  return hipGetLastError();
}

__global__ void k_fill_f64(double *dst, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

// A fill kernel rather than hipMemsetAsync, for paths a caller may capture in
// a HIP graph.
hipError_t kp_launch_fill_f64(double *dst, int64_t n, double v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)blocks), dim3(256), 0, stream, dst, n, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming-read probe: the achievable HBM read bandwidth for a buffer of
// the sweep's size (the ceiling its roofline fraction is also quoted
// against).  Every thread reads 16-byte words with four loads in flight,
// folds them with XOR (so no load is dead) and every block XORs its result
// into one word; XOR is order-free, so the word is deterministic.
// ---------------------------------------------------------------------------
#define SR_NT 256
typedef unsigned int sr_v4u __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(SR_NT) k_stream_read(const uint4 *src, int64_t n16, unsigned long long *out) {
  // eight nontemporal 16-byte loads per thread in flight (the sweep kernels'
  // staging uses the same cache policy)
  const sr_v4u *s = (const sr_v4u *)src;
  sr_v4u acc = {0u, 0u, 0u, 0u};
  const int64_t stride = (int64_t)gridDim.x * SR_NT;
  int64_t i = (int64_t)blockIdx.x * SR_NT + threadIdx.x;
  for (; i + 7 * stride < n16; i += 8 * stride) {
    sr_v4u v[8];
    #pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(s + i + u * stride);
    #pragma unroll
    for (int u = 0; u < 8; ++u) acc ^= v[u];
  }
  for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(s + i);
  unsigned long long v = ((unsigned long long)(acc.x ^ acc.z) << 32) | (unsigned long long)(acc.y ^ acc.w);
  for (int off = 32; off > 0; off >>= 1) v ^= __shfl_xor(v, off, 64);
  __shared__ unsigned long long part[SR_NT / 64];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < SR_NT / 64; ++w) t ^= part[w];
    atomicXor(out, t);
  }
}

// The resident blocks of the probe (at most `grid` when grid > 0).
hipError_t kp_launch_stream_read(const void *src, int64_t n16, unsigned long long *out, int grid,
                                 hipStream_t stream) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_stream_read, SR_NT, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 8;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  int g = per_cu * cus;
  if (grid > 0 && grid < g) g = grid;
  hipLaunchKernelGGL(k_stream_read, dim3(g), dim3(SR_NT), 0, stream, (const uint4 *)src, n16, out);
  return hipGetLastError();
}
