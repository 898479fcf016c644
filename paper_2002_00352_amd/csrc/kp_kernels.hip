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
// Sums across users are atomic-free: per (user,k) values go to LDS and are
// added in user order, per block into a private slot, and slots are added in
// block order by a second kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "kp_internal.h"

#define NT 256

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

__device__ __forceinline__ uint64_t dkey(double v) {
  return (uint64_t)__double_as_longlong(v);
}
__device__ __forceinline__ double kdbl(uint64_t k) { return __longlong_as_double((long long)k); }

// Exponential bucket of a breakpoint around the previous multiplier: 0 inside
// (center - delta, center + delta), else sign * (1 + floor(log2(|d| / delta)))
// capped at 31; delta is a power of two, so the log is an exponent difference.
// Monotone non-decreasing in v.
__device__ __forceinline__ int exp_bucket(double v, double center, double delta) {
  double d = v - center;
  double a = fabs(d);
  if (!(a >= delta)) return 0;
  int ea = (int)((dkey(a) >> 52) & 0x7FF);
  int ed = (int)((dkey(delta) >> 52) & 0x7FF);
  int id = 1 + (ea - ed);
  id = id > 31 ? 31 : id;
  return d < 0.0 ? -id : id;
}

struct TileGeom {
  int U;            // users per tile
  int M, K;
};

// Laminar-matroid greedy over the ranked items: accept an eligible item when
// no node containing it is full.  Equivalent to Alg.1 (both return the unique
// maximum-weight independent set under the strict order (p~ desc, j asc)).
__device__ __forceinline__ uint64_t greedy_mask(const uint8_t *perm, int M, uint64_t eligible,
                                                const TreeDev &T) {
  uint64_t S = 0, blocked = 0;
  for (int r = 0; r < M; ++r) {
    const int j = perm[r];
    const uint64_t bit = 1ull << j;
    if ((eligible & bit) && !(blocked & bit)) {
      S |= bit;
      for (int l = 0; l < T.L; ++l) {
        const uint64_t m = T.mask[l];
        if ((m & bit) && popc64(S & m) >= T.cap[l]) blocked |= m;
      }
    }
  }
  return S;
}

// ---------------------------------------------------------------------------
// the sweep kernel
// ---------------------------------------------------------------------------
template <int FMT, bool SCD>
__global__ void __launch_bounds__(NT) k_sweep(const SweepArgs a, const TileGeom g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int M = g.M, K = g.K, U = g.U;
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
  double *vk = (double *)carve((size_t)Q * 8);            // per (user,k) consumption
  double *uPG = (double *)carve((size_t)U * 16);          // per user P_i, G_i
  double *acc = (double *)carve((size_t)(K + 2) * 8);     // block running sums
  double *hs = nullptr;
  uint32_t *hc = nullptr;
  int *kmode = nullptr;
  if (SCD) {
    hs = (double *)carve((size_t)K * KP_NB * 8);
    hc = (uint32_t *)carve((size_t)K * KP_NB * 4);
    kmode = (int *)carve((size_t)K * 4);
  }
  for (int t = tid; t < K + 2; t += NT) acc[t] = 0.0;
  if (SCD) {
    for (int t = tid; t < K * KP_NB; t += NT) { hs[t] = 0.0; hc[t] = 0u; }
    for (int t = tid; t < K; t += NT) kmode[t] = a.st[t].mode;
  }
  const int64_t N = a.pr.N;
  const double *lam = a.lam;

  for (int64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int64_t u0 = tile * (int64_t)U;
    const int nu = (int)((N - u0) < U ? (N - u0) : U);     // users in this tile
    const int nr = nu * M;
    __syncthreads();   // previous tile's readers are done with the LDS tile
    // ---- phase 0 + A: stage costs, score ----
    if (FMT == 0) {
      // dense: the tile's costs are one contiguous run of nr*K floats
      const float *src = a.pr.b + u0 * (int64_t)M * K;
      const int64_t nf = (int64_t)nr * K;
      const bool al = ((((uintptr_t)src) & 15) == 0);
      if (al) {
        const int n4 = (int)(nf >> 2);
        typedef float v4f __attribute__((ext_vector_type(4)));
        const v4f *s4 = (const v4f *)src;
        v4f *d4 = (v4f *)bt;
        for (int t = tid; t < n4; t += NT) d4[t] = __builtin_nontemporal_load(s4 + t);
        for (int t = (n4 << 2) + tid; t < nf; t += NT) bt[t] = src[t];
      } else {
        for (int t = tid; t < nf; t += NT) bt[t] = src[t];
      }
      __syncthreads();
      for (int r = tid; r < nr; r += NT) {
        double accp = (double)a.pr.p[u0 * M + r];
        const float *br = bt + (size_t)r * K;
        for (int k = 0; k < K; ++k) {
          const double prod = lam[k] * (double)br[k];
          accp = accp - prod;
        }
        pt[r] = accp;
      }
    } else {
      // CSR: zero the dense tile, scatter each row's stored entries and
      // score over the stored columns in ascending order (skipping zeros is
      // bit-identical: acc - lambda*0 == acc).
      for (int t = tid; t < R * K; t += NT) bt[t] = 0.0f;
      __syncthreads();
      for (int r = tid; r < nr; r += NT) {
        const int64_t row = u0 * M + r;
        const int64_t e0 = a.pr.rowptr[row], e1 = a.pr.rowptr[row + 1];
        double accp = (double)a.pr.p[row];
        for (int64_t e = e0; e < e1; ++e) {
          const int k = a.pr.col[e];
          if ((unsigned)k >= (unsigned)K) continue;   // malformed column: ignored (kp_validate_inputs reports it)
          const float v = a.pr.val[e];
          bt[(size_t)r * K + k] = v;
          const double prod = lam[k] * (double)v;
          accp = accp - prod;
        }
        pt[r] = accp;
      }
    }
    __syncthreads();
    // ---- phase B1: rank items and run the greedy, one thread per user ----
    if (tid < nu) {
      const int u = tid;
      const double *z = pt + u * M;
      uint8_t rank[KP_MAX_M];
      uint64_t pos = 0;
      for (int j = 0; j < M; ++j) { rank[j] = 0; if (z[j] > 0.0) pos |= 1ull << j; }
      for (int j = 0; j < M; ++j) {
        const double zj = z[j];
        int rj = rank[j];
        for (int jj = j + 1; jj < M; ++jj) {
          if (z[jj] > zj) ++rj; else rank[jj]++;
        }
        rank[j] = (uint8_t)rj;
      }
      uint8_t *pu = perm + u * M;
      for (int j = 0; j < M; ++j) pu[rank[j]] = (uint8_t)j;
      const uint64_t S = greedy_mask(pu, M, pos, a.tree);
      Sm[u] = S;
      Pm[u] = pos;
      double Pi = 0.0, Gi = 0.0;
      const float *pp = a.pr.p + (u0 + u) * M;
      for (int j = 0; j < M; ++j) {
        if (S >> j & 1) { Pi = Pi + (double)pp[j]; Gi = Gi + z[j]; }
      }
      uPG[2 * u] = Pi;
      uPG[2 * u + 1] = Gi;
      if (a.x_out) {
        uint8_t *xo = a.x_out + (u0 + u) * M;
        for (int j = 0; j < M; ++j) xo[j] = (uint8_t)(S >> j & 1);
      }
    }
    __syncthreads();
    // ---- phase B2: one thread per (user, knapsack) ----
    for (int q = tid; q < nu * K; q += NT) {
      const int u = q / K, k = q - u * K;
      const uint64_t S0 = Sm[u];
      const float *bu = bt + (size_t)u * M * K;
      double v = 0.0;
      for (int j = 0; j < M; ++j)
        if (S0 >> j & 1) v = v + (double)bu[j * K + k];
      vk[q] = v;
      if (SCD) {
        const int mode = kmode[k];
        if (mode == KS_EXP || mode == KS_EMIT_BUCKET || mode == KS_HULL_BUCKET ||
            mode == KS_REFINE || mode == KS_EMIT_RANGE) {
          const double lk = lam[k];
          const double *zu = pt + u * M;
          uint64_t A = 0;   // moving lines: b_jk > 0
          for (int j = 0; j < M; ++j) if (bu[j * K + k] > 0.0f) A |= 1ull << j;
          if (A) {
            // start above every breakpoint: only horizontal positive lines,
            // ranked by p~ (their lines are c_j = p~_j exactly)
            uint64_t S = greedy_mask(perm + u * M, M, Pm[u] & ~A, a.tree);
            const KState &ks = a.st[k];
            const double center = ks.center, delta = ks.delta;
            const int bstar = ks.bstar;
            const uint64_t klo = ks.klo, khi = ks.khi;
            const int shift = ks.shift;
            const int maxev = M * M + M + 8;
            for (int ev = 0; ; ++ev) {
              if (ev >= maxev) { atomicAdd(a.err, 1ull); break; }
              double best = 0.0;
              int bo = -1, bs = -1;
              uint64_t cand = A & ~S;
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
                if (!tight) {
                  if (co > 0.0) {
                    const double val = co / bo_d;
                    if (val > best) { best = val; bo = o; bs = -1; }
                  }
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
                      const double val = num / den;
                      if (val > best) { best = val; bo = o; bs = s; }
                    }
                  }
                }
              }
              if (bo < 0) break;
              const double bo_d = (double)bu[bo * K + k];
              const double v2 = bs >= 0 ? bo_d - (double)bu[bs * K + k] : bo_d;
              S = (S | (1ull << bo)) & ~(bs >= 0 ? (1ull << bs) : 0ull);
              // bin / emit (v1 = best, v2)
              const uint64_t key = dkey(best);
              bool emit = false;
              if (mode == KS_EXP) {
                const int id = exp_bucket(best, center, delta);
                atomicAdd(&hs[k * KP_NB + 32 + id], v2);
                atomicAdd(&hc[k * KP_NB + 32 + id], 1u);
                emit = (id >= -KP_CENTRAL_W && id <= KP_CENTRAL_W);
              } else if (mode == KS_EMIT_BUCKET || mode == KS_HULL_BUCKET) {
                if (exp_bucket(best, center, delta) == bstar) {
                  atomicMin((unsigned long long *)&a.st[k].hull_lo, (unsigned long long)key);
                  atomicMax((unsigned long long *)&a.st[k].hull_hi, (unsigned long long)key);
                  emit = (mode == KS_EMIT_BUCKET);
                }
              } else if (mode == KS_REFINE) {
                if (key >= klo && key <= khi) {
                  const int bin = (int)((key - klo) >> shift);
                  atomicAdd(&hs[k * KP_NB + bin], v2);
                  atomicAdd(&hc[k * KP_NB + bin], 1u);
                }
              } else {  // KS_EMIT_RANGE
                emit = (key >= klo && key <= khi);
              }
              if (emit) {
                const uint32_t slot = atomicAdd(&a.st[k].n_emit, 1u);
                if (slot < a.emit_cap) {
                  a.emit_v1[(size_t)k * a.emit_cap + slot] = best;
                  a.emit_v2[(size_t)k * a.emit_cap + slot] = v2;
                } else {
                  a.st[k].overflow = 1;
                }
              }
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
    for (int t = tid; t < K + 2; t += NT) a.partials[(size_t)blockIdx.x * (K + 2) + t] = acc[t];
  }
  if (SCD) {
    for (int t = tid; t < K * KP_NB; t += NT) {
      if (hc[t]) {
        atomicAdd(&a.hist_sum[t], hs[t]);
        atomicAdd(&a.hist_cnt[t], hc[t]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// second-level reduction of the block partials (fixed order), dual value
// ---------------------------------------------------------------------------
__global__ void k_reduce_stats(const double *partials, int nblk, int K, const double *lam,
                               const double *B, double *R, double *g, double *P) {
  // one thread per output column; columns K (G) and K+1 (P)
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K + 2) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s = s + partials[(size_t)b * (K + 2) + c];
  if (c < K) {
    if (R) R[c] = s;
  } else if (c == K) {
    // g = sum_i G_i + sum_k lambda_k B_k
    double t = s;
    for (int k = 0; k < K; ++k) { const double lb = lam[k] * B[k]; t = t + lb; }
    if (g) *g = t;
  } else {
    if (P) *P = s;
  }
}

// ---------------------------------------------------------------------------
// SCD threshold search
// ---------------------------------------------------------------------------
__global__ void k_scd_init(KState *st, int K, const double *lam_in, const uint8_t *kmask,
                           const double *delta_hint) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  KState s;
  s.mode = (kmask && !kmask[k]) ? KS_DONE : KS_EXP;
  s.bstar = 0;
  s.shift = 0;
  s.overflow = 0;
  s.n_emit = 0;
  s.pad = 0;
  s.center = lam_in[k];
  double d = delta_hint ? delta_hint[k] : 0.0;
  if (!(d > 0.0)) {
    // no history: 2^-10 of the multiplier (or 2^-30 absolute), a power of two
    const double base = lam_in[k] > 0x1p-20 ? lam_in[k] : 0x1p-20;
    d = ldexp(1.0, ilogb(base) - 10);
  }
  s.delta = d;
  s.F_above = 0.0;
  s.result = lam_in[k];
  s.klo = 0;
  s.khi = ~0ull;
  s.hull_lo = ~0ull;
  s.hull_hi = 0;
  st[k] = s;
}

__device__ __forceinline__ int bits_needed(uint64_t x) { return x ? 64 - __clzll((long long)x) : 0; }

__device__ __forceinline__ void set_refine(KState &s, uint64_t lo, uint64_t hi) {
  s.klo = lo;
  s.khi = hi;
  const int nb = bits_needed(hi - lo);
  s.shift = nb > 6 ? nb - 6 : 0;   // (hi - lo) >> shift < 64
  s.mode = KS_REFINE;
}

// After a pass: pick the bin holding the threshold and choose the next step.
__global__ void k_scd_locate(KState *st, int K, const double *B, double *hist_sum,
                             uint32_t *hist_cnt, uint32_t emit_cap) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  KState s = st[k];
  const double Bk = B[k];
  const double *hsum = hist_sum + (size_t)k * KP_NB;
  const uint32_t *hcnt = hist_cnt + (size_t)k * KP_NB;
  if (s.mode == KS_EXP) {
    double total = 0.0;
    for (int b = 0; b < KP_NB; ++b) total = total + hsum[b];
    if (total <= Bk) {
      s.mode = KS_DONE;
      s.result = 0.0;
    } else {
      double cum = 0.0;
      int bin = 1;
      for (int b = KP_NB - 1; b >= 1; --b) {
        if (hcnt[b] && cum + hsum[b] > Bk) { bin = b; break; }
        cum = cum + hsum[b];
      }
      s.bstar = bin - 32;
      s.F_above = cum;
      const bool central = s.bstar >= -KP_CENTRAL_W && s.bstar <= KP_CENTRAL_W;
      if (central && !s.overflow) {
        s.mode = KS_SELECT_BUCKET;
      } else {
        s.mode = hcnt[bin] <= emit_cap ? KS_EMIT_BUCKET : KS_HULL_BUCKET;
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
    double cum = s.F_above;
    int bin = -1;
    for (int b = KP_NB - 1; b >= 0; --b) {
      if (hcnt[b] && cum + hsum[b] > Bk) { bin = b; break; }
      cum = cum + hsum[b];
    }
    if (bin < 0) {  // cannot happen with exact sums; fall back to the lowest bin
      bin = 0;
      cum = s.F_above;
      for (int b = KP_NB - 1; b >= 1; --b) cum = cum + hsum[b];
    }
    s.F_above = cum;
    const uint64_t lo = s.klo + ((uint64_t)bin << s.shift);
    const uint64_t hi0 = lo + ((((uint64_t)1) << s.shift) - 1);
    const uint64_t hi = hi0 < s.khi ? hi0 : s.khi;
    if (lo == hi) {
      s.mode = KS_DONE;
      s.result = kdbl(lo);
    } else if (hcnt[bin] <= emit_cap) {
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
  }
  st[k] = s;
  for (int b = 0; b < KP_NB; ++b) { hist_sum[(size_t)k * KP_NB + b] = 0.0; hist_cnt[(size_t)k * KP_NB + b] = 0u; }
}

// Exact threshold among the emitted events of one knapsack (one block per k):
// narrow the key range with LDS histograms until at most KP_SORT_MAX events
// remain, sort them (bitonic, descending), scan the increments and return the
// first distinct breakpoint whose cumulative increment exceeds B_k.
#define SEL_NT 1024
__global__ void __launch_bounds__(SEL_NT) k_scd_select(KState *st, const double *B,
                                                       const double *emit_v1, const double *emit_v2,
                                                       uint32_t emit_cap) {
  const int k = blockIdx.x;
  __shared__ KState s;
  __shared__ double hsum[256];
  __shared__ uint32_t hcnt[256];
  __shared__ uint64_t skey[KP_SORT_MAX];
  __shared__ double sval[KP_SORT_MAX];
  __shared__ uint64_t lo, hi;
  __shared__ double Fab;
  __shared__ uint32_t nsel;
  __shared__ int done;
  __shared__ double result;
  const int tid = threadIdx.x;
  if (tid == 0) s = st[k];
  __syncthreads();
  if (s.mode != KS_SELECT_BUCKET && s.mode != KS_SELECT_RANGE) return;
  const uint32_t n = s.n_emit < emit_cap ? s.n_emit : emit_cap;
  const double *V1 = emit_v1 + (size_t)k * emit_cap;
  const double *V2 = emit_v2 + (size_t)k * emit_cap;
  const bool bucket = s.mode == KS_SELECT_BUCKET;
  const double Bk = B[k];
  if (tid == 0) {
    lo = bucket ? 0ull : s.klo;
    hi = bucket ? ~0ull : s.khi;
    Fab = s.F_above;
    done = 0;
  }
  __syncthreads();
  // narrowing loop
  for (int it = 0; it < 80; ++it) {
    if (tid == 0) nsel = 0;
    if (tid < 256) { hsum[tid] = 0.0; hcnt[tid] = 0u; }
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
      atomicAdd(&hsum[bin], V2[e]);
      atomicAdd(&hcnt[bin], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      double cum = Fab;
      int bin = -1;
      for (int b = 255; b >= 0; --b) {
        if (hcnt[b] && cum + hsum[b] > Bk) { bin = b; break; }
        cum = cum + hsum[b];
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
      double cum = Fab;
      double ans = m ? kdbl(skey[m - 1]) : kdbl(lo);
      uint32_t e = 0;
      while (e < m) {
        const uint64_t key = skey[e];
        while (e < m && skey[e] == key) { cum = cum + sval[e]; ++e; }
        if (cum > Bk) { ans = kdbl(key); break; }
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
    // next central window: the power of two at or above this step
    const double step = fabs(nl - lam_in[k]);
    const double floor_ = (nl > 0x1p-20 ? nl : 0x1p-20) * 0x1p-30;
    const double w = step > floor_ ? step : floor_;
    delta_next[k] = ldexp(1.0, ilogb(w) + 1);
  }
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
// host-side launch helpers (called from the C ABI)
// ---------------------------------------------------------------------------
size_t kp_sweep_lds_bytes(int U, int M, int K, bool scd) {
  auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  const size_t R = (size_t)U * M, Q = (size_t)U * K;
  size_t s = r16(R * K * 4) + r16(R * 8) + r16(R) + r16((size_t)U * 8) * 2 + r16(Q * 8) +
             r16((size_t)U * 16) + r16((size_t)(K + 2) * 8);
  if (scd) s += r16((size_t)K * KP_NB * 8) + r16((size_t)K * KP_NB * 4) + r16((size_t)K * 4);
  return s;
}

hipError_t kp_launch_sweep(const SweepArgs &a, int U, int grid, bool scd, hipStream_t stream) {
  TileGeom g;
  g.U = U;
  g.M = a.pr.M;
  g.K = a.pr.K;
  const size_t lds = kp_sweep_lds_bytes(U, g.M, g.K, scd);
  if (a.pr.fmt == 0) {
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
  const int n = K + 2;
  hipLaunchKernelGGL(k_reduce_stats, dim3((n + 255) / 256), dim3(256), 0, stream, partials, nblk,
                     K, lam, B, R, g, P);
  return hipGetLastError();
}

hipError_t kp_launch_scd_init(KState *st, int K, const double *lam_in, const uint8_t *kmask,
                              const double *delta_hint, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_init, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, lam_in, kmask,
                     delta_hint);
  return hipGetLastError();
}

hipError_t kp_launch_scd_locate_select(KState *st, int K, const double *B, double *hist_sum,
                                       uint32_t *hist_cnt, const double *ev1, const double *ev2,
                                       uint32_t emit_cap, int *pending, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_locate, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, B, hist_sum,
                     hist_cnt, emit_cap);
  hipLaunchKernelGGL(k_scd_select, dim3(K), dim3(SEL_NT), 0, stream, st, B, ev1, ev2, emit_cap);
  hipLaunchKernelGGL(k_count_pending, dim3(1), dim3(256), 0, stream, st, K, pending);
  return hipGetLastError();
}

hipError_t kp_launch_scd_finish(const KState *st, int K, const double *lam_in, double *lam_out,
                                double *delta_next, hipStream_t stream) {
  hipLaunchKernelGGL(k_scd_finish, dim3((K + 63) / 64), dim3(64), 0, stream, st, K, lam_in,
                     lam_out, delta_next, (int *)nullptr);
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
