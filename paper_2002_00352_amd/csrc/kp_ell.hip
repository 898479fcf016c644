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
// queued and walked exactly once the one-item cases are done, so lanes walk
// together.  Sums across users are atomic-free (fixed-order wave reductions,
// waves added in order per block, blocks added in order by a second kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include "kp_device.h"

#define EW 4                 // waves per block
#define ENT (EW * 64)
#define EM 16                // largest M of this kernel

// wave-wide sum in a fixed butterfly order; every lane gets lane 0's value
__device__ __forceinline__ double wave_sum(double v) {
  #pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, 64);
  return __shfl(v, 0, 64);
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Copy n dwords from global src to LDS dst (coalesced; lanes past the end
// reload the last dword into the padded tail of dst).
__device__ __forceinline__ void stage_dwords(const void *src, int n, void *dst, int lane) {
  const uint32_t *s = (const uint32_t *)src;
  uint32_t *d = (uint32_t *)dst;
  for (int c = 0; c * 64 < n; ++c) {
    int i = c * 64 + lane;
    i = i < n ? i : n - 1;
    __builtin_amdgcn_global_load_lds((const void *)(s + i), (lds_void_t *)(d + c * 64), 4, 0, 0);
  }
}

struct EllGeom {
  int M, K, region;   // region: bytes of per-wave LDS
  int pad;
};

template <int D, bool SCD>
__global__ void __launch_bounds__(ENT) k_ell(const SweepArgs a, const EllGeom g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int M = g.M, K = g.K;
  size_t off = 0;
  auto carve = [&](size_t bytes) { unsigned char *p = smem + off; off += (bytes + 15) & ~(size_t)15; return p; };
  double *lam = (double *)carve((size_t)K * 8);
  uint64_t *tmask = (uint64_t *)carve((size_t)a.tree.L * 8 + 8);
  int *tcap = (int *)carve((size_t)a.tree.L * 4 + 4);
  double *wacc = (double *)carve((size_t)EW * (K + 2) * 8);
  KState *kst = SCD ? (KState *)carve((size_t)K * sizeof(KState)) : nullptr;
  double *hs = nullptr;
  uint32_t *hc = nullptr, *kcnt = nullptr, *kpos = nullptr, *kovf = nullptr, *nstage = nullptr;
  int *kmode = nullptr;
  unsigned long long *hmin = nullptr, *hmax = nullptr;
  if (SCD) {
    hs = (double *)carve((size_t)K * KP_NB * 8);
    hc = (uint32_t *)carve((size_t)K * KP_NB * 4);
    kmode = (int *)carve((size_t)K * 4);
    kcnt = (uint32_t *)carve((size_t)K * 4);
    kpos = (uint32_t *)carve((size_t)K * 4);
    kovf = (uint32_t *)carve((size_t)K * 4);
    hmin = (unsigned long long *)carve((size_t)K * 8);
    hmax = (unsigned long long *)carve((size_t)K * 8);
    nstage = (uint32_t *)carve(16);
  }
  unsigned char *wreg = smem + off + (size_t)wv * g.region;   // this wave's region
  for (int t = tid; t < K; t += ENT) lam[t] = a.lam[t];
  for (int t = tid; t < a.tree.L; t += ENT) { tmask[t] = a.tree.mask[t]; tcap[t] = a.tree.cap[t]; }
  for (int t = tid; t < EW * (K + 2); t += ENT) wacc[t] = 0.0;
  if (SCD) {
    for (int t = tid; t < K; t += ENT) {
      kst[t] = a.st[t];
      kmode[t] = a.st[t].mode;
      kcnt[t] = 0u; kpos[t] = 0u; kovf[t] = 0u;
      hmin[t] = ~0ull; hmax[t] = 0ull;
    }
    for (int t = tid; t < K * KP_NB; t += ENT) { hs[t] = 0.0; hc[t] = 0u; }
    if (tid == 0) *nstage = 0u;
  }
  __syncthreads();
  const int L = a.tree.L;
  const int64_t N = a.pr.N;
  const int64_t W = (int64_t)gridDim.x * EW;

  for (int64_t tile = (int64_t)blockIdx.x * EW + wv; tile < a.ntiles; tile += W) {
    const int64_t u0 = tile * 64;
    const int nu = (int)((N - u0) < 64 ? (N - u0) : 64);
    const bool act = lane < nu;
    // ---- stage the tile (coalesced) and move the lane's user into registers ----
    float *sp = (float *)wreg;
    int32_t *sc = (int32_t *)(wreg + (size_t)64 * M * 4);
    float *sv = (float *)(wreg + (size_t)64 * M * 4 + (size_t)64 * M * D * 4);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    stage_dwords(a.pr.p + u0 * M, nu * M, sp, lane);
    stage_dwords(a.pr.col + u0 * M * D, nu * M * D, sc, lane);
    stage_dwords(a.pr.val + u0 * M * D, nu * M * D, sv, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    float pv[EM];
    int cl[EM * D];
    float vl[EM * D];
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      if (j < M) {
        pv[j] = act ? sp[lane * M + j] : 0.0f;
        #pragma unroll
        for (int t = 0; t < D; ++t) {
          cl[j * D + t] = act ? sc[(lane * M + j) * D + t] : -1;
          vl[j * D + t] = act ? sv[(lane * M + j) * D + t] : 0.0f;
        }
      } else {
        pv[j] = 0.0f;
        #pragma unroll
        for (int t = 0; t < D; ++t) { cl[j * D + t] = -1; vl[j * D + t] = 0.0f; }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    __asm__ volatile("" ::: "memory");
    // ---- cost-adjusted profits ----
    double pt[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      double acc = (double)pv[j];
      #pragma unroll
      for (int t = 0; t < D; ++t) {
        const int k = cl[j * D + t];
        if ((unsigned)k < (unsigned)K) {
          const double prod = lam[k] * (double)vl[j * D + t];
          acc = acc - prod;
        }
      }
      pt[j] = acc;
    }
    // ---- ranks by (p~ desc, index asc), packed permutation ----
    int rk[EM];
    #pragma unroll
    for (int j = 0; j < EM; ++j) rk[j] = 0;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      #pragma unroll
      for (int jj = j + 1; jj < EM; ++jj) {
        if (jj < M) {
          if (pt[jj] > pt[j]) rk[j]++; else rk[jj]++;
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
    // ---- greedy over the ranked items ----
    uint64_t S = 0;
    {
      uint64_t blocked = 0;
      for (int r = 0; r < M; ++r) {
        const int j = (int)((perm >> (4 * r)) & 15);
        const uint64_t bit = 1ull << j;
        if ((pos & bit) && !(blocked & bit)) {
          S |= bit;
          for (int l = 0; l < L; ++l) {
            const uint64_t m = tmask[l];
            if ((m & bit) && popc64(S & m) >= tcap[l]) blocked |= m;
          }
        }
      }
    }
    // ---- statistics: profit, group dual value, consumption ----
    double Pi = 0.0, Gi = 0.0;
    #pragma unroll
    for (int j = 0; j < EM; ++j) {
      if (S >> j & 1) { Pi = Pi + (double)pv[j]; Gi = Gi + pt[j]; }
    }
    if (a.x_out && act) {
      uint8_t *xo = a.x_out + (u0 + lane) * M;
      for (int j = 0; j < M; ++j) xo[j] = (uint8_t)(S >> j & 1);
    }
    if (a.want_stats) {
      const double sP = wave_sum(Pi), sG = wave_sum(Gi);
      if (lane == 0) {
        wacc[wv * (K + 2) + K] = wacc[wv * (K + 2) + K] + sG;
        wacc[wv * (K + 2) + K + 1] = wacc[wv * (K + 2) + K + 1] + sP;
      }
      // consumption, 8 knapsacks at a time through per-lane rows in the region
      double *rows = (double *)wreg;   // [8][64]
      for (int c0 = 0; c0 < K; c0 += 8) {
        #pragma unroll
        for (int q = 0; q < 8; ++q) rows[q * 64 + lane] = 0.0;
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          if (S >> j & 1) {
            #pragma unroll
            for (int t = 0; t < D; ++t) {
              const int q = cl[j * D + t] - c0;
              if ((unsigned)q < 8u) rows[q * 64 + lane] = rows[q * 64 + lane] + (double)vl[j * D + t];
            }
          }
        }
        const int nq = K - c0 < 8 ? K - c0 : 8;
        for (int q = 0; q < nq; ++q) {
          const double s = wave_sum(rows[q * 64 + lane]);
          if (lane == 0) wacc[wv * (K + 2) + c0 + q] = wacc[wv * (K + 2) + c0 + q] + s;
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
    if (SCD) {
      // per-lane scratch: p~ copy [EM][64], costs of the walked knapsack [EM][64],
      // moving-item masks per knapsack [K][64]
      double *ptl = (double *)wreg;
      float *bkl = (float *)(wreg + (size_t)EM * 64 * 8);
      uint16_t *mskl = (uint16_t *)(wreg + (size_t)EM * 64 * 12);
      #pragma unroll
      for (int j = 0; j < EM; ++j) if (j < M) ptl[j * 64 + lane] = pt[j];
      for (int k = 0; k < K; ++k) mskl[k * 64 + lane] = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        #pragma unroll
        for (int t = 0; t < D; ++t) {
          const int k = cl[j * D + t];
          if ((unsigned)k < (unsigned)K) mskl[k * 64 + lane] = (uint16_t)(mskl[k * 64 + lane] | (1u << j));
        }
      }
      // threshold element of every item against the greedy solution of the
      // other items (valid when it is the only item that moves with lambda_k)
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
      // one event per (item, knapsack) that moves alone; queue the others
      uint64_t pending = 0;
      #pragma unroll
      for (int j = 0; j < EM; ++j) {
        #pragma unroll
        for (int t = 0; t < D; ++t) {
          const int k = cl[j * D + t];
          if (!act || (unsigned)k >= (unsigned)K) continue;
          const int mode = kmode[k];
          if (!(mode == KS_EXP || mode == KS_EMIT_BUCKET || mode == KS_HULL_BUCKET ||
                mode == KS_REFINE || mode == KS_EMIT_RANGE))
            continue;
          const uint32_t A = mskl[k * 64 + lane];
          if (A != (1u << j)) {
            if (j == __ffs((int)A) - 1) pending |= 1ull << k;
            continue;
          }
          const double lk = lam[k];
          const double bo_d = (double)vl[j * D + t];
          const double add_o = lk * bo_d;
          const double co = pt[j] + add_o;
          double best = 0.0;
          if (zlev >> j & 1) {
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
        }
      }
      // knapsacks moving several items: exact walk from above every breakpoint
      while (pending) {
        const int k = __ffsll((long long)pending) - 1;
        pending &= pending - 1;
        const int mode = kmode[k];
        const uint64_t A = mskl[k * 64 + lane];
        #pragma unroll
        for (int j = 0; j < EM; ++j) {
          #pragma unroll
          for (int t = 0; t < D; ++t)
            if (cl[j * D + t] == k) bkl[j * 64 + lane] = vl[j * D + t];
        }
        const double lk = lam[k];
        // start: only horizontal positive lines, in p~ order
        uint64_t Sw = 0;
        {
          uint64_t blocked = 0;
          const uint64_t elig = pos & ~A;
          for (int r = 0; r < M; ++r) {
            const int j = (int)((perm >> (4 * r)) & 15);
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
        const int maxev = M * M + M + 8;
        for (int ev = 0;; ++ev) {
          if (ev >= maxev) { atomicAdd(a.err, 1ull); break; }
          double best = 0.0;
          int bo = -1, bs = -1;
          uint64_t cand = A & ~Sw;
          while (cand) {
            const int o = __ffsll((long long)cand) - 1;
            cand &= cand - 1;
            const double bo_d = (double)bkl[o * 64 + lane];
            const double add_o = lk * bo_d;
            const double co = ptl[o * 64 + lane] + add_o;
            uint64_t circ = 0;
            bool tight = false;
            for (int l = 0; l < L; ++l) {
              const uint64_t m = tmask[l];
              if ((m >> o & 1) && popc64(Sw & m) >= tcap[l]) { circ = Sw & m; tight = true; break; }
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
                const double bs_d = (A >> s & 1) ? (double)bkl[s * 64 + lane] : 0.0;
                if (bs_d < bo_d) {
                  const double add_s = lk * bs_d;
                  const double cs = ptl[s * 64 + lane] + add_s;
                  const double num = co - cs;
                  const double den = bo_d - bs_d;
                  const double val = num / den;
                  if (val > best) { best = val; bo = o; bs = s; }
                }
              }
            }
          }
          if (bo < 0) break;
          const double bo_d = (double)bkl[bo * 64 + lane];
          const double bsv = (bs >= 0 && (A >> bs & 1)) ? (double)bkl[bs * 64 + lane] : 0.0;
          const double v2 = bs >= 0 ? bo_d - bsv : bo_d;
          Sw = (Sw | (1ull << bo)) & ~(bs >= 0 ? (1ull << bs) : 0ull);
          record_event(a, kst[k], k, best, v2, mode, hs, hc, hmin, hmax, kcnt, kovf, nstage, blockIdx.x);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  if (a.want_stats) {
    for (int c = tid; c < K + 2; c += ENT) {
      double s = 0.0;
      for (int w = 0; w < EW; ++w) s = s + wacc[w * (K + 2) + c];
      a.partials[(size_t)blockIdx.x * (K + 2) + c] = s;
    }
  }
  if (SCD) publish_block(a, K, hs, hc, hmin, hmax, kcnt, kpos, kovf, nstage, tid, ENT, blockIdx.x);
}

size_t kp_ell_lds_bytes(int M, int K, int D, int L, bool scd, int *region_out) {
  auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  size_t region = (size_t)64 * M * 4 + (size_t)64 * M * D * 8;        // staged tile
  region = region > 4096 ? region : 4096;                               // consumption rows
  if (scd) {
    const size_t need = (size_t)EM * 64 * 12 + (size_t)K * 64 * 2;     // p~, costs, masks
    region = region > need ? region : need;
  }
  region = r16(region);
  size_t s = r16((size_t)K * 8) + r16((size_t)L * 8 + 8) + r16((size_t)L * 4 + 4) +
             r16((size_t)EW * (K + 2) * 8);
  if (scd)
    s += r16((size_t)K * sizeof(KState)) + r16((size_t)K * KP_NB * 8) + r16((size_t)K * KP_NB * 4) +
         4 * r16((size_t)K * 4) + 2 * r16((size_t)K * 8) + r16(16);
  s += (size_t)EW * region;
  if (region_out) *region_out = (int)region;
  return s;
}

hipError_t kp_launch_ell(const SweepArgs &a, int D, int grid, bool scd, hipStream_t stream) {
  EllGeom g;
  g.M = a.pr.M;
  g.K = a.pr.K;
  g.pad = 0;
  const size_t lds = kp_ell_lds_bytes(g.M, g.K, D, a.tree.L, scd, &g.region);
  const void *fn = D == 1 ? (scd ? (const void *)k_ell<1, true> : (const void *)k_ell<1, false>)
                          : (scd ? (const void *)k_ell<2, true> : (const void *)k_ell<2, false>);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (D == 1) {
    if (scd) hipLaunchKernelGGL((k_ell<1, true>), dim3(grid), dim3(ENT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_ell<1, false>), dim3(grid), dim3(ENT), lds, stream, a, g);
  } else {
    if (scd) hipLaunchKernelGGL((k_ell<2, true>), dim3(grid), dim3(ENT), lds, stream, a, g);
    else hipLaunchKernelGGL((k_ell<2, false>), dim3(grid), dim3(ENT), lds, stream, a, g);
  }
  return hipGetLastError();
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
