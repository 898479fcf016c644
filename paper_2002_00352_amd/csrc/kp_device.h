// Device helpers shared by the sweep kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "kp_internal.h"

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


// Bin or emit one breakpoint (v1, v2) of knapsack k according to its search
// mode: the first pass bins every breakpoint into exponential buckets around
// lambda_k^t and emits the central ones; later passes emit one bucket or key
// range, record a bucket's key hull, or bin a key range linearly.  Emitted
// events go to the block's staging region (published by publish_block).
__device__ __forceinline__ void record_event(const SweepArgs &a, const KState &ks, int k, double best,
                                             double v2, int mode, double *hs, uint32_t *hc,
                                             unsigned long long *hmin, unsigned long long *hmax,
                                             uint32_t *kcnt, uint32_t *kovf, uint32_t *nstage,
                                             int bid) {
  const uint64_t key = dkey(best);
  bool emit = false;
  if (mode == KS_EXP) {
    const int id = exp_bucket(best, ks.center, ks.delta);
    atomicAdd(&hs[k * KP_NB + 32 + id], v2);
    atomicAdd(&hc[k * KP_NB + 32 + id], 1u);
    emit = (id >= -KP_CENTRAL_W && id <= KP_CENTRAL_W);
  } else if (mode == KS_EMIT_BUCKET || mode == KS_HULL_BUCKET) {
    if (exp_bucket(best, ks.center, ks.delta) == ks.bstar) {
      atomicMin(&hmin[k], (unsigned long long)key);
      atomicMax(&hmax[k], (unsigned long long)key);
      emit = (mode == KS_EMIT_BUCKET);
    }
  } else if (mode == KS_REFINE) {
    if (key >= ks.klo && key <= ks.khi) {
      const int bin = (int)((key - ks.klo) >> ks.shift);
      atomicAdd(&hs[k * KP_NB + bin], v2);
      atomicAdd(&hc[k * KP_NB + bin], 1u);
    }
  } else {  // KS_EMIT_RANGE
    emit = (key >= ks.klo && key <= ks.khi);
  }
  if (emit) {
    const uint32_t slot = atomicAdd(nstage, 1u);
    if (slot < a.stage_cap) {
      const size_t e = (size_t)bid * a.stage_cap + slot;
      a.stage_v1[e] = best;
      a.stage_v2[e] = v2;
      a.stage_k[e] = (uint16_t)k;
      atomicAdd(&kcnt[k], 1u);
    } else {
      kovf[k] = 1u;
    }
  }
}

// End of a sweep block: add its histograms to the global ones, reserve space
// for its staged events with one atomic per knapsack and copy them there.
// Every thread of the block calls this.
__device__ __forceinline__ void publish_block(const SweepArgs &a, int K, double *hs, uint32_t *hc,
                                              unsigned long long *hmin, unsigned long long *hmax,
                                              uint32_t *kcnt, uint32_t *kpos, uint32_t *kovf,
                                              uint32_t *nstage, int tid, int nthreads, int bid) {
  for (int t = tid; t < K * KP_NB; t += nthreads) {
    if (hc[t]) {
      atomicAdd(&a.hist_sum[t], hs[t]);
      atomicAdd(&a.hist_cnt[t], hc[t]);
    }
  }
  for (int k = tid; k < K; k += nthreads) {
    if (kcnt[k]) kpos[k] = atomicAdd(&a.st[k].n_emit, kcnt[k]);
    if (kovf[k]) atomicOr(&a.st[k].overflow, 1);
    if (hmin[k] != ~0ull) {
      atomicMin((unsigned long long *)&a.st[k].hull_lo, hmin[k]);
      atomicMax((unsigned long long *)&a.st[k].hull_hi, hmax[k]);
    }
    kcnt[k] = 0u;
  }
  __syncthreads();
  const uint32_t ns = *nstage < a.stage_cap ? *nstage : a.stage_cap;
  for (uint32_t t = tid; t < ns; t += nthreads) {
    const size_t e = (size_t)bid * a.stage_cap + t;
    const int k = a.stage_k[e];
    const uint32_t dst = kpos[k] + atomicAdd(&kcnt[k], 1u);
    if (dst < a.emit_cap) {
      a.emit_v1[(size_t)k * a.emit_cap + dst] = a.stage_v1[e];
      a.emit_v2[(size_t)k * a.emit_cap + dst] = a.stage_v2[e];
    } else {
      atomicOr(&a.st[k].overflow, 1);
    }
  }
}
