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


// ---- exact sums (XSum) ----
// x = sign (hi 2^-24 + lo 2^-56) with hi = floor(|x| 2^24) and lo the rest in
// units of 2^-56 (|x| < 2^39): s - floor(s) is exact for s >= 0, and the
// scalings by powers of two are exact, so lo is an integer on the grid.
__device__ __forceinline__ void xs_parts(double x, long long &h, long long &l) {
  const double s = fabs(x) * 0x1p24;
  const double f = floor(s);
  const double r = (s - f) * 0x1p32;
  long long hi = (long long)f;
  long long lo = (long long)rint(r);
  if (lo == 0x100000000ll) { lo = 0; hi += 1; }
  if (x < 0.0) { hi = -hi; lo = -lo; }
  h = hi;
  l = lo;
}
__device__ __forceinline__ XSum xs_of(double x) {
  XSum r;
  xs_parts(x, r.hi, r.lo);
  return r;
}
__device__ __forceinline__ XSum xs_plus(XSum a, XSum b) {
  XSum r;
  r.hi = a.hi + b.hi;
  r.lo = a.lo + b.lo;
  return r;
}
__device__ __forceinline__ XSum xs_minus(const XSum &a, const XSum &b) {
  XSum r;
  r.hi = a.hi - b.hi;
  r.lo = a.lo - b.lo;
  return r;
}
__device__ __forceinline__ void xs_add(XSum &a, double x) { a = xs_plus(a, xs_of(x)); }
__device__ __forceinline__ XSum xs_zero() {
  XSum r;
  r.hi = 0;
  r.lo = 0;
  return r;
}
__device__ __forceinline__ bool xs_nonzero(const XSum &a) { return a.hi != 0 || a.lo != 0; }
// Integer adds: the same total whatever order the lanes and blocks add in.
__device__ __forceinline__ void xs_atomic_add_sum(XSum *dst, const XSum &v) {
  if (v.hi) atomicAdd((unsigned long long *)&dst->hi, (unsigned long long)v.hi);
  if (v.lo) atomicAdd((unsigned long long *)&dst->lo, (unsigned long long)v.lo);
}
__device__ __forceinline__ void xs_atomic_add(XSum *dst, double x) { xs_atomic_add_sum(dst, xs_of(x)); }
// The nearest doubles to the parts, added (exact when the total needs no
// more than 53 bits, e.g. on the 2^-24 grid below 2^29).
__device__ __forceinline__ double xs_to_double(const XSum &a) {
  const long long H = a.hi + (a.lo >> 32);
  const long long L = a.lo & 0xFFFFFFFFll;
  const double h = (double)H * 0x1p-24;
  const double l = (double)L * 0x1p-56;
  return h + l;
}
// a > B exactly, for B >= 0 (B's own bits below 2^-56 are kept in the
// comparison).
__device__ __forceinline__ bool xs_gt(const XSum &a, double B) {
  if (!(B < 0x1p38)) return xs_to_double(a) > B;   // outside the exact range (budgets below 2^38)
  const long long H = a.hi + (a.lo >> 32);
  const long long L = a.lo & 0xFFFFFFFFll;
  const double sB = B * 0x1p24;
  const double fB = floor(sB);
  const double rB = (sB - fB) * 0x1p32;
  const long long HB = (long long)fB;
  return H > HB || (H == HB && (double)L > rB);
}

// Bin of a post-processing key: the number of the nb - 1 ascending
// splitters below it.
__device__ __forceinline__ int fx_bin_of(const uint64_t *split, int nb, uint64_t key) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (split[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Breakpoint arithmetic of the walks.  For lines z_a = c_a - lambda b_a and
// z_b = c_b - lambda b_b with b_a > b_b, the crossing is
// fl(fl(c_a - c_b) / fl(b_a - b_b)) and line a ranks above line b for lambda
// below it; a line's zero crossing is fl(c_a / b_a).  cr_gt / cr_ge decide
// fl(num / den) > t and >= t for den > 0 from exact fma residual signs and
// divide only when the quotient lies within one ulp of t, so that the
// decisions agree with the divided crossings bit for bit.
__device__ __forceinline__ bool cr_gt(double num, double den, double t) {   // t >= 0
  const double r = fma(-t, den, num);            // sign of num - t*den, exact
  if (!(r > 0.0)) return false;                  // quotient <= t
  const double up = kdbl(dkey(t) + 1);           // next double above t
  const double r2 = fma(-up, den, num);
  if (r2 >= 0.0) return true;                    // quotient >= up
  return num / den > t;
}
__device__ __forceinline__ bool cr_ge(double num, double den, double t) {   // t > 0
  const double r = fma(-t, den, num);
  if (r >= 0.0) return true;                     // quotient >= t
  const double dn = kdbl(dkey(t) - 1);           // next double below t
  const double r2 = fma(-dn, den, num);
  if (!(r2 > 0.0)) return false;                 // quotient <= dn
  return num / den >= t;
}
// Is the line (c, b), b >= 0, positive just above t (side > 0) or just below
// t (side < 0, t > 0)?
__device__ __forceinline__ bool line_pos(double c, double b, double t, int side) {
  if (b == 0.0) return c > 0.0;
  return side > 0 ? cr_gt(c, b, t) : cr_ge(c, b, t);
}
// Does line o rank above line s just above / below t?  Parallel lines keep
// the order (c desc, index asc).
__device__ __forceinline__ bool line_beats(double co, double bo, int o, double cs, double bs, int s,
                                           double t, int side) {
  if (bo == bs) return co > cs || (co == cs && o < s);
  if (bo > bs) {
    const double num = co - cs, den = bo - bs;
    return side > 0 ? cr_gt(num, den, t) : cr_ge(num, den, t);
  }
  const double num = cs - co, den = bs - bo;
  return side > 0 ? !cr_gt(num, den, t) : !cr_ge(num, den, t);
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
                                             double v2, int mode, XSum *hs, uint32_t *hc,
                                             unsigned long long *hmin, unsigned long long *hmax,
                                             uint32_t *kcnt, uint32_t *kovf, uint32_t *nstage,
                                             int bid) {
  const uint64_t key = dkey(best);
  bool emit = false;
  if (mode == KS_EXP && hs) {
    const int id = exp_bucket(best, ks.center, ks.delta);
    xs_atomic_add(&hs[k * KP_NB + 32 + id], v2);
    atomicAdd(&hc[k * KP_NB + 32 + id], 1u);
    emit = (id >= -KP_CENTRAL_W && id <= KP_CENTRAL_W);
  } else if (mode == KS_EMIT_BUCKET || mode == KS_HULL_BUCKET) {
    if (exp_bucket(best, ks.center, ks.delta) == ks.bstar) {
      atomicMin(&hmin[k], (unsigned long long)key);
      atomicMax(&hmax[k], (unsigned long long)key);
      emit = (mode == KS_EMIT_BUCKET);
    }
  } else if (mode == KS_REFINE) {
    if (hs && key >= ks.klo && key <= ks.khi) {
      const int bin = (int)((key - ks.klo) >> ks.shift);
      xs_atomic_add(&hs[k * KP_NB + bin], v2);
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

// Does a knapsack in search state m need another pass over its users?
__device__ __forceinline__ bool walk_mode(int m) {
  return m == KS_EXP || m == KS_EMIT_BUCKET || m == KS_HULL_BUCKET || m == KS_REFINE ||
         m == KS_EMIT_RANGE || m == KS_WINDOW;
}

// End of a sweep block: add its histograms to the global ones, reserve space
// for its staged events with one atomic per knapsack and copy them there.
// Every thread of the block calls this.
__device__ __forceinline__ void publish_block(const SweepArgs &a, int K, XSum *hs, uint32_t *hc,
                                              unsigned long long *hmin, unsigned long long *hmax,
                                              uint32_t *kcnt, uint32_t *kpos, uint32_t *kovf,
                                              uint32_t *nstage, int tid, int nthreads, int bid,
                                              const XSum *kcorr = nullptr) {
  for (int t = tid; hc && t < K * KP_NB; t += nthreads) {
    if (hc[t]) {
      xs_atomic_add_sum(&a.hist_sum[t], hs[t]);
      atomicAdd(&a.hist_cnt[t], hc[t]);
    }
  }
  for (int k = tid; k < K; k += nthreads) {
    if (kcnt[k]) kpos[k] = atomicAdd(&a.st[k].n_emit, kcnt[k]);
    if (kovf[k]) atomicOr(&a.st[k].overflow, 1);
    if (kcorr && xs_nonzero(kcorr[k])) xs_atomic_add_sum(&a.st[k].corr, kcorr[k]);
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

// Is S, the greedy set at lambda^t, still the greedy solution of the lines
// z_j = c_j - lambda_k b_jk just above t (side > 0) or just below t
// (side < 0)?  Only relations that involve an item moving with k (A) can
// differ from those at lambda^t.  S is the greedy solution iff its members
// stay positive and every positive non-member closes a circuit with S (the
// members of the innermost full set containing it) and ranks below every
// member of it.  line(j, c, b) gives item j's line (b = 0 outside A); Bpos:
// the items with p~ > 0 outside S.
template <class LINE>
__device__ __forceinline__ bool window_keeps(uint64_t S, uint64_t A, uint64_t Bpos, LINE line,
                                             const uint64_t *tmask, const int *tcap, int L, double t,
                                             int side) {
  auto circuit = [&](int o) -> uint64_t {
    for (int l = 0; l < L; ++l) {
      const uint64_t m = tmask[l];
      if ((m >> o & 1) && popc64(S & m) >= tcap[l]) return S & m;
    }
    return 0;
  };
  for (uint64_t m = S & A; m; m &= m - 1) {
    const int s = __ffsll((long long)m) - 1;
    double c, b;
    line(s, c, b);
    if (!line_pos(c, b, t, side)) return false;
  }
  for (uint64_t m = A & ~S; m; m &= m - 1) {
    const int o = __ffsll((long long)m) - 1;
    double co, bo;
    line(o, co, bo);
    if (!line_pos(co, bo, t, side)) continue;
    uint64_t circ = circuit(o);
    if (!circ) return false;
    for (; circ; circ &= circ - 1) {
      const int s = __ffsll((long long)circ) - 1;
      double cs, bs;
      line(s, cs, bs);
      if (line_beats(co, bo, o, cs, bs, s, t, side)) return false;
    }
  }
  for (uint64_t m = Bpos & ~A; m; m &= m - 1) {
    const int o = __ffsll((long long)m) - 1;
    uint64_t circ = circuit(o) & A;
    if (!circ) continue;
    double co, bo;
    line(o, co, bo);
    for (; circ; circ &= circ - 1) {
      const int s = __ffsll((long long)circ) - 1;
      double cs, bs;
      line(s, cs, bs);
      if (line_beats(co, bo, o, cs, bs, s, t, side)) return false;
    }
  }
  return true;
}

// Window filter (one user): the smallest distance between two of its lines
// that can turn positive within h of lambda_k^t, or between such a line and
// zero, must exceed h * bmax (plus a rounding margin): lines move against
// each other by at most |b_a - b_b| <= bmax per unit of lambda_k.  gmin and
// gscale come from the user's p~ in rank order (lines below -H, H the widest
// window's bound, never turn positive).
__device__ __forceinline__ bool window_calm(double gmin, double gscale, double h, double bmax,
                                           double lk) {
  const double need = h * bmax * (1.0 + 0x1p-30) + 0x1p-36 * (1.0 + gscale + lk * bmax + h * bmax);
  return gmin > need;
}
