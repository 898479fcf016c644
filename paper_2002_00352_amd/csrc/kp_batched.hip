// Device-side split of a batched plan's later passes (the passes over the
// instances whose threshold search is still open after the first pass), so
// that a whole SCD iteration -- the first pass and a fixed number of later
// passes -- can be captured in one HIP graph and replayed without a host
// round trip between passes.
//
// The split is the host's (the plan's re-split): the open instances, in the
// block layout's order (costliest tiles first), share G blocks in proportion
// to their tiles, each at least one; every block's share of staged events
// is scaled from its share of (user, knapsack) pairs and the whole launch's
// staging area is divided among them.  One thread makes the sequential
// decisions in the host's order with the host's arithmetic (so the device
// and host splits agree), the others load the tables and copy the
// descriptors.  A pass with no open instance launches blocks that exit at
// once.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include "kp_internal.h"

#define RS_NT 1024

// LDS per position: instance, tiles, pairs, blocks, cap, staging offset
__global__ void __launch_bounds__(RS_NT) k_plan_resplit(const ResplitArgs r) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = r.n, tid = threadIdx.x;
  int *act = (int *)smem;                                       // [n] open instances in layout order
  int64_t *nt = (int64_t *)(smem + (((size_t)n * 4 + 15) & ~(size_t)15));
  double *pr = (double *)(nt + n);
  int *nb = (int *)(pr + n);
  uint32_t *cp = (uint32_t *)(nb + n);
  size_t *so = (size_t *)((unsigned char *)smem + ((((size_t)n * 4 + 15) & ~(size_t)15) +
                                                   (size_t)n * 16 + (((size_t)n * 8 + 15) & ~(size_t)15)));
  __shared__ int na_s;
  // every position: its instance when that instance sweeps, else -1
  for (int i = tid; i < n; i += RS_NT) {
    const int s = r.order[i];
    const bool open = r.active[s] != 0 && r.ntiles[s] > 0;
    act[i] = open ? s : -1;
    nt[i] = r.ntiles[s];
    pr[i] = r.pairs[s];
  }
  __syncthreads();
  if (tid == 0) {
    if (r.reset) r.ctl[1] = 0;
    // compact the open positions in order; the sums and the split in the
    // host's order and arithmetic
    int na = 0;
    int64_t TA = 0;
    for (int i = 0; i < n; ++i) {
      if (act[i] < 0) continue;
      act[na] = act[i];
      nt[na] = nt[i];
      pr[na] = pr[i];
      TA += nt[na];
      ++na;
    }
    r.rboff[0] = 0;
    if (na > 0) {
      const int64_t Gl = TA < (int64_t)r.gmax ? TA : (int64_t)r.gmax;
      const int G = (int)(Gl > na ? Gl : na);
      double tot = 0.0;
      for (int i = 0; i < na; ++i) {
        int64_t b = llround((double)G * nt[i] / (double)TA);
        b = b < nt[i] ? b : nt[i];
        b = b > 1 ? b : 1;
        nb[i] = (int)b;
        const double w = fmin((double)r.cap_max, fmax((double)r.cap_min, pr[i] / nb[i] / 64.0));
        pr[i] = w;   // (the pairs are not needed again)
        tot += w * nb[i];
      }
      const double scale = tot > (double)r.stage_total ? (double)r.stage_total / tot : 1.0;
      size_t off = 0;
      int blk = 0;
      for (int i = 0; i < na; ++i) {
        const uint32_t cap = (uint32_t)fmax(1.0, floor(pr[i] * scale));
        cp[i] = cap;
        so[i] = off;
        off += (size_t)nb[i] * cap;
        blk += nb[i];
        r.rboff[i + 1] = blk;
      }
      if (off > r.stage_total) {   // cannot happen: the caps were scaled to fit
        r.ctl[2] = 1;
        na = 0;
      } else {
        r.ctl[1] += 1;
      }
    }
    na_s = na;
    r.ctl[0] = na;
  }
  __syncthreads();
  const int na = na_s;
  for (int i = tid; i < na; i += RS_NT) {
    const int s = act[i];
    SweepArgs d = r.hd[s];
    d.stage_v1 = r.s1 + so[i];
    d.stage_v2 = r.s2 + so[i];
    d.stage_k = r.sk + so[i];
    d.stage_cap = cp[i];
    r.rd[i] = d;
    r.rg[i] = r.hg[s];
  }
}

// LDS of the split for n instances (0: too many for one block's LDS)
size_t kp_resplit_lds(int n) {
  auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
  const size_t b = r16((size_t)n * 4) + (size_t)n * 16 + r16((size_t)n * 8) + (size_t)n * 8;
  return b <= (size_t)60 * 1024 ? b : 0;
}

hipError_t kp_launch_plan_resplit(const ResplitArgs &r, hipStream_t stream) {
  const size_t lds = kp_resplit_lds(r.n);
  if (r.n < 1 || lds == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plan_resplit, dim3(1), dim3(RS_NT), lds, stream, r);
  return hipGetLastError();
}
