// Shared host/device definitions of the gfx950 sweep library.
#pragma once
#include <stdint.h>

#define KP_MAX_M 64
#define KP_MAX_NODES 128
#define KP_NB 64               // histogram bins per knapsack per pass
#define KP_MAX_K_SCD 64        // per-block LDS histograms bound K for the SCD calls
#define KP_CENTRAL_W 2         // exponential buckets |id| <= W are emitted in the first pass
#define KP_SORT_MAX 4096       // candidates sorted in LDS by the selection kernel
#define KP_PROBE_USERS 4096   // users sampled by the dense window pass's probe
#define KP_WIN_MULT 1.25       // window half-width around lambda_k^t, in units of the last step
#define KP_WIN_MAX_REL 0.03125 // windows wider than this fraction of lambda_k^t are not tried
#define KP_LIST_CHUNK 256u     // list slots a wave reserves at a time in the window pass
#define KP_LIST_HOLE 0xFFFFFFFFu  // unused list slot
#define KP_SEL_MAX 4           // the uniform-row kernel gathers the selected entries when at most this many items can be selected

// An exact, order-free sum of the threshold search: hi counts units of
// 2^-24 and lo units of 2^-56, so the value is hi 2^-24 + lo 2^-56.  Terms on
// the 2^-56 grid (fp32 costs of at least 2^-33, their differences and sums
// of a few of them) add exactly as integers, in any order; terms off that
// grid round their last part to the nearest unit, the same way in every run.
struct XSum {
  long long hi, lo;
};

// Laminar local constraints after pruning: only sets that can bind
// (C_l < |S_l|), duplicates merged with the smaller cap, ordered subsets
// first (size ascending, then first item).
struct TreeDev {
  int L;
  int pad;
  uint64_t mask[KP_MAX_NODES];
  int cap[KP_MAX_NODES];
};

struct TileGeom {
  int U;            // users per tile
  int M, K;
  int aligned;      // dense costs: 16-byte aligned base and U*M*K % 4 == 0
};

struct ProbDev {
  int64_t N;
  int M, K, fmt, pad;
  const float *p;
  const float *b;
  const int64_t *rowptr;
  const int32_t *col;
  const float *val;
};

// Per-knapsack state of the threshold search of one SCD iteration.
enum {
  KS_DONE = 0,
  KS_EXP = 1,          // first pass: exponential-bucket histogram + central emission
  KS_EMIT_BUCKET = 2,  // emit the events of exponential bucket bstar (+ their key hull)
  KS_HULL_BUCKET = 3,  // only the key hull of bucket bstar (too many events to emit)
  KS_REFINE = 4,       // linear key bins over [klo, khi]
  KS_EMIT_RANGE = 5,   // emit the events with key in [klo, khi]
  KS_SELECT_BUCKET = 6,// emitted events of bucket bstar are complete: select
  KS_SELECT_RANGE = 7, // emitted events of [klo, khi] are complete: select
  KS_WINDOW = 8        // first pass around lambda_k^t: users whose greedy set stays optimal over
                       // [wlo, whi] are only checked; the others emit the breakpoints inside it
                       // and report how their consumption just above whi differs from x(lambda^t)
};

#define KS_FLAG_WINDOW 1u  // the key range of KS_SELECT_RANGE is a window: the threshold may lie outside
#define KS_FLAG_INTERP 2u  // approximate reduce: interpolate inside the bucket that holds the threshold

struct KState {
  int mode;
  int bstar;           // exponential bucket id (-31..31) for the bucket modes
  int shift;           // key-bin shift for KS_REFINE
  int overflow;        // emission exceeded the buffer
  uint32_t n_emit;     // emitted events (atomic)
  uint32_t flags;      // KS_FLAG_*
  double center;       // lambda_k^t
  double delta;        // central bucket half-width (a power of two)
  XSum fab;            // sum of increments strictly above the current target
  double result;       // lambda_k^{t+1} once mode == KS_DONE
  uint64_t klo, khi;   // inclusive key range
  uint64_t hull_lo, hull_hi;  // atomics: key hull of the bucket's events
  double wlo, whi;     // KS_WINDOW: breakpoints with wlo <= v1 <= whi are emitted (wlo may be 0)
  double hw;           // KS_WINDOW: half-width h (whi = center + h, wlo = max(center - h, 0))
  uint64_t eoff;       // batched: this knapsack's emission buffer (elements from the base), when ecap > 0
  uint32_t ecap;       // batched: its capacity (0: the uniform capacity of the call)
  uint32_t pad2;
  XSum corr;           // KS_WINDOW: sum over users of C_ik(whi+) - v_ik(x(lambda^t))
};

// The post-processing's per-user pass (Sec. 5.4): every candidate (a user
// whose selection consumes a violated knapsack) gets the bin of its group dual
// value among nb bins cut by the splitters, and its costs on the violated
// knapsacks are added into the bin's exact sums.
struct FixBins {
  uint8_t *bin;            // [N] bin per user (0xFF: not a candidate)
  const int *kv;           // [K] slot of a violated knapsack, or -1
  const uint64_t *split;   // [nb - 1] ascending splitter keys
  XSum *hsum;              // [nb][nv] exact consumption per bin and slot
  uint32_t *hcnt;          // [nb] candidates per bin
  int nb, nv;
};

struct SweepArgs {
  ProbDev pr;
  TreeDev tree;
  const double *lam;       // [K]
  int64_t ntiles;
  // statistics (first pass only)
  int want_stats;
  int no_hist;             // SCD: no knapsack bins events (no EXP / REFINE mode): no histograms in LDS
  double *partials;        // [gridDim.x][K + 2]
  uint8_t *x_out;          // [N*M] or null
  // SCD
  KState *st;              // [K]
  XSum *hist_sum;          // [K][KP_NB]
  uint32_t *hist_cnt;      // [K][KP_NB]
  double *emit_v1;         // [K][emit_cap]
  double *emit_v2;
  uint32_t emit_cap;
  // per-block staging regions of emitted events (one global reservation per
  // (block, k) at the end of the kernel instead of one atomic per event)
  double *stage_v1;        // [gridDim.x][stage_cap]
  double *stage_v2;
  uint16_t *stage_k;
  uint32_t stage_cap;
  int pass;
  unsigned long long *err; // walk-limit counter
  // post-processing bins (uniform-row kernel, evaluation only; fx.bin null otherwise)
  FixBins fx;
  // window pass split in two kernels: users listed by the first
  unsigned int *flist;     // [fcap] user indices
  unsigned int *fcount;    // [0] reserved list slots (atomic; may exceed fcap), [1] listed users
  unsigned int fcap;
  // Alg.5 map (uniform-row kernel, one entry per item row): Q of the single
  // top-Q set, for users whose item j consumes only knapsack j (M = K); 0 = off
  int alg5_q;
};

// Device-side split of a batched plan's later pass among the instances still
// searching (k_plan_resplit): the tables it reads, the descriptors it writes.
struct ResplitArgs {
  const int *order;          // [n] instance at each position of the block layout
  const int *active;         // [n] instance still searching (by instance)
  const int64_t *ntiles;     // [n] tiles of every instance
  const double *pairs;       // [n] users x knapsacks of every instance
  const SweepArgs *hd;       // [n] later-pass descriptors (by instance)
  const TileGeom *hg;        // [n] tile geometry (by instance)
  int n, gmax;
  uint32_t cap_min, cap_max; // staged events per block: bounds
  size_t stage_total;        // staged events of the whole launch
  double *s1, *s2;           // staging areas of the launch
  uint16_t *sk;
  SweepArgs *rd;             // [n] out: descriptors of the open instances
  TileGeom *rg;              // [n] out
  int *rboff;                // [n + 1] out: first block of every open instance
  int *ctl;                  // [0] out: open instances, [1] passes with work (cleared when reset),
                             // [2] staging overflow flag
  int reset;                 // first later pass of the iteration: clear ctl[1]
};
