/*
 * kp.h -- C ABI of the MI355X (gfx950) per-user subproblem sweep for the
 * Lagrangian-dual knapsack solver of "Solving Billion-Scale Knapsack Problems"
 * (Zhang, Qi, Hua, Yang, WWW'20).
 *
 * Problem (Eq.1-4, Sec. 2):  max sum_ij p_ij x_ij
 *   s.t. sum_ij b_ijk x_ij <= B_k  for every knapsack k      (global, Eq.2)
 *        sum_{j in S_l} x_ij <= C_l for every user i, set l  (local,  Eq.3)
 *        x_ij in {0,1}                                        (Eq.4)
 * with B_k, C_l > 0 and p, b >= 0, and local sets forming a laminar
 * (hierarchical) family (Sec. 2.1).
 *
 * Memory and threading rules for every call below:
 *  - Pointers marked DEV are device (HIP) pointers; HOST are host pointers.
 *    The caller owns every buffer passed in; the library keeps no pointer to
 *    caller memory after the call's work has been enqueued.
 *  - Host-side validation runs synchronously before anything is enqueued.  On
 *    any non-OK return nothing was enqueued (except KP_ERR_HIP, which reports
 *    a HIP runtime failure) and kp_last_error() gives a message.
 *  - All work is enqueued on the context's stream.  Outputs are valid once
 *    that stream reaches them.  kp_scd_sweep and kp_primal_fixup synchronise
 *    the stream internally (they read a small status word back per pass).
 *  - A context is used by one host thread at a time.  Calls that share a
 *    context serialise on its workspace.
 *  - Non-finite or negative p, b are undefined behaviour unless
 *    kp_validate_inputs reported them absent.
 */
#ifndef KP_H
#define KP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KP_OK = 0,
  KP_ERR_INVALID = -1,      /* bad sizes, NULL pointers, B_k <= 0, cap < 1, bad tree links */
  KP_ERR_NOT_LAMINAR = -2,  /* kp_tree_from_sets: two sets overlap without nesting */
  KP_ERR_NONFINITE = -3,    /* kp_validate_inputs found NaN/Inf in p or b */
  KP_ERR_NEGATIVE = -4,     /* kp_validate_inputs found a negative p or b */
  KP_ERR_UNSUPPORTED = -5,  /* outside the built limits (M > 64, K too large for SCD, ...) */
  KP_ERR_NOMEM = -6,        /* the workspace would exceed max_workspace_bytes, or hipMalloc failed */
  KP_ERR_HIP = -7,          /* a HIP runtime call failed */
  KP_ERR_INTERNAL = -8      /* an internal iteration limit was hit (reported, never silent) */
} kp_status;

enum { KP_B_DENSE = 0, KP_B_CSR = 1 };

/* One knapsack instance.  Local constraints are a forest: node l has cap[l]
   (C_l >= 1) and parent[l] (-1 for a root); S_l is every item whose ancestor
   chain from leaf_of_item[j] passes through l.  Any laminar family is such a
   forest (the containment DAG of Sec. 2.1 reduced to its covering arcs);
   kp_tree_from_sets builds one from explicit sets.  A single top-Q cap is
   {L=1, parent={-1}, cap={Q}, leaf_of_item[j]=0 for all j}.
   The local constraints are the same for every user (Eq.3 indexes S_l, C_l
   by l only). */
typedef struct {
  int64_t N;                  /* users, >= 0 */
  int32_t M;                  /* items per user, 1..64 */
  int32_t K;                  /* knapsacks (global constraints), >= 1 */
  const float *p;             /* DEV [N*M] profits, item fastest */
  int32_t b_format;           /* KP_B_DENSE or KP_B_CSR */
  const float *b;             /* DEV dense [N*M*K] costs, k fastest */
  const int64_t *b_rowptr;    /* DEV CSR [N*M+1] offsets per item row (row r = i*M + j) */
  const int32_t *b_col;       /* DEV CSR column (knapsack) ids, strictly ascending per row */
  const float *b_val;         /* DEV CSR values */
  const double *B;            /* HOST [K] budgets, each finite and > 0 */
  int32_t L;                  /* HOST number of local-constraint nodes, >= 0 */
  const int32_t *parent;      /* HOST [L], -1 = root, else a node id in [0,L) */
  const int32_t *cap;         /* HOST [L], >= 1 */
  const int32_t *leaf_of_item;/* HOST [M], innermost node containing item j, or -1 */
  int32_t b_row_nnz;          /* CSR only: 0 = general rows; D in {1, 2} = the caller declares that
                                 every item row holds exactly D stored entries, row r's at
                                 [r*D, r*D + D) (rowptr[r] == r*D).  With M <= 16 the library then
                                 runs a lean per-user kernel that never reads b_rowptr.
                                 kp_csr_row_nnz finds D; kp_validate_inputs checks a declared D.
                                 A false declaration is undefined behaviour, like an unsorted row.
                                 Must be 0 for dense costs. */
} kp_problem;

/* Message for the last non-OK status returned on this thread. */
const char *kp_last_error(void);

/* Create a context bound to a HIP stream (hipStream_t passed as void*; NULL =
   the null stream).  max_workspace_bytes caps the device workspace the
   context may allocate (0 = no cap); exceeding it returns KP_ERR_NOMEM. */
kp_status kp_create(void **ctx_out, void *hip_stream, size_t max_workspace_bytes);
/* Free the context and its workspace (synchronises its stream first). */
kp_status kp_destroy(void *ctx);
/* Rebind the context to another stream. */
kp_status kp_set_stream(void *ctx, void *hip_stream);

/* Dual evaluation at lambda (Eq.5 with Alg.2's Map and Reduce):
   every user scores its items p~_ij = p_ij - sum_k lambda_k b_ijk (FP64,
   k ascending, no FMA), solves its local integer program with Alg.1 (ties in
   p~ go to the lower item index; only p~ > 0 is selected), and the library
   reduces R_k = sum_ij b_ijk x_ij, primal P = sum_ij p_ij x_ij and
   g = sum_i sum_j p~_ij x_ij + sum_k lambda_k B_k in FP64.
   lambda: DEV [K] >= 0.  R: DEV [K].  g, primal: DEV [1].
   x: DEV [N*M] uint8 decisions, or NULL. */
kp_status kp_eval_dual(void *ctx, const kp_problem *prob, const double *lambda,
                       double *R, double *g, double *primal, uint8_t *x);

/* kp_eval_dual for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same evaluation and the same outputs, with no context and no
   workspace.  It calls no hipMalloc, hipFree or other allocating routine;
   its scratch memory (the budgets and one row of K + 2 partial sums per
   block) is a static 8 MiB device array that every GPU the library runs on
   holds until the process ends.  Work is enqueued on hip_stream (hipStream_t
   as void*, NULL = the null stream); lambda, R, g, primal (DEV, none NULL)
   and x (DEV or NULL) as in kp_eval_dual.  Every call on one GPU shares that
   GPU's scratch array, which keeps the last call's contents: calls that
   overlap on one GPU (on different streams or host threads) race, so the
   caller serialises them.  KP_ERR_UNSUPPORTED when the K + 2 partial sums of
   one block do not fit the scratch array (K above about a million); the
   grid is reduced to what fits.  Costs declared with b_row_nnz use the
   lean per-user kernel; nothing is tuned. */
kp_status kp_eval_dual_noalloc(void *hip_stream, const kp_problem *prob, const double *lambda,
                               double *R, double *g, double *primal, uint8_t *x);

/* One synchronous coordinate-descent iteration (Alg.4 with Alg.3's
   candidates): for every knapsack k, the consumption step function of every
   user as lambda_k alone moves (lines c_j - lambda_k b_ijk with
   c_j = p~_ij + lambda_k^t b_ijk), and the global threshold: lambda_out[k] = 0
   when the total increment fits in B_k, else the largest breakpoint at which
   the cumulative increment from above exceeds B_k.  All k are updated from
   the same lambda_in.  R, g, primal (DEV, may be NULL) are the statistics at
   lambda_in.  lambda_in and lambda_out: DEV [K]; they may alias.
   Synchronises the context stream. */
kp_status kp_scd_sweep(void *ctx, const kp_problem *prob, const double *lambda_in,
                       double *lambda_out, double *R, double *g, double *primal);

/* Same, updating only the coordinates with kmask[k] != 0 (HOST [K]); the
   others are copied from lambda_in.  Cyclic CD passes one coordinate per
   call, block CD a block (Sec. 4.3.2). */
kp_status kp_scd_sweep_masked(void *ctx, const kp_problem *prob, const double *lambda_in,
                              double *lambda_out, const uint8_t *kmask, double *R, double *g,
                              double *primal);

/* One dual-descent step (Eq.14, Alg.2):
   lambda_k <- max(lambda_k + alpha (R_k - B_k), 0), with R, g, primal (DEV,
   may be NULL) the statistics at the old lambda.  lambda_inout: DEV [K]. */
kp_status kp_dd_step(void *ctx, const kp_problem *prob, double alpha, double *lambda_inout,
                     double *R, double *g, double *primal);

/* Gradient of the dual for the autograd backward: grad_lambda[k] =
   grad_out[0] * (B_k - R[k]) (g is convex with subgradient B - R, Sec. 4.1).
   R: DEV [K] from kp_eval_dual at the same lambda.  grad_out: DEV [1].
   grad_lambda: DEV [K]. */
kp_status kp_dual_backward(void *ctx, const kp_problem *prob, const double *R,
                           const double *grad_out, double *grad_lambda);

/* Post-processing for feasibility (Sec. 5.4) at lambda: users that consume
   at least one knapsack violated by x(lambda) are ordered by their group dual
   value p~_i = sum_j p_ij x_ij - sum_k lambda_k sum_j b_ijk x_ij ascending
   (ties: lower user index first) and the shortest prefix of that order whose
   removal brings every violated knapsack within budget is reset to x_i = 0.
   A violated knapsack counts as within budget once its total consumption
   minus the reset users' consumption, both summed exactly, is at most B_k
   (so the reset set does not depend on a summation order; exact for costs
   that are multiples of 2^-56 with totals below 2^38).  R_out = R(x(lambda))
   minus the removed consumption; primal_out likewise.  N < 2^32.
   Outputs (DEV): x_out [N*M] (may be NULL), primal_out [1], R_out [K],
   n_reset_out [1] (int64).  Synchronises the context stream (three times). */
kp_status kp_primal_fixup(void *ctx, const kp_problem *prob, const double *lambda,
                          uint8_t *x_out, double *primal_out, double *R_out,
                          int64_t *n_reset_out);

/* Batched SCD: one iteration for n independent instances (probs: HOST [n]),
   lambda_in[s] / lambda_out[s]: DEV [K_s] per instance (HOST arrays of n DEV
   pointers).  stats: DEV [sum_s (K_s + 2)] -- per instance R[K_s], g, primal at
   lambda_in, concatenated in instance order (may be NULL).
   Synchronises the context stream. */
kp_status kp_scd_sweep_batched(void *ctx, const kp_problem *probs, int32_t n,
                               const double *const *lambda_in, double *const *lambda_out,
                               double *stats);

/* Batched plan for repeated iterations: validates the instances and builds
   the device tables once for two multiplier buffers per instance, lam_a[s]
   and lam_b[s] (HOST arrays of n DEV pointers, each [K_s]).
   kp_batched_step(plan, dir, stats, use_graph) runs one SCD iteration from
   lam_a into lam_b (dir 0) or from lam_b into lam_a (dir 1); stats as in
   kp_scd_sweep_batched (DEV, may be NULL).  With use_graph != 0 the
   iteration (init, sweep, statistics, threshold search, update) is captured
   once per direction as a HIP graph and replayed: the first pass and five
   later passes, each later pass splitting the blocks among the instances
   whose threshold is still open on the device (a pass with none open does
   no work; plans of more than 1706 instances capture the first pass
   only); passes beyond those run eagerly, split on the host.  With
   use_graph == 0 every pass is launched eagerly.  The plan borrows the
   context's stream and owns its workspace;
   the caller keeps the instances' buffers alive until kp_batched_destroy.
   Synchronises the stream at the end of every step. */
kp_status kp_batched_create(void *ctx, const kp_problem *probs, int32_t n,
                            const double *const *lam_a, double *const *lam_b, void **plan_out);
kp_status kp_batched_step(void *plan, int32_t dir, double *stats, int32_t use_graph);
kp_status kp_batched_destroy(void *plan);
/* Launch shape of a batched plan's first pass: blocks, LDS bytes per block,
   and the smallest and largest users per tile over its instances.  HOST
   outputs, each may be NULL. */
kp_status kp_batched_shape(void *plan, int32_t *blocks, int32_t *lds_bytes, int32_t *min_users_per_tile,
                           int32_t *max_users_per_tile);

/* Pre-solving by sampling (Sec. 5.3): SCD iterations on the sub-instance of
   the sampled users, with every budget scaled by n/N (B_k * (n / N) in
   FP64), from lambda_inout until the multipliers repeat or max_iter sweeps;
   the result (a starting point lambda^0 for the full instance) is written
   back to lambda_inout (DEV [K]).  users: HOST [n] distinct indices in
   [0, N), drawn by the caller.  iterations_out (HOST, may be NULL): sweeps
   run.  Allocates and frees one device buffer for the sample; synchronises
   the context stream; resets the context's window hints. */
kp_status kp_presolve(void *ctx, const kp_problem *prob, const int64_t *users, int64_t n,
                      int32_t max_iter, double *lambda_inout, int32_t *iterations_out);

/* Optional full pass over p and b: KP_ERR_NONFINITE / KP_ERR_NEGATIVE if any
   value is NaN/Inf or negative, KP_OK otherwise (a CSR column outside [0,K) or
   not ascending, or a declared b_row_nnz that some row does not meet, is
   KP_ERR_INVALID).  Synchronises the context stream. */
kp_status kp_validate_inputs(void *ctx, const kp_problem *prob);

/* Host helper: explicit local sets {S_l, C_l} (set_offsets HOST [L+1] into
   set_items HOST, caps HOST [L]) to the forest form above.  Identical sets are
   merged keeping the smaller cap; KP_ERR_NOT_LAMINAR if two sets overlap
   without one containing the other (Definition in Sec. 2.1).  Outputs (HOST,
   sized L and M by the caller): L_out, parent_out, cap_out, leaf_of_item_out. */
kp_status kp_tree_from_sets(int32_t M, int32_t L, const int32_t *set_offsets,
                            const int32_t *set_items, const int32_t *caps, int32_t *L_out,
                            int32_t *parent_out, int32_t *cap_out,
                            int32_t *leaf_of_item_out);

/* Optional timing of the sweep kernel: when on, every sweep pass made
   through this context (the uniform-row kernel's window pass: both of its
   launches) is bracketed by HIP events on the context's stream, and so is
   every whole iteration of a batched plan created on it.  kp_get_timing
   waits for them and returns the summed time (ms), the number of timed
   intervals and their algorithmic input bytes: every byte of p and b in the
   layout above once per interval (dense 4*N*M*(1+K); CSR
   4*N*M + 8*(N*M+1) + 8*nnz, rowptr included even where the lean kernel does
   not read it; a batched iteration: the sum over its instances).
   kp_get_batched_passes: the sweep passes inside the timed batched
   iterations.  kp_set_timing resets the totals. */
kp_status kp_set_timing(void *ctx, int32_t on);
kp_status kp_get_timing(void *ctx, double *sweep_ms_total, int64_t *sweep_launches,
                        double *sweep_bytes_total);
kp_status kp_get_batched_passes(void *ctx, int64_t *passes);

/* Streaming-read probe (the roofline's measured ceiling): reads bytes (a
   multiple of 16) from the 16-byte aligned DEV buffer src once with
   nontemporal 16-byte loads (the cache policy of the sweep kernels' staging),
   on hip_stream, and XORs a checksum into *out (DEV [1], not cleared: the
   caller zeroes it): with (x, y, z, w) the XOR of all 16-byte words as four
   32-bit words, ((x ^ z) << 32) | (y ^ w).  Time it with events on the
   same stream.  KP_ERR_INVALID for NULL pointers, a misaligned src or bytes
   not a multiple of 16. */
kp_status kp_stream_read(void *hip_stream, const void *src, size_t bytes, uint64_t *out);

/* Tile-size override for one problem shape (M, K, b_format): users per tile
   and grid size (blocks) used by every later call on this context for that
   shape; 0 keeps the built-in choice, (0, 0) removes the override.  The
   general kernel takes both (users per tile capped by its LDS); the
   uniform-row kernel takes the grid only (one lane per user, 64 users per
   wave); dense evaluations with M <= 16 and K <= 16 run the lane-per-user
   dense kernel unless the override names users per tile (then the general
   kernel runs with them), and take its grid; batched plans created later
   take the users per tile of each instance's shape.  Grids are capped at the blocks that can be resident.
   x, lambda and R do not depend on these values; g and P are FP64 sums whose
   grouping follows the grid, so their last bits may.  Used by the autotuner. */
kp_status kp_set_tuning(void *ctx, int32_t M, int32_t K, int32_t b_format, int32_t users_per_tile,
                        int32_t grid);
/* Shape of the last sweep launch made through this context: kernel (0 the
   general kernel, 1 the uniform-row kernel, 2 the lane-per-user evaluation
   of dense costs, 3 its SCD window pass, -1 none yet), users per tile and
   blocks launched.  HOST outputs, each may be NULL. */
kp_status kp_get_launch_shape(void *ctx, int32_t *kernel, int32_t *users_per_tile, int32_t *grid);
/* Tuning of batched plans created later on this context: LDS bytes per block
   of the batched launch (instances with long rows take fewer users per tile
   to fit it; 0 = 40 KB) and blocks per block that can be resident (the
   finer the split, the better the dispatcher balances ragged instances;
   0 = 64).  Results do not depend on these values (g and P up to the
   grouping of their FP64 sums). */
kp_status kp_set_batched_tuning(void *ctx, int32_t lds_bytes, int32_t block_mult);

/* Kernel choice for CSR costs: a problem that declares b_row_nnz = D (every
   item row holds D in {1, 2} entries at r*D) with M <= 16 runs the lean
   per-user kernel, which never reads b_rowptr; any other CSR problem runs
   the general kernel.  Evaluations (kp_eval_dual, kp_dd_step, the first
   pass of kp_primal_fixup) of dense costs with M <= 16 and K <= 16 run a
   lane-per-user kernel (one wave per 48-user tile, costs staged in LDS), and
   so do the SCD passes of such problems in which every threshold search
   starts with a window around lambda_k^t, or with windows away from it when
   a probe of 4096 users finds (almost) every line too far below zero to turn
   positive in any window (otherwise windows around lambda_k^{t-2} of
   alternating multipliers, and any other search mode: the general kernel).  The
   library keeps no record of a problem's structure between calls: the
   declaration travels with the problem.  kp_set_kernel_choice(ctx, 0)
   forces the general kernel for both (x and R are identical either way; g
   and P up to the grouping of their FP64 sums). */
kp_status kp_set_kernel_choice(void *ctx, int32_t allow_uniform_rows);

/* Structure query for per-item CSR costs (Sec. 2 layout): *D_out = D when
   every row r of the N*M item rows holds exactly D in {1, 2} stored entries
   at [r*D, r*D + D) (b_rowptr[r] == r*D for r = 0..N*M), else 0.  Reads
   b_rowptr once on the device (8 bytes per item row); b_row_nnz of prob is
   ignored.  D_out: HOST.  Synchronises the context stream. */
kp_status kp_csr_row_nnz(void *ctx, const kp_problem *prob, int32_t *D_out);

/* Alg.5's linear-time map (Sec. 5.1) in the SCD calls of this context (off
   by default): for problems in its setting -- M = K, CSR declared with one
   entry per item row (b_row_nnz = 1), at most one binding local set and it
   holds every item (top-Q) -- every user whose item j's entry is knapsack j
   takes Alg.5's single breakpoint per knapsack: with adj_j = max(p~_j, 0)
   and qth, q1th the Q-th and (Q+1)-th largest adj (0 past the last item),
   p_bar = q1th if adj_k >= qth else qth, and when p_k > p_bar the pair
   ((p_k - p_bar) / b_kk, b_kk).  The breakpoint uses the raw profit p_k as
   Alg.5 does, where the general map uses p~_k + lambda_k b_kk (reading A9),
   so the two agree to rounding of that intercept (a few ulp), not bit for
   bit.  Other users and problems keep the general map. */
kp_status kp_set_alg5(void *ctx, int32_t on);

/* Reduce of the SCD calls of this context: 0 (default) the exact threshold
   of Alg.4's reduce; 1 Sec. 5.2's approximate reduce -- the increments are
   summed per bucket of the breakpoints (a central bucket of half-width
   delta_k around lambda_k^t and base-2 buckets growing away from it, ids
   capped at +-31; delta_k the power of two 2^-20 of lambda_k^t, of 2^-20
   when lambda_k^t is smaller), the bucket [lo, hi] where the running sum from
   the top first exceeds B_k is found, and the threshold is
   max(lo, hi - (B_k - above) / S_bucket * (hi - lo)) with lo clamped at 0;
   0 when the total increment fits.  One pass per iteration, no windows. */
kp_status kp_set_reduce(void *ctx, int32_t mode);

/* Sampled start of the full threshold search (the search of a knapsack with
   no window, e.g. the first sweeps from lambda^0): on problems with at least
   min_users users (default 2^22; 0 = never) every stride-th user
   (n = max(N/64, min(N/2, 2^20)) of them) is gathered into a buffer of the
   context, the same search runs on that sample with every budget scaled by
   n/N (the scaling of Sec. 5.3), and the full search places its central
   buckets (half-width 2^-8 of the sample's threshold) around the sample's
   threshold, so that one pass usually emits the threshold's breakpoints.
   The result is the exact threshold either way. */
kp_status kp_set_sampled_start(void *ctx, int64_t min_users);

/* Threshold search of kp_scd_sweep (Alg.4 reduce, located near the
   previous multiplier).  After one sweep on a context, each
   knapsack whose last step was small against its multiplier starts with a
   window around lambda_k^t: users whose greedy set stays optimal over the
   whole window are checked in O(M) instead of walked, and only the
   breakpoints inside the window are emitted.  A threshold outside the window
   costs one more pass with the full search.  The result is the same
   lambda_out either way; kp_set_window(ctx, 0) turns the window off
   (default on). */
kp_status kp_set_window(void *ctx, int32_t on);
/* Window searches on this context since its creation: knapsack searches
   that started with a window, how many of them found the threshold above /
   below it (and so took the full search), and the breakpoints emitted inside
   windows.  HOST outputs, each may be NULL. */
kp_status kp_get_window_stats(void *ctx, int64_t *tried, int64_t *above, int64_t *below,
                              int64_t *emitted);
/* Users that the uniform-row kernel's window passes on this context listed
   for exact checks (their lines may cross inside a window; the others were
   proven calm by the gap filter), summed over sweeps.  HOST output, may be
   NULL.  Diagnostic: the results do not depend on it. */
kp_status kp_get_window_listed(void *ctx, int64_t *listed);

/* Size limits of the library. */
int32_t kp_max_items(void);        /* 64 */
int32_t kp_max_knapsacks_scd(void);/* largest K accepted by the SCD calls */

#ifdef __cplusplus
}
#endif
#endif /* KP_H */
