/*
 * apx.h -- C ABI of the MI355X (gfx950) dense affinity-propagation library.
 *
 * Method: Xia, Wu, Zhang, Zhuang, "Local and global approaches of affinity
 * propagation clustering for large scale data".
 *   Section 2, Algorithm 1  affinity propagation (Eqs. (1)-(4), damping,
 *                           exemplar decision, stop rules)
 *   Section 3, Algorithm 2  partition affinity propagation (PAP)
 *   Section 4, Algorithm 3  landmark affinity propagation (LAP), Steps 1-2
 * plus a learned warm start that is this library's own addition (the paper
 * starts from zero availabilities, Eq. (1), or from PAP's merge).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Matrices (S, R, A) are DEVICE pointers to FP32, row-major, n rows with
 *   leading dimension ld (elements): ld >= n, ld % 4 == 0, base address
 *   16-byte aligned.  Padding columns [n, ld) are never read as data and
 *   never written.
 * - Point sets X are DEVICE pointers to FP32, row-major n x d, leading
 *   dimension ldx >= d.
 * - Label / decision vectors are DEVICE int32 arrays of length n, 0-based.
 *   A label of -1 means "no exemplar" (only when the exemplar set is empty).
 * - Host-side arrays (partition permutations, offsets, results) are marked
 *   "host".  The caller owns every buffer it passes.  Scratch memory (column
 *   partials, run state, implicit-message lists, sub-problem matrices) comes
 *   from the context's workspace: either a device buffer the caller hands
 *   over with apx_set_workspace (sized with apx_workspace_size; the library
 *   then never allocates device memory on a compute call and returns
 *   APX_ENOMEM when a call needs more than was set), or, by default, a
 *   buffer the library allocates on first need, grows on demand and
 *   releases in apx_destroy.
 * - Every call returns an apx_status and never aborts.  Arguments are
 *   validated before any write, so APX_EINVAL leaves all outputs untouched.
 *   apx_last_error() returns a text for the last failure on the context.
 * - Work is enqueued on the context's HIP stream.  ap_iterate is
 *   asynchronous (stream-ordered); ap_similarity and the *_solve calls
 *   synchronise the stream before they return (ap_similarity to report
 *   non-finite input, the solves to fill their host result structs).
 * - One context per host thread; contexts share no mutable state.
 */
#ifndef APX_H
#define APX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APX_OK = 0,
    APX_EINVAL = 1,    /* invalid argument (shape, alignment, range, null) */
    APX_ENOMEM = 2,    /* device workspace could not be allocated */
    APX_EDEVICE = 3,   /* HIP runtime error; text via apx_last_error */
    APX_ENOTIMPL = 4   /* size or mode outside what the library supports */
} apx_status;

/* Preference modes for ap_similarity (Section 2: the diagonal s(k,k)). */
enum {
    APX_PREF_MEDIAN = 0, /* median of the n(n-1) off-diagonal similarities */
    APX_PREF_SCALAR = 1, /* one value for every point */
    APX_PREF_VECTOR = 2  /* per-point device vector of n floats */
};

/* Warm-start modes for ap_solve. */
enum {
    APX_COLD = 0,     /* A_0 = 0 (Eq. (1)) and R_0 = 0; A, R are outputs only */
    APX_WARM_A = 1,   /* A holds A_0 on entry (e.g. PAP's A'); R_0 = 0 */
    APX_WARM_AR = 2,  /* A and R hold A_0 and R_0 on entry */
    APX_WARM_COLUMNS = 3  /* A holds a column-structured A_0 (every off-diagonal
                             element of a column equal, as apx_warm_a0 and
                             ap_warmstart write it) and R_0 is the undamped
                             Eq. (2) step from it, which the solve forms itself
                             (R is not read); R_1 = R_0, since damping a
                             message towards itself leaves it unchanged.  Runs
                             with implicit R (alpha_t = 1) and implicit A from
                             A_0's column vectors where cold starts do */
};

typedef struct apx_ctx apx_ctx;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream). */
apx_status apx_create(apx_ctx **out, int device, void *hip_stream);
void apx_destroy(apx_ctx *ctx);
apx_status apx_set_stream(apx_ctx *ctx, void *hip_stream);
const char *apx_last_error(const apx_ctx *ctx);
/* Bytes of device workspace currently held by (or set on) the context. */
size_t apx_workspace_bytes(const apx_ctx *ctx);

/* Operations for apx_workspace_size. */
enum {
    APX_OP_SIMILARITY = 0,    /* ap_similarity: n points (d unused)                    */
    APX_OP_ITERATE = 1,       /* ap_iterate: n x n, leading dimension ld                */
    APX_OP_SOLVE = 2,         /* ap_solve (and pap_solve's Step 4): n x n, ld           */
    APX_OP_SOLVE_BATCHED = 3, /* ap_solve_batched: count instances of sizes[j] points,
                                 leading dimensions rounded up to 4 (sizes: host)      */
    APX_OP_PAP = 4,           /* pap_solve: n x n, ld, k = count parts of sizes[j]
                                 points (sizes: host, nullable = the paper's split)    */
    APX_OP_LAP = 5,           /* lap_solve: n points in d dimensions, count landmarks  */
    APX_OP_FEATURES = 6,      /* apx_features: n points                                */
    APX_OP_MLP_BACKWARD = 7,  /* apx_mlp_backward: count points                        */
    APX_OP_WARMSTART = 8,     /* ap_warmstart: n x n, ld                               */
    APX_OP_LAP_FULL = 9,      /* lap_full_solve: n points in d dimensions, count
                                 landmarks, m0 = ld                                    */
    APX_OP_SOLVE_MF = 10      /* ap_solve_mf: n points, count = panel_rows (0: the
                                 default panel)                                        */
};

/*
 * apx_workspace_size -- device workspace bytes one call of `op` needs for
 * the given sizes (see the op list above for which arguments are used).
 * Returns 0 for an unknown op or invalid sizes.  Every call uses the
 * workspace from its start, so one buffer of the largest size any call
 * needs serves a sequence of calls on one stream.
 */
size_t apx_workspace_size(const apx_ctx *ctx, int32_t op, int64_t n, int64_t ld, int64_t d,
                          int32_t count, const int64_t *sizes);

/*
 * apx_set_workspace -- use `bytes` bytes of caller-owned device memory at
 * dev_ptr (256-byte aligned, e.g. torch.empty(bytes, dtype=torch.uint8,
 * device='cuda')) as the context's workspace.  The library frees its own
 * buffer (after synchronising the stream) and from then on calls no
 * hipMalloc on compute calls: a call that needs more than `bytes` returns
 * APX_ENOMEM without launching work, and the automatic tuner (which
 * allocates a scratch problem) stays off for unseen sizes.  The caller keeps
 * the memory alive and unused by others until it sets another workspace or
 * destroys the context.  dev_ptr = NULL (bytes ignored) returns to a
 * library-owned workspace.  Calls that overlap on one stream are ordered;
 * contexts must not share one buffer.
 */
apx_status apx_set_workspace(apx_ctx *ctx, void *dev_ptr, size_t bytes);

/* apx_set_implicit -- list capacity of the implicit responsibilities used by
 * ap_solve when R_0 = 0 (APX_COLD, APX_WARM_A): unrolling the damped Eq. (2)
 * gives R_t(i,k) = (1 - lambda^t) s(i,k) - beta_t(i) on every column k that
 * was never row i's argmax of a+s; each row keeps beta and, for up to
 * list_capacity columns that were, (column, r_t(i,k)) pairs updated by the
 * damped Eq. (2), so an iteration reads S and A and writes A (12 bytes per
 * matrix element instead of 20).  When a row needs more
 * entries, R is made explicit and the run continues with explicit R.
 * 0 = always explicit R; default 16 (the maximum); the environment variable
 * APX_IMPLICIT_K sets it at context creation.  Only problems with
 * n >= min_n use it (default 8192: below that the explicit pass is faster).
 * Results agree with explicit R to rounding (the same arithmetic in another
 * order). */
apx_status apx_set_implicit(apx_ctx *ctx, int32_t list_capacity, int64_t min_n);

/* apx_set_implicit_a -- exception list capacity of the implicit
 * availabilities used by ap_solve on a cold start (A_0 = 0) together with
 * implicit R.  By Eq. (3) with damping, every off-diagonal a(i,k) whose
 * responsibility r(i,k) has never been positive equals one value per column,
 * acol_t(k) = lambda acol_{t-1}(k) + (1 - lambda) min(0, r(k,k) + sum_{i' != k}
 * max(0, r(i',k))), and by Eq. (4) the diagonal is a column vector as well.
 * Each row keeps the other elements (columns where its responsibility was
 * ever positive) as up to list_capacity (column, value) pairs, so an
 * iteration reads S and writes no matrix (4 bytes per element).  When a row
 * needs more entries, A is made explicit and the run continues with
 * explicit A.  0 = explicit A; default 1024 (the maximum); the environment
 * variable APX_IMPLICIT_A sets it at context creation.  Only cold starts
 * with n >= min_n use it (default 4096: below that the explicit pass is
 * faster); with it, R is implicit too whatever apx_set_implicit's min_n.
 * A is the same arithmetic as the explicit update, element for element. */
apx_status apx_set_implicit_a(apx_ctx *ctx, int32_t list_capacity, int64_t min_n);

/* apx_last_solve_info -- how many iterations of the last ap_solve on this
 * context ran with implicit R and how many with explicit R; and (nullable)
 * how many ran with implicit A. */
apx_status apx_last_solve_info(apx_ctx *ctx, int32_t *implicit_iters, int32_t *explicit_iters,
                               int32_t *implicit_a_iters);

/* apx_last_fallback -- why the last ap_solve on this context left an
 * implicit form and continued with explicit messages (0: it did not): an OR
 * of APX_FALLBACK_R_LIST (a row's list of ever-argmax columns was full),
 * APX_FALLBACK_R_OWNER (a new list column would have given one thread of the
 * implicit-R pass more listed columns than it keeps in registers) and
 * APX_FALLBACK_A_LIST (a row's list of ever-positive responsibilities was
 * full).  APX_NOTE_R_OWNER (no fallback by itself) says that the implicit-A
 * pass let a row list break that owner rule, so a fallback of A would have
 * made R explicit too.  Diagnostic only; results do not depend on it. */
enum { APX_FALLBACK_R_LIST = 1, APX_FALLBACK_A_LIST = 2, APX_FALLBACK_R_OWNER = 4, APX_NOTE_R_OWNER = 8 };
apx_status apx_last_fallback(apx_ctx *ctx, int32_t *reasons);

/* apx_set_lean_scan -- the implicit-A pass leaves the ordinary columns out
 * of the exemplar decision of Algorithm 1 (argmax of a + r, Eqs. (2)-(4))
 * where they cannot change it (enable = 1, the default): a row's listed and
 * new columns already beat the diagonal, or D = a(i,i) + r(i,i) > 0 while
 * every column value is <= 0; any other row is decided again over its
 * ordinary columns after the reduction.  Positivity of the off-list
 * responsibility al*s - beta is a compare of s against a per-row threshold
 * certified to give the same answer in FP32.  enable = 0 (a cross-check)
 * tests positivity as fl(al*s) > beta and decides every row over its
 * ordinary columns after the reduction.  Results are bit-identical either
 * way. */
apx_status apx_set_lean_scan(apx_ctx *ctx, int enable);

/* apx_last_lean_rescans -- rows of the last ap_solve on this context (summed
 * over its implicit-A passes) whose ordinary columns had to be tested after
 * the reduction.  Diagnostic only. */
apx_status apx_last_lean_rescans(apx_ctx *ctx, int32_t *rows);

/* apx_set_graphs -- replay the iteration loop of ap_solve as a captured HIP
 * graph (enable = 1, the default; the environment variable APX_GRAPHS=0
 * turns it off at context creation) or launch every kernel from the host
 * (enable = 0).  The graph runs on a private stream of the context, ordered
 * after the context stream with an event; results are identical either way. */
apx_status apx_set_graphs(apx_ctx *ctx, int enable);

/* ---------------------------------------------------------------------------
 * Autotuner.  Sizes are grouped into buckets that share one row-pass shape
 * (n <= 4096: ceil(n/1024); above: 4 + ceil((n-4096)/4096)).  For a bucket
 * the tuner times every instantiated row-pass workgroup size (256, 512, 1024
 * threads) and variant (LDS-resident or register) on a scratch problem with
 * the same row length and keeps the fastest; it also sets the host poll
 * interval of the stop flag (used when apx_params.check_every is 0) so that
 * a poll costs about 1% of the iterations between polls.  All candidates
 * share the row -> workgroup map, so tuning never changes a result bit.
 * The environment variable APX_TUNE_FILE names a file loaded at context
 * creation; APX_AUTOTUNE=1 tunes unseen buckets on first use.
 * ------------------------------------------------------------------------- */

/* apx_autotune -- measure the bucket of n now (allocates and frees a scratch
 * problem of up to 4 x #CU rows; synchronises the context stream). */
apx_status apx_autotune(apx_ctx *ctx, int64_t n);
/* apx_set_autotune -- tune unseen buckets automatically (enable = 1). */
apx_status apx_set_autotune(apx_ctx *ctx, int enable);
/* apx_tune_set -- set the bucket of n by hand (EINVAL if that workgroup size
 * has no row pass for n). */
apx_status apx_tune_set(apx_ctx *ctx, int64_t n, int32_t threads, int32_t lds, int32_t check_every);
/* apx_tune_get -- the entry used for n (threads = 0 if none); lds reports the
 * variant that actually runs at this n. */
apx_status apx_tune_get(apx_ctx *ctx, int64_t n, int32_t *threads, int32_t *lds, int32_t *check_every,
                        double *ms_per_iter);
/*
 * Message forms of a cold (or column-structured warm) ap_solve:
 * APX_FORM_EXPLICIT (R and A in memory, 20 bytes per element and iteration),
 * APX_FORM_IMPLICIT_R (R kept implicitly, 12 bytes) and APX_FORM_IMPLICIT_RA
 * (R and A implicit, 4 bytes).  Without a tuned form the solve picks by size
 * (apx_set_implicit, apx_set_implicit_a).  The forms agree to rounding, not
 * bit for bit, so a tuned form can change results at the rounding level.
 */
enum { APX_FORM_DEFAULT = 0, APX_FORM_EXPLICIT = 1, APX_FORM_IMPLICIT_R = 2, APX_FORM_IMPLICIT_RA = 3 };
/* apx_autotune_form -- time the three forms on a synthetic problem of n
 * points (a 16-D Gaussian mixture built on the device: S, R and A of n x n
 * are allocated and freed; a few short solves per form) and keep the
 * fastest per iteration for the bucket of n.  form (nullable) receives the
 * pick, ms (nullable, 3 doubles) the measured ms per iteration of each. */
apx_status apx_autotune_form(apx_ctx *ctx, int64_t n, int32_t *form, double *ms);
/* apx_tune_set_form -- set the form of the bucket of n by hand
 * (APX_FORM_DEFAULT clears it). */
apx_status apx_tune_set_form(apx_ctx *ctx, int64_t n, int32_t form);
/* apx_tune_get_form -- the form recorded for n (APX_FORM_DEFAULT if none)
 * and, if ms is non-null, the 3 measured ms per iteration (0 if not timed). */
apx_status apx_tune_get_form(apx_ctx *ctx, int64_t n, int32_t *form, double *ms);
/* apx_autotune_batched -- time the plans of the persistent batched launch
 * (ap_solve_batched, pap_solve's Step 2) for a batch of `count` instances of
 * sizes[j] points (host) on scratch instances of those sizes (allocated and
 * freed: 3 n x n matrices each), over workgroups per compute unit 1..4 and
 * 2, 8 or 32 rows at least per team member, and keep the fastest for
 * batches of that shape (the bit lengths of count and of the largest n).
 * Outputs (nullable): the pick and its time for 12 iterations.  Plans group
 * the column partial sums differently, so a tuned plan changes results at
 * the rounding level. */
apx_status apx_autotune_batched(apx_ctx *ctx, int32_t count, const int64_t *sizes, int32_t *wpc,
                                int32_t *min_rows, double *ms);
/* apx_tune_clear -- forget every entry (back to the default plans). */
apx_status apx_tune_clear(apx_ctx *ctx);
/* apx_tune_save / apx_tune_load -- the context's entries as JSON (path: host
 * string).  Loading rejects a file tuned for another compute-unit count. */
apx_status apx_tune_save(apx_ctx *ctx, const char *path);
apx_status apx_tune_load(apx_ctx *ctx, const char *path);

/* Kernel timing for benchmarks: while enabled, ap_solve brackets every full
 * row pass (the dominant kernel) with HIP events on the context stream (the
 * passes are then launched from the host, not replayed as a graph) and
 * accumulates the launch count and total duration of the passes that did
 * work.  apx_profile_read returns and clears the totals.  Timing never
 * changes results. */
apx_status apx_profile(apx_ctx *ctx, int enable);
apx_status apx_profile_read(apx_ctx *ctx, int64_t *launches, double *total_ms);

/* apx_params.flags */
enum {
    /* idx receives the raw decisions d_i = argmax_k a(i,k)+r(i,k) of the stop
     * iteration (lowest k on ties) instead of the valid labelling; dpsim and
     * expref are then summed over those labels (Section 2, the decision rule). */
    APX_RAW_LABELS = 1,
    /* Before any write, scan S (the solve's input) and return APX_EINVAL if
     * any entry is NaN or infinite.  Without it, non-finite S gives
     * unspecified messages and labels. */
    APX_CHECK_FINITE = 2,
    /* Also stop (converged = 1) after the first iteration t >= 2 whose
     * message changes are all at most msg_tol:
     * max_{i,k} |r_t(i,k) - r_{t-1}(i,k)| <= msg_tol and
     * max_{i,k} |a_t(i,k) - a_{t-1}(i,k)| <= msg_tol (Algorithm 1, Step 4,
     * "changes in the messages fall below a threshold").  Runs the explicit
     * form of the iteration (R and A in memory). */
    APX_MSG_THRESHOLD = 4
};

typedef struct {
    float damping;       /* lambda in [0,1): new = lambda*old + (1-lambda)*update (Section 2) */
    int32_t max_iter;    /* >= 1: iteration cap (Section 2, Step 4) */
    int32_t conv_iter;   /* >= 0: stop once the exemplar set has been the same, and
                            non-empty, for conv_iter consecutive iterations;
                            0 = no exemplar-set rule (max_iter, or the message
                            threshold, ends the run) */
    int32_t check_every; /* iterations between host polls of the stop flag
                            (0 = library default 16; odd values are rounded
                            up to even, the length of one graph replay);
                            never changes results */
    uint32_t flags;      /* APX_RAW_LABELS | APX_CHECK_FINITE | APX_MSG_THRESHOLD */
    float msg_tol;       /* >= 0: threshold of APX_MSG_THRESHOLD (units of S) */
} apx_params;

typedef struct {
    int32_t iterations;  /* iterations run (the stop iteration) */
    int32_t converged;   /* 1 if the exemplar-set rule stopped the run */
    int32_t n_exemplars; /* |E| */
    int32_t status;      /* apx_status of this instance */
    double dpsim;        /* sum of s(i, idx(i)) over non-exemplars (Algorithm 1 output) */
    double expref;       /* sum of s(k,k) over exemplars */
    double netsim;       /* dpsim + expref (= -E(c), Section 2) */
} apx_result;

/*
 * ap_similarity -- S from points (Section 2): s(i,k) = -||x_i - x_k||^2,
 * computed as 2<x_i,x_k> - (||x_i||^2 + ||x_k||^2) with FP32 matrix cores and
 * mirrored so that S is exactly symmetric before noise.  Then the diagonal
 * is set to the preferences (pref_mode; pref_vec is a device vector used by
 * APX_PREF_VECTOR, pref_scalar by APX_PREF_SCALAR), and, if noise_rel > 0,
 * every entry gets noise_rel * (max S - min S) * u(noise_seed, i, k), where
 * u is the SplitMix64 output function of the counter i*n+k+1 (top 53 bits
 * scaled to [0,1)) and the range is taken over S with the preferences set.
 * pref_out (host, nullable) receives the preference used (median or scalar).
 * Non-finite input: X or pref_vec holding a NaN or infinity gives
 * APX_EINVAL before S is written; finite X whose similarities overflow
 * FP32 gives APX_EINVAL after the build (S is then unspecified).
 * Requires n >= 2, 1 <= d.  Synchronises the stream.
 */
apx_status ap_similarity(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                         float *S, int64_t ld, int32_t pref_mode, const float *pref_vec,
                         float pref_scalar, uint64_t noise_seed, double noise_rel,
                         double *pref_out);

/*
 * ap_iterate -- n_iter damped iterations of Algorithm 1 (Eqs. (2), (3), (4)).
 * On entry R, A hold the messages after some iteration t (zeros for a cold
 * start); on exit they hold those after iteration t + n_iter.  Each
 * iteration first updates and damps R from (S, A), then A from the new R.
 * decision (device, nullable) receives argmax_k a(i,k)+r(i,k) after the last
 * iteration (lowest k on ties).  Calls compose: n1 then n2 iterations give
 * bit-identical messages to n1 + n2 in one call.  Requires 2 <= n <= 131072
 * (APX_ENOTIMPL above) and n_iter >= 1; rows beyond 49152 elements are
 * streamed twice per pass instead of held in registers.  Asynchronous.
 */
apx_status ap_iterate(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                      float damping, int32_t n_iter, int32_t *decision);

/*
 * ap_iterate_noalloc -- ap_iterate for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels, launch plan and results (bit for
 * bit), with the column vectors and partials in a fixed scratch array
 * compiled into the library (12 MiB per GPU, held until the process ends)
 * instead of the context workspace.  It calls no allocating routine.
 * Serves 2 <= n <= 8192; larger n gives APX_EINVAL.  Every call on one GPU
 * shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other contexts or threads) race and give undefined results;
 * calls ordered on one stream are safe.  Asynchronous.
 */
apx_status ap_iterate_noalloc(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                              float damping, int32_t n_iter, int32_t *decision);

/*
 * ap_solve -- Algorithm 1 to its stop rule.  S holds the similarities with
 * the preferences on the diagonal.  warm selects the start (APX_COLD,
 * APX_WARM_A, APX_WARM_AR).  On exit R and A hold the messages of the stop
 * iteration, idx (device, n) the labels: exemplars E = {k : argmax_j
 * a(k,j)+r(k,j) = k} label themselves and every other point takes the
 * exemplar of largest s(i,k) (lowest k on ties).  res (host) gets the
 * iteration count, convergence flag, |E| and dpsim/expref/netsim in FP64.
 * n = 1 returns idx = [0] and netsim = s(0,0) without iterating; n above
 * 131072 gives APX_ENOTIMPL (the caller's S, R, A and one more n x n buffer
 * of the library must fit in device memory).  Non-convergence is not an
 * error (converged = 0).  Synchronises the stream.
 */
apx_status ap_solve(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                    int32_t warm, const apx_params *params, int32_t *idx, apx_result *res);

/*
 * ap_solve_mf -- Algorithm 1 from the points, without any n x n buffer
 * (matrix-free; beyond the paper, for problems whose S does not fit in
 * memory).  Every iteration rebuilds S one panel of rows at a time from X
 * (device, n x d FP32, row stride ldx) on the matrix cores, each entry with
 * the value ap_similarity would store for the same pref_mode / pref_vec /
 * pref_scalar / noise_seed / noise_rel (Section 2: s(i,k) = -||x_i -
 * x_k||^2, preferences on the diagonal, tie noise), and runs the implicit
 * message passes on those rows; the median preference takes three sweeps of
 * panels before the run.  Memory: two panels of panel_rows x round64(n)
 * floats (panel_rows = 0: at most 1 GiB per panel, at least 8 rows per
 * workgroup) plus O(n) state and the column partials of the panels.  A
 * cold start only; the exemplar set, labels (idx, device, n), iteration
 * count and sums are those of ap_similarity + ap_solve up to the rounding of
 * the column sums' grouping (each panel sums its own rows).  pref_out (host,
 * nullable) gets the scalar preference.  APX_ENOTIMPL when n is outside the
 * implicit passes (2 .. 40448: a row of at most ten 4-float chunks per
 * thread, the implicit-R prologue's partials in LDS), when a row's message list overflows (the explicit form would
 * need R and A), and for APX_RAW_LABELS or APX_MSG_THRESHOLD; APX_EINVAL for non-finite X or
 * pref_vec, a bad preference mode, or panel_rows below one row per
 * workgroup.  Synchronises the stream.
 */
apx_status ap_solve_mf(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx, int32_t pref_mode,
                       const float *pref_vec, float pref_scalar, uint64_t noise_seed, double noise_rel,
                       int64_t panel_rows, const apx_params *params, int32_t *idx, apx_result *res,
                       double *pref_out);

/* One instance of a batched solve: its own S (preferences on the diagonal),
 * R, A (device, FP32, ld >= n, ld % 4 == 0) and labels idx (device, n). */
typedef struct {
    int64_t n;
    int64_t ld;
    const float *S;
    float *R;
    float *A;
    int32_t *idx;
} apx_instance;

/*
 * ap_solve_batched -- Algorithm 1 on `count` independent instances of uneven
 * size (inst: host array) in one persistent cooperative launch: each
 * instance gets a team of workgroups (sized in proportion to its n^2; with
 * more instances than workgroups, instances are dealt to single workgroups
 * largest first), teams meet at device-side barriers, and each instance
 * keeps its own stop rule and stops independently.  Per instance the arithmetic is that of ap_solve;
 * only the grouping of the FP32 column partial sums differs (rows are split
 * into blocks differently), so results agree with ap_solve to rounding.
 * The results are deterministic.  res (host, count).  Instances need
 * 2 <= n <= 12288.  Synchronises.
 */
apx_status ap_solve_batched(apx_ctx *ctx, int32_t count, const apx_instance *inst, int32_t warm,
                            const apx_params *params, apx_result *res);

/*
 * pap_solve -- partition affinity propagation (Section 3, Algorithm 2).
 * Step 1: the points are split into k parts; part j holds the points
 * perm[offsets[j] .. offsets[j+1]-1] (perm: host, n entries, a permutation;
 * NULL = identity; offsets: host, k+1 entries from 0 to n; NULL = the
 * paper's split into k-1 parts of floor(n/k) points and a last part of the
 * rest).  Step 2: AP on every diagonal block S_jj (with its diagonal, i.e.
 * the global preferences), all blocks in one batch.  Step 3: A' holds each
 * A_jj at its points' positions and zeros elsewhere.  Step 4: AP on S from
 * A' with R_0 = 0.  Outputs as ap_solve; sub (host, k, nullable) receives
 * the per-part results of Step 2.  Needs 1 <= k <= n.  Synchronises.
 */
apx_status pap_solve(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                     int32_t k, const int64_t *perm, const int64_t *offsets,
                     const apx_params *params, int32_t *idx, apx_result *res, apx_result *sub);

/*
 * lap_solve -- landmark affinity propagation (Section 4, Algorithm 3, Steps
 * 1-2 without the per-class distance threshold).  Step 1: the landmark set M
 * (host array `landmarks` of n_landmarks distinct indices, or NULL to draw a
 * uniform sample without replacement from a SplitMix64 stream seeded with
 * `seed`) gets its similarity matrix (ap_similarity with pref_mode
 * APX_PREF_MEDIAN, the median of the landmark similarities, or
 * APX_PREF_SCALAR, pref_scalar for every landmark; tie noise noise_rel from
 * `seed`) and AP with `params`.  Step 2: every point
 * goes to the exemplar of least squared Euclidean distance (exact: FP32
 * distances with an FP64 recheck of every candidate within the FP32 error
 * bound; lowest exemplar index on ties); exemplars label themselves.  The
 * n x n similarity matrix is never formed.  X: device n x d (ldx).  idx:
 * device, n global labels.  res: iterations/converged of the landmark AP,
 * |E|, dpsim = -sum of squared distances of non-exemplars to their exemplar
 * (FP64), expref = |E| * landmark preference, netsim.  params->flags:
 * APX_CHECK_FINITE and APX_MSG_THRESHOLD apply to the landmark AP;
 * APX_RAW_LABELS is rejected (labels here are assignments).  exemplars_out (host,
 * nullable, capacity n_landmarks) receives the exemplar indices ascending.
 * Needs 2 <= n_landmarks <= n, d <= 4096.  Synchronises.
 */
apx_status lap_solve(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                     int64_t n_landmarks, const int64_t *landmarks, uint64_t seed, double noise_rel,
                     int32_t pref_mode, float pref_scalar, const apx_params *params, int32_t *idx,
                     apx_result *res, int64_t *exemplars_out);

/*
 * apx_lap_landmarks -- a landmark set for Step 1 of Algorithm 3 that keeps
 * given points, e.g. a previous run's exemplars (re-seeding the landmarks;
 * the paper's closing section names a better choice of landmarks as future
 * work), and fills the rest with a uniform sample without replacement of
 * the other points: a partial Fisher-Yates shuffle of their positions (in
 * ascending index order) driven by the SplitMix64 stream seeded with `seed`.
 * keep: host, n_keep distinct indices in [0, n) (n_keep <= n_landmarks);
 * out: host, n_landmarks entries, ascending.  Host only (no device work, no
 * context); EINVAL on bad arguments.
 */
apx_status apx_lap_landmarks(int64_t n, int64_t n_landmarks, const int64_t *keep, int64_t n_keep, uint64_t seed,
                             int64_t *out);

/* What the full landmark method did at its top level. */
typedef struct {
    int32_t levels;          /* recursion levels run (1: Step 3 needed no recursion) */
    int32_t step1_centres;   /* |C1|: centres of the landmark AP (Step 1) */
    int64_t assigned;        /* points Step 2 assigned below their class's max_distance */
    int64_t unassigned;      /* m: points left for Step 3 */
    int32_t merged_centres;  /* |C1| plus Step 3's centres */
    int32_t step3_mode;      /* 0: nothing left, 1: AP on the m points, 2: the method on them */
    int32_t refined_centres; /* centres after Step 4 (the exemplars) */
    int32_t pad;
    double preference;       /* p of the landmark AP, used by every later AP and by expref */
} apx_lap_stats;

/*
 * lap_full_solve -- landmark affinity propagation, Section 4, Algorithm 3,
 * Steps 1-4 (lap_solve is Steps 1-2 without the threshold).
 *   Step 1: AP on the landmarks (given, or sampled as in lap_solve from
 *           `seed`): centres C1 and each landmark's class; preference p from
 *           pref_mode (APX_PREF_MEDIAN: the median of the landmark
 *           similarities; APX_PREF_SCALAR: pref_scalar).
 *   Step 2: max_distance(c) = the largest squared Euclidean distance of a
 *           landmark of class c to c; every other point goes to its nearest
 *           centre c (exact, lowest index on ties) when its distance is
 *           strictly below max_distance(c); the m others stay unassigned.
 *   Step 3: m <= m0: AP on the m points; m > m0: the whole method on them,
 *           with min(n_landmarks, m0) landmarks drawn uniformly from them (a
 *           partial Fisher-Yates shuffle driven by the SplitMix64 stream
 *           seeded with seed + 3 per level); their centres join C1.
 *   Step 4: every point goes to its nearest merged centre, and each class's
 *           centre becomes its medoid (least summed FP64 squared distance to
 *           the class, lowest index on ties).
 * Finally every point goes to its nearest refined centre; the refined
 * centres are the exemplars (they label themselves).  Every AP after the
 * first uses p; tie noise noise_rel with seed + 3l (Step 1), + 1 (Step 3)
 * at recursion level l.  X: device n x d (ldx), d <= 300, all finite
 * (else APX_EINVAL).  idx: device, n labels.  res: the landmark AP's
 * iterations and convergence, |E|, dpsim = -sum of FP64 squared distances
 * of non-exemplars to their exemplar, expref = |E| p, netsim.  stats (host,
 * nullable): see apx_lap_stats.  exemplars_out (host, nullable, capacity
 * n) receives the exemplars ascending.  params->flags:
 * APX_MSG_THRESHOLD applies to every AP; APX_RAW_LABELS is rejected.
 * Synchronises.
 */
apx_status lap_full_solve(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx, int64_t n_landmarks,
                          const int64_t *landmarks, uint64_t seed, double noise_rel, int32_t pref_mode,
                          float pref_scalar, int64_t m0, const apx_params *params, int32_t *idx,
                          apx_result *res, apx_lap_stats *stats, int64_t *exemplars_out);

/* ---------------------------------------------------------------------------
 * Learned warm start.  The paper starts Algorithm 1 from a(i,k) = 0 (Eq. (1))
 * and warm-starts only through PAP's merged availabilities (Section 3,
 * Algorithm 2, steps 3-4).  These calls predict the starting messages per
 * point from its row of S with a small network instead; none of it is in the
 * paper.  All pointers are DEVICE pointers; all calls are stream-ordered and
 * do not synchronise (except when the context workspace has to grow).
 * ------------------------------------------------------------------------- */

/* Network 16 -> 128 -> 128 -> 2 (GELU after each hidden layer).  Parameters
 * are one flat FP32 vector of APX_MLP_PARAMS values: W1 [16][128], b1 [128],
 * W2 [128][128], b2 [128], W3 [128][2], b3 [2], each row-major, in that
 * order; layer l computes z = h W_l + b_l.  The forward pass rounds the
 * features, W1..W3 and both hidden activations to bfloat16 (nearest even)
 * and accumulates in FP32 on the matrix cores; biases stay FP32. */
#define APX_MLP_FEATURES 16
#define APX_MLP_PARAMS 18946

/*
 * apx_features -- 16 features per point from S (n >= 2, preferences on the
 * diagonal), written to F (n x 16, row-major, 16-byte aligned), and the scale
 * sigma (one float) they are divided by.  With o_0 <= ... <= o_{m-1} the
 * m = n-1 off-diagonal values of row k and mu_k = o_{floor((m-1)/2)}:
 *   sigma    |lower median of mu_0..mu_{n-1}| (1 if that is 0 or not finite)
 *   f0..f5   o_{m-1-min(j,m-1)}/sigma, j = 0,1,3,7,15,31 (1st..32nd largest)
 *   f6       mean of the min(32,m) largest / sigma
 *   f7..f11  o_{floor(q(m-1)/100)}/sigma, q = 1,10,25,50,75
 *   f12      (s(k,k) - mu_k)/sigma         f13  (s(k,k) - f6 sigma)/sigma
 *   f14      #{j != k : s(k,j) > s(k,k)} / m      f15  ln(n)/10
 * Order statistics are exact; each feature is formed in FP64 and rounded to
 * FP32 once.
 */
apx_status apx_features(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *F, float *sigma);

/* apx_mlp_forward -- Y (count x 2) = network(theta, F (count x 16, 16-byte
 * aligned)). */
apx_status apx_mlp_forward(apx_ctx *ctx, const float *theta, const float *F, int64_t count, float *Y);

/*
 * apx_mlp_backward -- gradient of the loss
 *   L = sum_p w_p sum_o huber(y_po - T_po),  huber(e) = e^2/2 (|e| <= 1), |e| - 1/2,
 * with respect to the FP32 parameters, over the batch of `count` points
 * rows[0..count-1] of F (x 16), T (x 2) and w (rows: device int64, nullable =
 * points 0..count-1).  The bfloat16 roundings of the forward pass are treated
 * as the identity.  grad (APX_MLP_PARAMS floats) is overwritten; loss
 * (nullable, one double) receives L.  Reductions have a fixed order, so the
 * result is deterministic.
 */
apx_status apx_mlp_backward(apx_ctx *ctx, const float *theta, const float *F, const float *T,
                            const float *w, const int64_t *rows, int64_t count, float *grad,
                            double *loss);

/* apx_mlp_adam -- one Adam step (Kingma and Ba, 2015) on theta with moment
 * buffers m, v (all count floats) and bias correction for step >= 1:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * theta -= lr (m/(1-b1^step)) / (sqrt(v/(1-b2^step)) + eps). */
apx_status apx_mlp_adam(apx_ctx *ctx, float *theta, float *m, float *v, const float *grad,
                        int64_t count, int32_t step, float lr, float beta1, float beta2, float eps);

/* apx_targets -- training targets from converged responsibilities R: with
 * c_k = sum_{i != k} max(0, r(i,k)) and t_k = r(k,k) + c_k (the column
 * quantities of Eqs. (3)-(4), summed in FP64), Y[k] = (t_k/sigma, c_k/sigma)
 * (n x 2); sigma is a device float (as written by apx_features). */
apx_status apx_targets(apx_ctx *ctx, const float *R, int64_t n, int64_t ld, const float *sigma, float *Y);

/* apx_warm_a0 -- A_0 from per-point predictions Y (n x 2): a(i,k) =
 * min(0, sigma Y[k][0]) for i != k, a(k,k) = max(0, sigma Y[k][1]) (FP32
 * products), i.e. Eqs. (3)-(4) with the predicted column quantities. */
apx_status apx_warm_a0(apx_ctx *ctx, const float *Y, const float *sigma, int64_t n, float *A, int64_t ld);

/*
 * ap_warmstart -- starting messages for ap_solve(..., APX_WARM_AR, ...):
 * features of S, the network with parameters theta, A_0 as apx_warm_a0, and
 * R_0 = the undamped responsibility update of Eq. (2) from A_0,
 * r(i,k) = s(i,k) - max_{k' != k} (a_0(i,k') + s(i,k')).  Overwrites R and A.
 * sigma (device, nullable) receives the feature scale.  Needs 2 <= n <= 65536.
 */
apx_status ap_warmstart(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, const float *theta,
                        float *R, float *A, float *sigma);

#ifdef __cplusplus
}
#endif
#endif /* APX_H */
