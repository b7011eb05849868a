// apx_internal.h -- shared declarations of the HIP library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/apx.h"

namespace apx {

// Device-side run state of one AP instance (one solve).  Updated by the
// column-reduce kernel after every full row pass; read by the host every few
// iterations.  All counters are integers, so their atomics are deterministic.
struct ApState {
    int32_t iter;       // completed iterations t (A_t computed)
    int32_t run;        // consecutive iterations with an unchanged exemplar set
    int32_t frozen;     // 1 once the stop rule fired: later passes are no-ops
    int32_t converged;  // 1 if the exemplar-set rule fired
    int32_t nex;        // |E_t| accumulated by the running pass
    int32_t changed;    // E_t != E_{t-1}, accumulated by the running pass
    int32_t max_iter;
    int32_t conv_iter;
    int32_t last_nex;   // |E| of the last completed iteration
    int32_t imp_abort;  // bit 0: an implicit-R row list was full; bit 2: its owner rule; bit 1: an implicit-A list was full
    float imp_lam;      // damping of the run
    float imp_al;       // alpha_t for the next full pass t (1 - lambda^t)
    float imp_al1;      // alpha_{t+1}
    float imp_al_prev;  // alpha of the last full pass that ran
    // Message-change stop rule (Algorithm 1, Step 4), explicit passes only:
    // bit patterns of non-negative floats, so unsigned atomicMax orders them.
    uint32_t d_a;       // max |a_t - a_{t-1}| of the running pass t
    uint32_t d_r_next;  // max |r_{t+1} - r_t| of the running pass t
    uint32_t d_r;       // max |r_t - r_{t-1}| (from pass t-1)
    int32_t msg_on;     // 1: stop once both changes are <= msg_tol (t >= 2)
    float msg_tol;
    int32_t imp_owner;  // 1: an implicit-A pass let a thread own more listed R columns than k_row_imp keeps
    int32_t imp_alpha_one;  // 1: alpha_t = 1 for every t (R_0 is the undamped Eq. (2) step, not 0)
    int32_t lean_rescans;   // rows of lean implicit-A scans that the ordinary columns had to decide
};

// Row-pass modes.  A full pass of iteration t reads R_t, A_{t-1}, S and the
// column vectors of R_t; it writes A_t, the decisions d_t and R_{t+1} with
// the column partials of max(0, R_{t+1}).
//   PASS_FULL    A_t, decisions, R_{t+1}          (reads S, R, A)
//   PASS_R_ONLY  R_{t+1} from (R_t, A_t)           (reads S, R, A)
//   PASS_R_COLD  R_1 from R_0 = A_0 = 0            (reads S)
//   PASS_A_ONLY  A_t and decisions, no R_{t+1}      (reads R, A)
//   PASS_FULL_DELTA  PASS_FULL that also records max |a_t - a_{t-1}| and
//                max |r_{t+1} - r_t| in the run state (message-change stop)
enum PassMode : int { PASS_FULL = 0, PASS_R_ONLY = 1, PASS_A_ONLY = 2, PASS_R_COLD = 3, PASS_FULL_DELTA = 4 };

struct PassArgs {
    const float *S;
    const float *Rin;   // R_t (may alias Rout: each element is read before it is written)
    float *Rout;        // R_{t+1}
    float *A;           // A_{t-1} in, A_t out (in place)
    int64_t ld;
    int32_t n;
    float lam;
    const float *tcol;  // t_k = r(k,k) + c_k of R_t
    const float *ccol;  // c_k = sum_{i != k} max(0, r(i,k)) of R_t
    float *partial;     // [gridDim.x][ldp] column partials of max(0, R_{t+1})
    int64_t ldp;
    float *rdiag;       // r_{t+1}(k,k)
    int32_t *dec;       // decisions d_t (nullable)
    uint8_t *eflag;     // exemplar flags of the previous iteration (nullable)
    ApState *st;        // nullable: no stop-rule bookkeeping
    int64_t row_begin;  // rows handled by this launch: [row_begin, row_end)
    int64_t row_end;
};

struct ColArgs {
    const float *partial;
    int64_t ldp;
    int32_t nparts;
    const float *rdiag;
    float *tcol;
    float *ccol;
    int32_t n;
    ApState *st;        // nullable
    int32_t bookkeep;   // 1: apply the stop rule for the pass just finished
    // Implicit availabilities (nullable): with the column vectors of R_{t+1}
    // just summed, acol_{t+1} = lam acol_t + (1-lam) min(0, t_k) and
    // adiag_{t+1} = lam adiag_t + (1-lam) c_k (Eqs. (3), (4), damping).
    const float *acol_in, *adiag_in;
    float *acol_out, *adiag_out;
    float lam;
};

// Largest n of ap_iterate and ap_solve: four n x n FP32 matrices (S, A and
// the two R buffers) fill the 288 GB of one MI355X at about this size.
constexpr int64_t kMaxSolveN = 131072;

// Launch helpers (ap_iter.hip).
struct PassPlan {
    int threads;   // workgroup size
    int chunks;    // float4 chunks per thread per row
    int grid;      // workgroups
    size_t lds_bytes;  // dynamic LDS of the LDS-resident variant (0: register variant)
    int two_sweep;     // 1: rows streamed twice (rows beyond the register-resident variants)
};
PassPlan plan_pass(int64_t n, int num_cus);
// The same row -> workgroup map with a chosen workgroup size and variant;
// threads = 0 in the result when that combination is not instantiated.
PassPlan plan_pass_variant(int64_t n, int num_cus, int threads, bool lds);
hipError_t launch_row_pass(const PassPlan &pl, int mode, const PassArgs &a, hipStream_t s);
hipError_t launch_col_reduce(const ColArgs &a, hipStream_t s);
hipError_t launch_state_init(ApState *st, int32_t max_iter, int32_t conv_iter, float lam, hipStream_t s,
                             int msg_on = 0, float msg_tol = 0.0f, int alpha_one = 0);
// acol[k] = A(r,k) for one r != k, adiag[k] = A(k,k) (column-structured A_0)
hipError_t launch_extract_cols(const float *A, int64_t ld, int32_t n, float *acol, float *adiag, hipStream_t s);
// flag |= 1 if any of the n x n entries of M (leading dimension ld) is NaN or
// infinite; flag |= 1 likewise for the rows x cols entries of X (ldx).
hipError_t launch_check_finite(const float *M, int64_t rows, int64_t cols, int64_t ld, int32_t *flag,
                               hipStream_t s);
// Raw decisions d_i = argmax_k a(i,k) + r(i,k), lowest k on ties.
hipError_t launch_decide(const float *A, const float *R, int64_t n, int64_t ld, int32_t *dec, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_fill_f32_rows(float *p, int64_t rows, int64_t cols, int64_t ld, float v,
                                hipStream_t s);
hipError_t launch_copy_rows(float *dst, const float *src, int64_t rows, int64_t cols, int64_t ld,
                            hipStream_t s);

// Implicit responsibilities (ap_iter.hip).  With R_0 = 0 the damped Eq. (2)
// unrolls to R_t(i,k) = alpha_t s(i,k) - beta_t(i) with alpha_t = 1 -
// lambda^t, beta_{t+1} = lambda beta_t + (1-lambda) v1_t, on every column k
// that was never row i's argmax k1 of a+s; the columns that were (a short
// list per row) keep r_t(i,k) itself, updated by the damped Eq. (2)
// r_{t+1} = (lambda r_t + (1-lambda) s) - (1-lambda)(k = k1_t ? v2_t : v1_t).
// (Keeping an offset gamma = r - (alpha s - beta) instead would cancel two
// large terms in rows whose argmax column has a large availability.)  State
// for R_t lives in parity t & 1 of the state arrays.
constexpr int IMP_K = 16;            // list capacity per row
enum ImpKind : int { IMP_FULL = 0, IMP_PRO_COLD = 1, IMP_PRO_WARM = 2 };

struct ImpArgs {
    const float *S;
    float *A;
    int64_t ld;
    int32_t n;
    float lam;
    const float *tcol, *ccol;   // column vectors of R_t (full passes)
    float *partial;             // [gridDim.x][ldp] partials of max(0, R_{t+1})
    int64_t ldp;
    float *rdiag;               // r_{t+1}(k,k)
    int32_t *dec;
    uint8_t *eflag;
    ApState *st;                // iteration counter, frozen flag, overflow flag
    char *state;                // row state, two parities of `stride` bytes each (ImpLayout)
    int64_t stride;
    float *Rx[2];               // R_{t+1} rows written explicitly on list overflow, by parity of t+1
    int32_t kmax;               // list capacity in use (<= IMP_K)
    int32_t prologue;           // 1: the t = 0 pass (alpha_0 = 0, alpha_1 from st)
    int64_t row_begin, row_end;
    // Implicit availabilities (k_row_ia only), see XLayout.
    const float *acol[2];       // acol_t by parity of t
    const float *adiag[2];      // adiag_t by parity of t
    char *xstate;               // exception lists, two parities of `xstride` bytes
    int64_t xstride;
    int32_t xcap;               // list capacity in use (<= IMP_KA)
    // Block-diagonal warm start (PAP's Step 4, implicit A): A holds A_0 = A'
    // (zero outside the diagonal blocks, read only), row i's block is the
    // column range [blk[2i], blk[2i+1]); an element whose responsibility was
    // never positive has a_t = acol_t(k) + lambda^t a_0(i,k).  Null: A_0 = 0.
    const int32_t *blk;
    int32_t lean;               // 1: rows with a certified threshold take the lean scan
    int64_t part0;              // first partial row of this launch (row panels of one pass)
};
// Implicit availabilities.  With A_0 = 0, Eq. (3) with damping gives every
// off-diagonal element (i,k) whose responsibility r_s(i,k) was never positive
// (s <= t) the same value acol_t(k) = lam acol_{t-1}(k) + (1-lam) min(0, t_k),
// and Eq. (4) gives the diagonal adiag_t(k) = lam adiag_{t-1}(k) + (1-lam) c_k:
// both are column vectors.  The other elements (the columns where row i ever
// had a positive responsibility) are kept per row as a list of (column,
// value): the exceptions.  The list of A_t lives in parity t & 1.
constexpr int IMP_KA = 1024;         // exception list capacity per row
struct XLayout {
    int64_t cnt, col, val, stride;
};
// cnt (n ints, -1 after an overflow), columns (n x IMP_KA), values (n x IMP_KA).
__host__ __device__ inline XLayout x_layout(int64_t n) {
    const int64_t a = (4 * n + 255) & ~int64_t(255), b = (4 * n * IMP_KA + 255) & ~int64_t(255);
    XLayout L{};
    L.cnt = 0;
    L.col = a;
    L.val = a + b;
    L.stride = a + 2 * b;
    return L;
}
// Byte layout of one parity of the implicit-R state for n rows: beta (n
// floats), list length (n ints, -1 after an overflow), columns (n x IMP_K
// ints), the listed columns' r values (n x IMP_K floats, field `gam`).
struct ImpLayout {
    int64_t beta, cnt, col, gam, stride;
};
// Each part starts on a 256-byte boundary.
__host__ __device__ inline ImpLayout imp_layout(int64_t n) {
    const int64_t a = (4 * n + 255) & ~int64_t(255), b = (4 * n * IMP_K + 255) & ~int64_t(255);
    ImpLayout L{};
    L.beta = 0;
    L.cnt = a;
    L.col = 2 * a;
    L.gam = 2 * a + b;
    L.stride = 2 * a + 2 * b;
    return L;
}
// Plan of the implicit pass for n (same row -> workgroup map as plan_pass);
// false when no implicit variant is instantiated for n.
bool imp_plan(int64_t n, int num_cus, PassPlan *pl);
hipError_t launch_row_imp(const PassPlan &pl, int kind, const ImpArgs &a, hipStream_t s);
// R (rows of the implicit state) = alpha_t S - beta 1^T + gamma; rows whose
// state is -1 (overflowed) are left alone.
hipError_t launch_imp_materialize(const float *S, float *R, int64_t ld, int32_t n, const float *alpha,
                                  const char *state_parity, hipStream_t s);
// Plan of the pass with implicit R and A (cold start); false when n has no
// instantiated variant or its LDS does not fit.
bool ia_plan(int64_t n, int num_cus, PassPlan *pl);
hipError_t launch_row_ia(const PassPlan &pl, const ImpArgs &a, hipStream_t s);
// A = acol off the diagonal, adiag on it, then the row's exceptions; rows
// whose list is -1 (overflowed: written by the pass) are left alone.
hipError_t launch_ia_materialize(float *A, int64_t ld, int32_t n, const float *acol, const float *adiag,
                                 const char *x_parity, hipStream_t s, const int32_t *blk = nullptr,
                                 float lam = 0.0f, int32_t t = 0);
// adiag[k] = A(k,k)
hipError_t launch_extract_diag(const float *A, int64_t ld, int32_t n, float *adiag, hipStream_t s);
// Clears the frozen and overflow flags after an overflow hand-over.
hipError_t launch_state_resume(ApState *st, hipStream_t s);

// Finalize: labels and FP64 dpsim / expref.
struct FinalArgs {
    const float *S;
    int64_t ld;
    int32_t n;
    const uint8_t *eflag;
    int32_t *ex;        // exemplar list scratch (n)
    int32_t *nex;       // device count
    int32_t *idx;       // labels out
    double *contrib;    // 2n scratch
    double *sums;       // [dpsim, expref]
    const int32_t *raw; // nullable: raw decisions to use as the labels
    int64_t row0, row1; // labels of rows [row0, row1) only (row1 = 0: all rows)
};
hipError_t launch_finalize(const FinalArgs &a, hipStream_t s);
// The finalize steps one by one (labels of one row panel at a time).
hipError_t launch_compact(const FinalArgs &a, hipStream_t s);
hipError_t launch_labels(const FinalArgs &a, hipStream_t s);
hipError_t launch_sum2(const FinalArgs &a, hipStream_t s);

// Autotuned choices for one problem-size bucket (see tune.hip).
struct TuneEntry {
    int64_t bucket;
    int64_t n;          // size it was measured at
    int threads;        // row-pass workgroup size
    int lds;            // 1: LDS-resident variant
    int check_every;    // host poll interval of the stop flag
    double ms_per_iter; // measured (row pass + column reduce)
    // message form of cold starts (apx_autotune_form): 0 = size thresholds,
    // APX_FORM_EXPLICIT / _IMPLICIT_R / _IMPLICIT_RA; measured ms per
    // iteration of each form (0 = not measured)
    int form = 0;
    double form_ms[3] = {0.0, 0.0, 0.0};
};
int64_t tune_bucket(int64_t n);
// Tuned plan of the persistent batched launch for batches of one shape
// (bit lengths of the instance count and of the largest n).
struct BatchTune {
    int32_t count_bits, n_bits;
    int32_t wpc;        // workgroups per compute unit
    int32_t min_rows;   // fewest rows per team member
    double ms;          // measured time of the timed iterations
};

}  // namespace apx

// Context ------------------------------------------------------------------
struct apx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    std::string err;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_external = false; // ws belongs to the caller (apx_set_workspace): never grown
    int32_t *dflag = nullptr; // small device buffer of the context (finite checks)
    void *scratch = nullptr;  // this device's fixed scratch array (ap_iterate_noalloc)
    size_t ws_base = 0;       // start of the slice handed to the running solver
    void *pinned = nullptr;   // small pinned host buffer for state read-back
    // hipGraph replay of the iteration loop: one captured chunk of
    // (row pass, column reduce) pairs, re-captured when its arguments change
    bool graphs = true;
    hipStream_t cap = nullptr;        // private stream the graph runs on
    hipEvent_t join = nullptr;        // orders the private stream after `stream`
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey[16] = {};
    // implicit responsibilities: list capacity in use (0 = explicit R only)
    int implicit_k = apx::IMP_K;
    int64_t implicit_min_n = 8192;    // smaller problems run explicit R (faster there)
    int32_t last_imp_iters = 0;       // iterations of the last ap_solve run with implicit R
    int32_t last_exp_iters = 0;       // ... and with explicit R
    int implicit_a = apx::IMP_KA;     // implicit-A exception list capacity (0 = explicit A)
    int64_t implicit_a_min_n = 4096;  // smaller cold starts run explicit (faster there)
    int32_t last_ia_iters = 0;        // iterations of the last ap_solve run with implicit A
    int32_t last_fallback = 0;        // why the last ap_solve left an implicit form (imp_abort bits)
    bool lean = true;                 // lean scan in the implicit-A pass (off: every row forms r)
    int32_t last_lean_rescans = 0;    // rows of the last ap_solve whose ordinary columns decided
    // autotuner (tune.hip)
    bool autotune = false;            // tune unseen size buckets on first use
    int force_form = 0;               // form timing in progress: the form every solve uses
    // PAP's Step 4 (pap_solve -> ap_solve with APX_WARM_A): per row, the
    // column range of its diagonal block of A' (device, 2n int32), set for
    // the duration of that call; ia_blk: the same while the implicit-A
    // passes of a solve use it
    const int32_t *warm_blk = nullptr;
    const int32_t *ia_blk = nullptr;
    std::vector<apx::BatchTune> btune;  // tuned batched plans (apx_autotune_batched)
    int force_bwpc = 0, force_bmin = 0;   // batched plan timing in progress
    std::vector<apx::TuneEntry> tune;
    // benchmark timing of full row passes (apx_profile)
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
};

namespace apx {

// Bump allocator over the context workspace (256-byte aligned slices).
struct WsLayout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    }
};

// Grow the workspace to at least `bytes` (contents are lost when it grows:
// callers that keep data in [0, ws_base) reserve the total first).
apx_status ws_reserve(apx_ctx *ctx, size_t bytes);

// One instance of a batched solve (device pointers; ld >= n, ld % 4 == 0).
struct BatchSpec {
    int64_t n, ld;
    const float *S;
    float *R, *A;
    int32_t *idx;
};
size_t batched_ws_bytes(int32_t count, const BatchSpec *spec, int num_cus);
// Workspace bytes of the other calls (apx_workspace_size).
size_t similarity_ws_bytes(int64_t n);
// Matrix-free S (similarity.hip): rows of S rebuilt from X one panel at a
// time, each entry with the value ap_similarity stores.
struct MfSim {
    const float *X;
    int64_t n, d, ldx;
    int32_t pref_mode;
    const float *pref_vec;
    float pref_scalar;
    uint64_t seed;
    double noise_rel;
    char *ws;   // mf_sim_bytes(n) of device scratch
};
size_t mf_sim_bytes(int64_t n);
hipError_t mf_sim_setup(const MfSim &m, float *panel, int64_t ld, int64_t prows, hipStream_t s);
hipError_t mf_sim_panel(const MfSim &m, float *panel, int64_t ld, int64_t p0, int64_t p1, const ApState *st,
                        hipStream_t s);
const double *mf_sim_pref(const MfSim &m);       // device: the scalar preference
const uint32_t *mf_sim_bounds(const MfSim &m);   // device: bounds of the off-diagonal keys
size_t pap_ws_bytes(int64_t n, int64_t ld, int32_t k, const int64_t *sizes, int num_cus);
size_t lap_ws_bytes(int64_t n, int64_t d, int64_t L, int num_cus);
size_t lap_full_ws_bytes(int64_t n, int64_t d, int64_t L, int64_t m0, int num_cus);
size_t features_ws_bytes(int64_t n);
size_t mlp_backward_ws_bytes(int64_t count);
size_t warmstart_ws_bytes(int64_t n, int64_t ld, int num_cus);
// APX_EINVAL (with a message) if any entry of the n x n matrix M is not
// finite; synchronises the context stream.
apx_status check_finite(apx_ctx *ctx, const float *M, int64_t n, int64_t ld, const char *name);
// Validates apx_params (damping, counts, flags, msg_tol).
apx_status check_params(apx_ctx *ctx, const apx_params *p);
apx_status batched_solve(apx_ctx *ctx, int32_t count, const BatchSpec *spec, int32_t warm,
                         const apx_params *params, apx_result *res);
// Single-instance solve on the workspace slice starting at ctx->ws_base.
size_t solve_ws_bytes(int64_t n, int64_t ld, int num_cus);
// R := the undamped responsibility update of Eq. (2) computed from (S, A),
// i.e. r(i,k) = s(i,k) - max_{k' != k} (a(i,k') + s(i,k')); R's previous
// contents are not used.  Workspace slice at ctx->ws_base.
apx_status resp_step(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A);
size_t resp_step_ws_bytes(int64_t n, int64_t ld, int num_cus);
apx_status set_err(apx_ctx *ctx, apx_status st, const char *fmt, ...);
// Row-pass plan for n on this context: the default plan with the tuned
// workgroup size and variant applied (tuning first if enabled and unseen);
// *check_every (nullable) receives the tuned poll interval or 0.
apx_status ctx_plan(apx_ctx *ctx, int64_t n, PassPlan *pl, int *check_every, bool may_tune = true,
                    int *form = nullptr);
// ap_iterate's argument checks, and its launches (column vectors t, c,
// r(k,k) and the partials [pl.grid][round4(n)] in caller-given memory).
apx_status check_iterate(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, const float *R, const float *A,
                         float damping, int32_t n_iter);
hipError_t iterate_passes(const PassPlan &pl, const float *S, int64_t n, int64_t ld, float *R, float *A,
                          float lam, int32_t n_iter, int32_t *decision, float *tcol, float *ccol, float *rdiag,
                          float *partial, hipStream_t s);
// Looks up this device's copy of the fixed scratch array of
// ap_iterate_noalloc (noalloc.hip); called by apx_create with the device current.
apx_status noalloc_init(apx_ctx *ctx);
apx_status hip_err(apx_ctx *ctx, hipError_t e, const char *what);

}  // namespace apx
