// api.hip -- C ABI entry points: context, validation, workspace, and the
// host side of the AP iteration loop (Algorithm 1, Section 2).
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "apx_internal.h"

using namespace apx;

namespace apx {

apx_status set_err(apx_ctx *ctx, apx_status st, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

apx_status hip_err(apx_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return APX_OK;
    if (e == hipErrorOutOfMemory)
        return set_err(ctx, APX_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return set_err(ctx, APX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

apx_status ws_reserve(apx_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return APX_OK;
    if (ctx->ws_external)
        return set_err(ctx, APX_ENOMEM, "the call needs %zu bytes of workspace; apx_set_workspace set %zu",
                       bytes, ctx->ws_bytes);
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_err(ctx, e, "workspace sync");
    if (ctx->ws) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t want = bytes + (bytes >> 3);   // grow with slack
    e = hipMalloc(&ctx->ws, want);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        (void)hipGetLastError();
        return set_err(ctx, APX_ENOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
    }
    ctx->ws_bytes = want;
    return APX_OK;
}

apx_status check_params(apx_ctx *ctx, const apx_params *p) {
    if (!p) return set_err(ctx, APX_EINVAL, "params is null");
    if (!(p->damping >= 0.0f && p->damping < 1.0f)) return set_err(ctx, APX_EINVAL, "damping must be in [0,1)");
    if (p->max_iter < 1 || p->conv_iter < 0)
        return set_err(ctx, APX_EINVAL, "max_iter must be >= 1 and conv_iter >= 0");
    if (p->flags & ~(uint32_t)(APX_RAW_LABELS | APX_CHECK_FINITE | APX_MSG_THRESHOLD))
        return set_err(ctx, APX_EINVAL, "unknown flags 0x%x", p->flags);
    if ((p->flags & APX_MSG_THRESHOLD) && !(p->msg_tol >= 0.0f && std::isfinite(p->msg_tol)))
        return set_err(ctx, APX_EINVAL, "msg_tol must be finite and >= 0");
    return APX_OK;
}

apx_status check_finite(apx_ctx *ctx, const float *M, int64_t n, int64_t ld, const char *name) {
    hipStream_t s = ctx->stream;
    hipError_t e = launch_fill_u8(reinterpret_cast<uint8_t *>(ctx->dflag), sizeof(int32_t), 0, s);
    if (e == hipSuccess) e = launch_check_finite(M, n, n, ld, ctx->dflag, s);
    int32_t *h = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 2048);
    if (e == hipSuccess) e = hipMemcpyAsync(h, ctx->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "finite check");
    if (*h) return set_err(ctx, APX_EINVAL, "%s holds a NaN or infinite entry", name);
    return APX_OK;
}

}  // namespace apx

#define APX_TRY(expr)                       \
    do {                                    \
        apx_status _st = (expr);            \
        if (_st != APX_OK) return _st;      \
    } while (0)
#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)

namespace {

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

apx_status check_matrix(apx_ctx *ctx, const void *M, const char *name, int64_t n, int64_t ld) {
    if (M == nullptr) return set_err(ctx, APX_EINVAL, "%s is null", name);
    if (!aligned16(M)) return set_err(ctx, APX_EINVAL, "%s is not 16-byte aligned", name);
    if (ld < n) return set_err(ctx, APX_EINVAL, "ld (%lld) < n (%lld)", (long long)ld, (long long)n);
    if (ld % 4 != 0) return set_err(ctx, APX_EINVAL, "ld (%lld) is not a multiple of 4", (long long)ld);
    return APX_OK;
}

int64_t round4(int64_t v) { return (v + 3) & ~int64_t(3); }

// Workspace of one AP run on an n x n problem.
struct IterWs {
    float *tcol, *ccol, *rdiag, *partial;
    int64_t ldp;
    int nparts;
    int32_t *dec;
    uint8_t *eflag;
    ApState *st;
    float *R2;            // second responsibility buffer (ap_solve)
    char *imp;            // implicit-R state, two parities (ap_solve)
    int64_t imp_stride;
    float *acol[2], *adiag[2];   // implicit-A column vectors by parity (ap_solve)
    char *xst;            // implicit-A exception lists, two parities
    int64_t xstride;
    int32_t *ex, *nex;
    double *contrib, *sums;
};

struct IterLayout {
    size_t o_t, o_c, o_d, o_p, o_dec, o_e, o_st, o_ex, o_nex, o_con, o_sum, o_r2, o_imp, o_acol, o_x, bytes;
};

IterLayout iter_layout(int64_t n, int64_t ld, bool second_r, int grid) {
    IterLayout o{};
    WsLayout L;
    const int64_t ldp = round4(n);
    o.o_t = L.take(sizeof(float) * ldp);
    o.o_c = L.take(sizeof(float) * ldp);
    o.o_d = L.take(sizeof(float) * ldp);
    o.o_p = L.take(sizeof(float) * ldp * (size_t)grid);
    o.o_dec = L.take(sizeof(int32_t) * n);
    o.o_e = L.take((size_t)n);
    o.o_st = L.take(sizeof(ApState));
    o.o_ex = L.take(sizeof(int32_t) * n);
    o.o_nex = L.take(sizeof(int32_t));
    o.o_con = L.take(sizeof(double) * 2 * (size_t)n);
    o.o_sum = L.take(sizeof(double) * 2);
    o.o_r2 = second_r ? L.take(sizeof(float) * (size_t)n * (size_t)ld) : 0;
    o.o_imp = second_r ? L.take(2 * (size_t)imp_layout(n).stride) : 0;
    o.o_acol = second_r ? L.take(4 * sizeof(float) * (size_t)ldp) : 0;
    o.o_x = second_r ? L.take(2 * (size_t)x_layout(n).stride) : 0;
    o.bytes = L.off;
    return o;
}

// Workspace of one AP run on an n x n problem, carved from ctx->ws_base.
apx_status iter_ws(apx_ctx *ctx, int64_t n, int64_t ld, bool second_r, const PassPlan &pl, IterWs &w) {
    const IterLayout o = iter_layout(n, ld, second_r, pl.grid);
    APX_TRY(ws_reserve(ctx, ctx->ws_base + o.bytes));
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;
    w.tcol = reinterpret_cast<float *>(b + o.o_t);
    w.ccol = reinterpret_cast<float *>(b + o.o_c);
    w.rdiag = reinterpret_cast<float *>(b + o.o_d);
    w.partial = reinterpret_cast<float *>(b + o.o_p);
    w.ldp = round4(n);
    w.nparts = pl.grid;
    w.dec = reinterpret_cast<int32_t *>(b + o.o_dec);
    w.eflag = reinterpret_cast<uint8_t *>(b + o.o_e);
    w.st = reinterpret_cast<ApState *>(b + o.o_st);
    w.ex = reinterpret_cast<int32_t *>(b + o.o_ex);
    w.nex = reinterpret_cast<int32_t *>(b + o.o_nex);
    w.contrib = reinterpret_cast<double *>(b + o.o_con);
    w.sums = reinterpret_cast<double *>(b + o.o_sum);
    w.R2 = second_r ? reinterpret_cast<float *>(b + o.o_r2) : nullptr;
    w.imp = second_r ? b + o.o_imp : nullptr;
    w.imp_stride = imp_layout(n).stride;
    for (int q = 0; q < 2; ++q) {
        w.acol[q] = second_r ? reinterpret_cast<float *>(b + o.o_acol) + q * w.ldp : nullptr;
        w.adiag[q] = second_r ? reinterpret_cast<float *>(b + o.o_acol) + (2 + q) * w.ldp : nullptr;
    }
    w.xst = second_r ? b + o.o_x : nullptr;
    w.xstride = x_layout(n).stride;
    return APX_OK;
}

PassArgs pass_args(const float *S, const float *Rin, float *Rout, float *A, int64_t n, int64_t ld,
                   float lam, const IterWs &w, int32_t *dec, uint8_t *eflag, ApState *st) {
    PassArgs a{};
    a.S = S;
    a.Rin = Rin;
    a.Rout = Rout;
    a.A = A;
    a.ld = ld;
    a.n = (int32_t)n;
    a.lam = lam;
    a.tcol = w.tcol;
    a.ccol = w.ccol;
    a.partial = w.partial;
    a.ldp = w.ldp;
    a.rdiag = w.rdiag;
    a.dec = dec;
    a.eflag = eflag;
    a.st = st;
    a.row_begin = 0;
    a.row_end = n;
    return a;
}

// Implicit pass (state R_t in parity t & 1, t from the run state); the
// prologue is the t = 0 pass.
ImpArgs imp_args(const float *S, float *A, int64_t n, int64_t ld, float lam, const IterWs &w,
                 float *const buf[2], bool prologue, int kmax, int xcap = 0) {
    ImpArgs a{};
    for (int q = 0; q < 2; ++q) {
        a.acol[q] = w.acol[q];
        a.adiag[q] = w.adiag[q];
    }
    a.xstate = w.xst;
    a.xstride = w.xstride;
    a.xcap = xcap;
    a.S = S;
    a.A = A;
    a.ld = ld;
    a.n = (int32_t)n;
    a.lam = lam;
    a.tcol = w.tcol;
    a.ccol = w.ccol;
    a.partial = w.partial;
    a.ldp = w.ldp;
    a.rdiag = w.rdiag;
    a.dec = prologue ? nullptr : w.dec;
    a.eflag = prologue ? nullptr : w.eflag;
    a.st = w.st;
    a.state = w.imp;
    a.stride = w.imp_stride;
    a.Rx[0] = buf[0];
    a.Rx[1] = buf[1];
    a.kmax = kmax;
    a.prologue = prologue ? 1 : 0;
    a.row_begin = 0;
    a.row_end = n;
    return a;
}

// ia_pass >= 0: the reduce after implicit-A pass ia_pass (0 = prologue) also
// advances the availability column vectors to iteration ia_pass + 1.
ColArgs col_args(const IterWs &w, int64_t n, ApState *st, int bookkeep, int32_t ia_pass = -1, float lam = 0.0f) {
    ColArgs c{};
    if (ia_pass >= 0) {
        c.acol_in = w.acol[ia_pass & 1];
        c.adiag_in = w.adiag[ia_pass & 1];
        c.acol_out = w.acol[(ia_pass + 1) & 1];
        c.adiag_out = w.adiag[(ia_pass + 1) & 1];
        c.lam = lam;
    }
    c.partial = w.partial;
    c.ldp = w.ldp;
    c.nparts = w.nparts;
    c.rdiag = w.rdiag;
    c.tcol = w.tcol;
    c.ccol = w.ccol;
    c.n = (int32_t)n;
    c.st = st;
    c.bookkeep = bookkeep;
    return c;
}

}  // namespace

namespace {

// How ap_solve keeps the messages: both explicit; R implicit (ImpArgs);
// R and A implicit (XLayout, cold start).
// SOLVE_EXPLICIT_DELTA: explicit, recording the message changes of each pass.
enum SolveMode : int { SOLVE_EXPLICIT = 0, SOLVE_IMPLICIT_R = 1, SOLVE_IMPLICIT_A = 2, SOLVE_EXPLICIT_DELTA = 3 };

// Runs iterations t0 .. t0+chunk-1 of ap_solve as one replay of a captured
// graph on the context's private stream, ordered after everything already
// enqueued on ctx->stream, then copies the run state to the host and waits.
// Returns APX_ENOTIMPL (and leaves nothing enqueued) when the capture itself
// fails, so that the caller can run the chunk with plain launches.
apx_status graph_chunk(apx_ctx *ctx, const PassPlan &pl, int mode, const float *S, float *const buf[2],
                       float *A, int64_t n, int64_t ld, float lam, const IterWs &w, int chunk, int32_t t0,
                       ApState *hst) {
    if (!ctx->cap) {
        HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking), "graph stream");
        HIP_TRY(hipEventCreateWithFlags(&ctx->join, hipEventDisableTiming), "graph event");
    }
    uint32_t lam_bits;
    std::memcpy(&lam_bits, &lam, sizeof lam_bits);
    const uint64_t key[16] = {(uint64_t)(uintptr_t)S, (uint64_t)(uintptr_t)buf[0], (uint64_t)(uintptr_t)buf[1],
                              (uint64_t)(uintptr_t)A, (uint64_t)n, (uint64_t)ld, lam_bits, (uint64_t)chunk,
                              (uint64_t)(t0 & 1) | (uint64_t)(uintptr_t)ctx->ia_blk, (uint64_t)(uintptr_t)w.st,
                              (uint64_t)(uintptr_t)w.partial,
                              (uint64_t)(uintptr_t)w.tcol, (uint64_t)(uintptr_t)w.imp,
                              (uint64_t)pl.grid | ((uint64_t)mode << 32) | ((uint64_t)ctx->implicit_k << 40) |
                                  ((uint64_t)ctx->implicit_a << 48),
                              (uint64_t)pl.threads | ((uint64_t)ctx->lean << 32) | ((uint64_t)pl.two_sweep << 33),
                              (uint64_t)pl.lds_bytes};
    if (!ctx->gexec || std::memcmp(key, ctx->gkey, sizeof key) != 0) {
        if (ctx->gexec) {
            (void)hipGraphExecDestroy(ctx->gexec);
            ctx->gexec = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed), "begin capture");
        hipError_t e = hipSuccess;
        for (int u = 0; u < chunk && e == hipSuccess; ++u) {
            const int32_t t = t0 + u;
            if (mode == SOLVE_IMPLICIT_A) {
                ImpArgs ia = imp_args(S, A, n, ld, lam, w, buf, false, ctx->implicit_k, ctx->implicit_a);
                ia.blk = ctx->ia_blk;
                ia.lean = ctx->lean ? 1 : 0;
                e = launch_row_ia(pl, ia,
                                  ctx->cap);
            } else if (mode == SOLVE_IMPLICIT_R) {
                e = launch_row_imp(pl, IMP_FULL, imp_args(S, A, n, ld, lam, w, buf, false, ctx->implicit_k),
                                   ctx->cap);
            } else {
                PassArgs pf = pass_args(S, buf[t & 1], buf[(t + 1) & 1], A, n, ld, lam, w, w.dec, w.eflag, w.st);
                e = launch_row_pass(pl, mode == SOLVE_EXPLICIT_DELTA ? PASS_FULL_DELTA : PASS_FULL, pf, ctx->cap);
            }
            if (e == hipSuccess)
                e = launch_col_reduce(col_args(w, n, w.st, 1, mode == SOLVE_IMPLICIT_A ? t : -1, lam), ctx->cap);
        }
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
        if (e == hipSuccess && e2 == hipSuccess && g != nullptr)
            e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess || e2 != hipSuccess || ctx->gexec == nullptr) {
            ctx->gexec = nullptr;
            (void)hipGetLastError();
            return APX_ENOTIMPL;
        }
        std::memcpy(ctx->gkey, key, sizeof key);
    }
    HIP_TRY(hipEventRecord(ctx->join, ctx->stream), "join");
    HIP_TRY(hipStreamWaitEvent(ctx->cap, ctx->join, 0), "join");
    HIP_TRY(hipGraphLaunch(ctx->gexec, ctx->cap), "graph launch");
    HIP_TRY(hipMemcpyAsync(hst, w.st, sizeof(ApState), hipMemcpyDeviceToHost, ctx->cap), "state");
    HIP_TRY(hipStreamSynchronize(ctx->cap), "sync");
    return APX_OK;
}

}  // namespace

namespace apx {
apx_status check_iterate(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, const float *R, const float *A,
                         float damping, int32_t n_iter) {
    if (!ctx) return APX_EINVAL;
    if (n < 2) return set_err(ctx, APX_EINVAL, "ap_iterate needs n >= 2 (n = %lld)", (long long)n);
    if (n > kMaxSolveN) return set_err(ctx, APX_ENOTIMPL, "n = %lld exceeds %lld", (long long)n, (long long)kMaxSolveN);
    APX_TRY(check_matrix(ctx, S, "S", n, ld));
    APX_TRY(check_matrix(ctx, R, "R", n, ld));
    APX_TRY(check_matrix(ctx, A, "A", n, ld));
    if (!(damping >= 0.0f && damping < 1.0f)) return set_err(ctx, APX_EINVAL, "damping must be in [0,1)");
    if (n_iter < 1) return set_err(ctx, APX_EINVAL, "n_iter must be >= 1");
    return APX_OK;
}

hipError_t iterate_passes(const PassPlan &pl, const float *S, int64_t n, int64_t ld, float *R, float *A,
                          float lam, int32_t n_iter, int32_t *decision, float *tcol, float *ccol, float *rdiag,
                          float *partial, hipStream_t s) {
    IterWs w{};
    w.tcol = tcol;
    w.ccol = ccol;
    w.rdiag = rdiag;
    w.partial = partial;
    w.ldp = round4(n);
    w.nparts = pl.grid;
    // R_{t+1} from (R_t, S, A_t), in place, with its column vectors.
    PassArgs pa = pass_args(S, R, R, A, n, ld, lam, w, nullptr, nullptr, nullptr);
    hipError_t e = launch_row_pass(pl, PASS_R_ONLY, pa, s);
    if (e == hipSuccess) e = launch_col_reduce(col_args(w, n, nullptr, 0), s);
    for (int32_t it = 1; it < n_iter && e == hipSuccess; ++it) {
        PassArgs pf = pass_args(S, R, R, A, n, ld, lam, w, nullptr, nullptr, nullptr);
        e = launch_row_pass(pl, PASS_FULL, pf, s);
        if (e == hipSuccess) e = launch_col_reduce(col_args(w, n, nullptr, 0), s);
    }
    if (e == hipSuccess) {
        PassArgs pe = pass_args(S, R, R, A, n, ld, lam, w, decision, nullptr, nullptr);
        e = launch_row_pass(pl, PASS_A_ONLY, pe, s);
    }
    return e;
}

size_t solve_ws_bytes(int64_t n, int64_t ld, int num_cus) {
    const PassPlan pl = plan_pass(n, num_cus);
    return iter_layout(n, ld, true, pl.grid).bytes;
}

size_t resp_step_ws_bytes(int64_t n, int64_t ld, int num_cus) {
    const PassPlan pl = plan_pass(n, num_cus);
    return iter_layout(n, ld, false, pl.grid).bytes;
}

apx_status resp_step(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A) {
    PassPlan pl{};
    APX_TRY(ctx_plan(ctx, n, &pl, nullptr));
    IterWs w{};
    APX_TRY(iter_ws(ctx, n, ld, false, pl, w));
    hipStream_t s = ctx->stream;
    // With damping 0 and R = 0 the responsibility pass computes
    // 0 * 0 + 1 * s(i,k) - 1 * max(...) exactly: the plain update of Eq. (2).
    HIP_TRY(launch_fill_f32_rows(R, n, n, ld, 0.0f, s), "R = 0");
    PassArgs pa = pass_args(S, R, R, A, n, ld, 0.0f, w, nullptr, nullptr, nullptr);
    HIP_TRY(launch_row_pass(pl, PASS_R_ONLY, pa, s), "responsibility step");
    return APX_OK;
}
}  // namespace apx

extern "C" {

apx_status apx_create(apx_ctx **out, int device, void *hip_stream) {
    if (out == nullptr) return APX_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return APX_EDEVICE;
    apx_ctx *ctx = new (std::nothrow) apx_ctx();
    if (!ctx) return APX_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    DevGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    if (hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return APX_ENOMEM;
    }
    if (hipMalloc(&ctx->dflag, 256) != hipSuccess) {
        (void)hipHostFree(ctx->pinned);
        delete ctx;
        return APX_ENOMEM;
    }
    // this device's fixed scratch array (ap_iterate_noalloc reports its absence)
    (void)noalloc_init(ctx);
    const char *gv = getenv("APX_GRAPHS");
    if (gv && gv[0] == '0') ctx->graphs = false;
    const char *iv = getenv("APX_IMPLICIT_K");
    if (iv && iv[0]) {
        const int k = atoi(iv);
        ctx->implicit_k = k < 0 ? 0 : (k > IMP_K ? IMP_K : k);
    }
    const char *xv = getenv("APX_IMPLICIT_A");
    if (xv && xv[0]) {
        const int k = atoi(xv);
        ctx->implicit_a = k < 0 ? 0 : (k > IMP_KA ? IMP_KA : k);
    }
    const char *av = getenv("APX_AUTOTUNE");
    if (av && av[0] == '1') ctx->autotune = true;
    const char *tf = getenv("APX_TUNE_FILE");
    if (tf && tf[0]) (void)apx_tune_load(ctx, tf);   // a missing or foreign file leaves the defaults
    ctx->err.clear();
    *out = ctx;
    return APX_OK;
}

void apx_destroy(apx_ctx *ctx) {
    if (!ctx) return;
    DevGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->cap) {
        (void)hipStreamSynchronize(ctx->cap);
        (void)hipStreamDestroy(ctx->cap);
    }
    if (ctx->join) (void)hipEventDestroy(ctx->join);
    if (ctx->ws && !ctx->ws_external) (void)hipFree(ctx->ws);
    if (ctx->dflag) (void)hipFree(ctx->dflag);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

apx_status apx_set_workspace(apx_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx) return APX_EINVAL;
    if (dev_ptr && (reinterpret_cast<uintptr_t>(dev_ptr) & 255u) != 0)
        return set_err(ctx, APX_EINVAL, "workspace must be 256-byte aligned");
    DevGuard g(ctx->device);
    HIP_TRY(hipStreamSynchronize(ctx->stream), "workspace sync");
    if (ctx->ws && !ctx->ws_external) (void)hipFree(ctx->ws);
    ctx->ws = dev_ptr;
    ctx->ws_bytes = dev_ptr ? bytes : 0;
    ctx->ws_external = dev_ptr != nullptr;
    ctx->ws_base = 0;
    return APX_OK;
}

namespace {
struct MfShape {
    int64_t ld, P, Q;
    int gmax;
    PassPlan ipl, apl;
};
bool mf_shape(int64_t n, int64_t panel_rows, int num_cus, MfShape *sh);
size_t mf_bytes(int64_t n, const MfShape &sh);
}  // namespace

size_t apx_workspace_size(const apx_ctx *ctx, int32_t op, int64_t n, int64_t ld, int64_t d, int32_t count,
                          const int64_t *sizes) {
    if (!ctx) return 0;
    const int cus = ctx->num_cus;
    switch (op) {
    case APX_OP_SIMILARITY:
        return n >= 2 ? similarity_ws_bytes(n) : 0;
    case APX_OP_ITERATE:
        return (n >= 2 && ld >= n) ? resp_step_ws_bytes(n, ld, cus) : 0;
    case APX_OP_SOLVE:
        return (n >= 1 && ld >= n) ? solve_ws_bytes(n, ld, cus) : 0;
    case APX_OP_SOLVE_BATCHED: {
        if (count < 1 || !sizes) return 0;
        std::vector<BatchSpec> spec(count);
        for (int j = 0; j < count; ++j) {
            if (sizes[j] < 2) return 0;
            spec[j] = BatchSpec{sizes[j], round4(sizes[j]), nullptr, nullptr, nullptr, nullptr};
        }
        return batched_ws_bytes(count, spec.data(), cus);
    }
    case APX_OP_PAP:
        return (n >= 2 && ld >= n && count >= 1 && count <= n) ? pap_ws_bytes(n, ld, count, sizes, cus) : 0;
    case APX_OP_LAP:
        return (n >= 2 && d >= 1 && count >= 2 && count <= n) ? lap_ws_bytes(n, d, count, cus) : 0;
    case APX_OP_FEATURES:
        return n >= 2 ? features_ws_bytes(n) : 0;
    case APX_OP_MLP_BACKWARD:
        return count >= 1 ? mlp_backward_ws_bytes(count) : 0;
    case APX_OP_WARMSTART:
        return (n >= 2 && ld >= n) ? warmstart_ws_bytes(n, ld, cus) : 0;
    case APX_OP_LAP_FULL:
        return (n >= 2 && d >= 1 && count >= 2 && count <= n && ld >= 2) ? lap_full_ws_bytes(n, d, count, ld, cus)
                                                                          : 0;
    case APX_OP_SOLVE_MF: {
        MfShape sh;
        return (count >= 0 && mf_shape(n, count, cus, &sh)) ? mf_bytes(n, sh) : 0;
    }
    default:
        return 0;
    }
}

apx_status apx_set_stream(apx_ctx *ctx, void *hip_stream) {
    if (!ctx) return APX_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return APX_OK;
}

const char *apx_last_error(const apx_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t apx_workspace_bytes(const apx_ctx *ctx) { return ctx ? ctx->ws_bytes : 0; }

apx_status apx_set_implicit(apx_ctx *ctx, int32_t list_capacity, int64_t min_n) {
    if (!ctx) return APX_EINVAL;
    if (list_capacity < 0 || list_capacity > IMP_K)
        return set_err(ctx, APX_EINVAL, "list capacity must be in [0, %d]", IMP_K);
    if (min_n < 0) return set_err(ctx, APX_EINVAL, "min_n < 0");
    ctx->implicit_k = list_capacity;
    ctx->implicit_min_n = min_n;
    return APX_OK;
}

apx_status apx_set_implicit_a(apx_ctx *ctx, int32_t list_capacity, int64_t min_n) {
    if (!ctx) return APX_EINVAL;
    if (list_capacity < 0 || list_capacity > IMP_KA)
        return set_err(ctx, APX_EINVAL, "exception list capacity must be in [0, %d]", IMP_KA);
    if (min_n < 0) return set_err(ctx, APX_EINVAL, "min_n < 0");
    ctx->implicit_a = list_capacity;
    ctx->implicit_a_min_n = min_n;
    return APX_OK;
}

apx_status apx_last_solve_info(apx_ctx *ctx, int32_t *implicit_iters, int32_t *explicit_iters,
                               int32_t *implicit_a_iters) {
    if (!ctx || !implicit_iters || !explicit_iters) return APX_EINVAL;
    *implicit_iters = ctx->last_imp_iters;
    *explicit_iters = ctx->last_exp_iters;
    if (implicit_a_iters) *implicit_a_iters = ctx->last_ia_iters;
    return APX_OK;
}

apx_status apx_last_fallback(apx_ctx *ctx, int32_t *reasons) {
    if (!ctx || !reasons) return APX_EINVAL;
    *reasons = ctx->last_fallback;
    return APX_OK;
}

apx_status apx_set_lean_scan(apx_ctx *ctx, int enable) {
    if (!ctx) return APX_EINVAL;
    ctx->lean = enable != 0;
    return APX_OK;
}

apx_status apx_last_lean_rescans(apx_ctx *ctx, int32_t *rows) {
    if (!ctx || !rows) return APX_EINVAL;
    *rows = ctx->last_lean_rescans;
    return APX_OK;
}

apx_status apx_set_graphs(apx_ctx *ctx, int enable) {
    if (!ctx) return APX_EINVAL;
    ctx->graphs = enable != 0;
    return APX_OK;
}

apx_status apx_profile(apx_ctx *ctx, int enable) {
    if (!ctx) return APX_EINVAL;
    ctx->prof = enable != 0;
    return APX_OK;
}

apx_status apx_profile_read(apx_ctx *ctx, int64_t *launches, double *total_ms) {
    if (!ctx || !launches || !total_ms) return APX_EINVAL;
    *launches = ctx->prof_launches;
    *total_ms = ctx->prof_ms;
    ctx->prof_launches = 0;
    ctx->prof_ms = 0.0;
    return APX_OK;
}

apx_status ap_iterate(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                      float damping, int32_t n_iter, int32_t *decision) {
    APX_TRY(check_iterate(ctx, S, n, ld, R, A, damping, n_iter));
    DevGuard g(ctx->device);
    PassPlan pl{};
    APX_TRY(ctx_plan(ctx, n, &pl, nullptr));
    IterWs w{};
    APX_TRY(iter_ws(ctx, n, ld, false, pl, w));
    HIP_TRY(iterate_passes(pl, S, n, ld, R, A, damping, n_iter, decision, w.tcol, w.ccol, w.rdiag, w.partial,
                           ctx->stream),
            "ap_iterate passes");
    return APX_OK;
}

apx_status ap_solve(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                    int32_t warm, const apx_params *params, int32_t *idx, apx_result *res) {
    if (!ctx) return APX_EINVAL;
    if (n < 1) return set_err(ctx, APX_EINVAL, "n must be >= 1");
    if (n > kMaxSolveN) return set_err(ctx, APX_ENOTIMPL, "n = %lld exceeds %lld", (long long)n, (long long)kMaxSolveN);
    APX_TRY(check_matrix(ctx, S, "S", n, ld));
    APX_TRY(check_matrix(ctx, R, "R", n, ld));
    APX_TRY(check_matrix(ctx, A, "A", n, ld));
    if (!params || !res || !idx) return set_err(ctx, APX_EINVAL, "params, idx and res must be non-null");
    if (warm < APX_COLD || warm > APX_WARM_COLUMNS) return set_err(ctx, APX_EINVAL, "bad warm mode %d", warm);
    APX_TRY(check_params(ctx, params));
    const float lam = params->damping;
    const bool raw_labels = (params->flags & APX_RAW_LABELS) != 0;
    const bool msg_rule = (params->flags & APX_MSG_THRESHOLD) != 0;
    DevGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    if (params->flags & APX_CHECK_FINITE) APX_TRY(check_finite(ctx, S, n, ld, "S"));
    std::memset(res, 0, sizeof *res);

    if (n == 1) {
        // A single point is its own exemplar; Eq. (2) has no other candidate.
        float s00 = 0.0f;
        int32_t *h = static_cast<int32_t *>(ctx->pinned);
        h[0] = 0;
        HIP_TRY(hipMemcpyAsync(idx, h, sizeof(int32_t), hipMemcpyHostToDevice, s), "idx");
        HIP_TRY(hipMemcpyAsync(&h[4], S, sizeof(float), hipMemcpyDeviceToHost, s), "s00");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        std::memcpy(&s00, &h[4], sizeof s00);
        res->iterations = 0;
        res->converged = 1;
        res->n_exemplars = 1;
        res->dpsim = 0.0;
        res->expref = s00;
        res->netsim = s00;
        return APX_OK;
    }

    PassPlan pl{};
    int tuned_chunk = 0, tuned_form = 0;
    APX_TRY(ctx_plan(ctx, n, &pl, &tuned_chunk, true, &tuned_form));
    IterWs w{};
    APX_TRY(iter_ws(ctx, n, ld, true, pl, w));
    const bool cols = warm == APX_WARM_COLUMNS;
    HIP_TRY(launch_state_init(w.st, params->max_iter, params->conv_iter, lam, s, msg_rule ? 1 : 0,
                              params->msg_tol, cols ? 1 : 0), "state init");
    HIP_TRY(launch_fill_u8(w.eflag, n, 0, s), "flags");

    // R_t lives in buf[t & 1]; buf[0] is the caller's R.  With R_0 = 0 (cold
    // start or A_0 only) R is kept implicitly (ImpArgs) unless disabled.
    float *buf[2] = {R, w.R2};
    // Cold start: A is kept implicitly too (XLayout) unless disabled; each
    // form has its own size threshold (below it the explicit pass is faster).
    PassPlan ipl{}, apl{};
    // the message-change rule needs both messages in memory: explicit form
    const bool r_ok = !msg_rule && ctx->implicit_k > 0 && warm != APX_WARM_AR && imp_plan(n, ctx->num_cus, &ipl);
    // PAP's block-diagonal A' (pap_solve sets the blocks): implicit A with
    // the lambda^t a_0 term, 1024-thread passes only (n > 4096)
    const bool wblk = warm == APX_WARM_A && ctx->warm_blk != nullptr && n > 4096;
    const bool ia_start = warm == APX_COLD || cols || wblk;
    bool imp_a = r_ok && ia_start && ctx->implicit_a > 0 && n >= ctx->implicit_a_min_n &&
                 ia_plan(n, ctx->num_cus, &apl);
    bool implicit = r_ok && (imp_a || n >= ctx->implicit_min_n);
    // a tuned (or, while the tuner times forms, forced) message form replaces
    // the size thresholds where the start allows it
    if (tuned_form == APX_FORM_EXPLICIT) {
        imp_a = implicit = false;
    } else if (tuned_form == APX_FORM_IMPLICIT_R) {
        imp_a = false;
        implicit = r_ok;
    } else if (tuned_form == APX_FORM_IMPLICIT_RA) {
        imp_a = r_ok && ia_start && ctx->implicit_a > 0 && ia_plan(n, ctx->num_cus, &apl);
        implicit = r_ok;
    }
    // the implicit-A passes of this solve read A' through its blocks
    struct BlkGuard {
        apx_ctx *c;
        ~BlkGuard() { c->ia_blk = nullptr; }
    } blk_guard{ctx};
    ctx->ia_blk = (imp_a && wblk) ? ctx->warm_blk : nullptr;
    const int32_t *const ia_blk = ctx->ia_blk;
    int32_t imp_until = implicit ? INT32_MAX : 0;   // last iteration run with implicit R
    int32_t ia_until = imp_a ? INT32_MAX : 0;       // last iteration run with implicit A
    int32_t fallback = 0;                           // imp_abort bits of the fallbacks
    if (implicit) {
        // parity 0 holds R_0 = 0: beta = 0 and empty lists
        const ImpLayout il = imp_layout(n);
        HIP_TRY(launch_fill_f32_rows(reinterpret_cast<float *>(w.imp + il.beta), 1, n, n, 0.0f, s),
                "implicit state");
        HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(w.imp + il.cnt), 4 * n, 0, s), "implicit state");
        // R_1: the damped step from R_0 = 0 and A_0; with A_0 column-structured
        // the undamped step (damping 0, alpha_1 = 1 in the run state), which
        // is R_0 itself
        const ImpArgs ia = imp_args(S, A, n, ld, cols ? 0.0f : lam, w, buf, true, ctx->implicit_k);
        HIP_TRY(launch_row_imp(ipl, warm == APX_COLD ? IMP_PRO_COLD : IMP_PRO_WARM, ia, s), "prologue");
        if (imp_a) {
            // A_0 = 0 (or A_0's column vectors): every exception list empty
            HIP_TRY(launch_fill_f32_rows(w.acol[0], 1, w.ldp, w.ldp, 0.0f, s), "implicit A");
            HIP_TRY(launch_fill_f32_rows(w.adiag[0], 1, w.ldp, w.ldp, 0.0f, s), "implicit A");
            if (cols) HIP_TRY(launch_extract_cols(A, ld, (int32_t)n, w.acol[0], w.adiag[0], s), "implicit A");
            // block warm start: acol_0 = 0 (A' enters as lambda^t a_0), adiag_0 = diag(A')
            if (ia_blk) HIP_TRY(launch_extract_diag(A, ld, (int32_t)n, w.adiag[0], s), "implicit A");
            HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(w.xst + x_layout(n).cnt), 4 * n, 0, s),
                    "implicit A");
        } else if (warm == APX_COLD) {
            HIP_TRY(launch_fill_f32_rows(A, n, n, ld, 0.0f, s), "A_0");
        }
    } else {
        PassArgs pr = pass_args(S, R, buf[1], A, n, ld, lam, w, nullptr, nullptr, nullptr);
        if (warm == APX_COLD) {
            // R_1 from R_0 = A_0 = 0, then A_0 = 0 in memory (Eq. (1)).
            HIP_TRY(launch_row_pass(pl, PASS_R_COLD, pr, s), "prologue");
            HIP_TRY(launch_fill_f32_rows(A, n, n, ld, 0.0f, s), "A_0");
        } else if (cols) {
            // R_1 = R_0: the undamped step from A_0 (damping 0 on R = 0)
            HIP_TRY(launch_fill_f32_rows(R, n, n, ld, 0.0f, s), "R_0");
            PassArgs pu = pr;
            pu.lam = 0.0f;
            HIP_TRY(launch_row_pass(pl, PASS_R_ONLY, pu, s), "prologue");
        } else {
            if (warm == APX_WARM_A) HIP_TRY(launch_fill_f32_rows(R, n, n, ld, 0.0f, s), "R_0");
            HIP_TRY(launch_row_pass(pl, PASS_R_ONLY, pr, s), "prologue");
        }
    }
    HIP_TRY(launch_col_reduce(col_args(w, n, nullptr, 0, imp_a ? 0 : -1, lam), s), "column reduce");

    // Host polls every `chunk` iterations (even, so every replay of the
    // captured chunk starts on the same responsibility buffer).  Passes after
    // the stop iteration are no-ops on the device, so results do not depend
    // on the chunk.
    int chunk = params->check_every > 0 ? params->check_every : (tuned_chunk > 0 ? tuned_chunk : 16);
    chunk += chunk & 1;
    // Kernel timing needs events on the host-launched passes (event records
    // captured inside a graph cannot be timed), so timing runs eagerly.
    bool use_graph = ctx->graphs && !ctx->prof;
    if (ctx->prof && (int)ctx->prof_ev.size() < 2 * chunk) {
        while ((int)ctx->prof_ev.size() < 2 * chunk) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e), "event");
            ctx->prof_ev.push_back(e);
        }
    }
    ApState *hst = static_cast<ApState *>(ctx->pinned);
    int32_t t = 1;   // next pass computes A_t and R_{t+1}
    for (;;) {
        int32_t stop_at = t + chunk;
        if (stop_at > params->max_iter + 1) stop_at = params->max_iter + 1;
        const int32_t t_first = t;
        bool done = false;
        if (use_graph && stop_at - t == chunk) {
            const int mode = imp_a      ? SOLVE_IMPLICIT_A
                             : implicit ? SOLVE_IMPLICIT_R
                             : msg_rule ? SOLVE_EXPLICIT_DELTA
                                        : SOLVE_EXPLICIT;
            const apx_status gs = graph_chunk(ctx, imp_a ? apl : implicit ? ipl : pl, mode, S, buf, A, n, ld, lam, w,
                                              chunk, t, hst);
            if (gs == APX_OK) {
                t = stop_at;
                done = true;
            } else if (gs == APX_ENOTIMPL) {
                use_graph = false;
            } else {
                return gs;
            }
        }
        if (!done) {
            for (; t < stop_at; ++t) {
                PassArgs pf = pass_args(S, buf[t & 1], buf[(t + 1) & 1], A, n, ld, lam, w, w.dec,
                                        w.eflag, w.st);
                const int slot = t - t_first;
                if (ctx->prof) HIP_TRY(hipEventRecord(ctx->prof_ev[2 * slot], s), "event");
                if (imp_a) {
                    ImpArgs ia = imp_args(S, A, n, ld, lam, w, buf, false, ctx->implicit_k, ctx->implicit_a);
                    ia.blk = ia_blk;
                    ia.lean = ctx->lean ? 1 : 0;
                    HIP_TRY(launch_row_ia(apl, ia, s), "row pass");
                }
                else if (implicit)
                    HIP_TRY(launch_row_imp(ipl, IMP_FULL,
                                           imp_args(S, A, n, ld, lam, w, buf, false, ctx->implicit_k), s),
                            "row pass");
                else
                    HIP_TRY(launch_row_pass(pl, msg_rule ? PASS_FULL_DELTA : PASS_FULL, pf, s), "row pass");
                if (ctx->prof) HIP_TRY(hipEventRecord(ctx->prof_ev[2 * slot + 1], s), "event");
                HIP_TRY(launch_col_reduce(col_args(w, n, w.st, 1, imp_a ? t : -1, lam), s), "column reduce");
            }
            HIP_TRY(hipMemcpyAsync(hst, w.st, sizeof(ApState), hipMemcpyDeviceToHost, s), "state");
            HIP_TRY(hipStreamSynchronize(s), "sync");
        }
        if (ctx->prof) {
            // only the passes that did work (iterations <= the stop iteration)
            for (int32_t u = t_first; u < t && u <= hst->iter; ++u) {
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, ctx->prof_ev[2 * (u - t_first)],
                                            ctx->prof_ev[2 * (u - t_first) + 1]), "elapsed");
                ctx->prof_ms += ms;
                ctx->prof_launches += 1;
            }
        }
        if (hst->frozen == 2) {
            // A row list overflowed in pass t_a (overflowed rows were written
            // explicitly by the pass itself).  A_{t_a} is made explicit when A
            // was implicit, R_{t_a+1} when its list overflowed; the column
            // vectors are rebuilt and the run continues with explicit messages.
            const int32_t ta = hst->iter;
            const int po = (ta + 1) & 1;
            fallback |= hst->imp_abort;
            // implicit R cannot continue without implicit A when a row list
            // breaks the implicit-R pass's owner rule
            const bool r_too = (hst->imp_abort & 5) || (imp_a && implicit && hst->imp_owner);
            if (imp_a && implicit && hst->imp_owner && !(hst->imp_abort & 5)) fallback |= APX_FALLBACK_R_OWNER;
            if (imp_a) {
                HIP_TRY(launch_ia_materialize(A, ld, (int32_t)n, w.acol[ta & 1], w.adiag[ta & 1],
                                              w.xst + (ta & 1) * w.xstride, s, ia_blk, lam, ta), "materialize A");
                imp_a = false;
                ia_until = ta;
            }
            if (r_too) {
                // alpha_{t_a+1} is the run state's current alpha after the reduce of pass t_a
                HIP_TRY(launch_imp_materialize(S, buf[po], ld, (int32_t)n, &w.st->imp_al,
                                               w.imp + po * w.imp_stride, s), "materialize R");
                implicit = false;
                imp_until = ta;
            }
            HIP_TRY(launch_col_reduce(col_args(w, n, nullptr, 0), s), "column reduce");
            HIP_TRY(launch_state_resume(w.st, s), "resume");
            t = ta + 1;
            continue;
        }
        if (hst->frozen || t > params->max_iter) break;
    }
    const int32_t T = hst->iter;
    res->iterations = T;
    res->converged = hst->converged;
    ctx->last_imp_iters = imp_until < T ? imp_until : T;
    ctx->last_exp_iters = T - ctx->last_imp_iters;
    ctx->last_ia_iters = ia_until < T ? ia_until : T;
    ctx->last_fallback = fallback | (hst->imp_owner ? APX_NOTE_R_OWNER : 0);
    ctx->last_lean_rescans = hst->lean_rescans;
    if (imp_a) {
        HIP_TRY(launch_ia_materialize(A, ld, (int32_t)n, w.acol[T & 1], w.adiag[T & 1],
                                      w.xst + (T & 1) * w.xstride, s, ia_blk, lam, T), "materialize A");
    }
    if (implicit) {
        // alpha_T is the previous alpha after the reduce of pass T
        HIP_TRY(launch_imp_materialize(S, R, ld, (int32_t)n, &w.st->imp_al_prev,
                                       w.imp + (T & 1) * w.imp_stride, s), "materialize R");
    } else if (T & 1) {
        HIP_TRY(launch_copy_rows(R, w.R2, n, n, ld, s), "copy R");
    }

    FinalArgs fa{};
    fa.S = S;
    fa.ld = ld;
    fa.n = (int32_t)n;
    fa.eflag = w.eflag;
    fa.ex = w.ex;
    fa.nex = w.nex;
    fa.idx = idx;
    fa.contrib = w.contrib;
    fa.sums = w.sums;
    if (raw_labels) {
        // d_T = argmax_k a_T(i,k) + r_T(i,k) from the messages just returned
        HIP_TRY(launch_decide(A, R, n, ld, w.dec, s), "decisions");
        fa.raw = w.dec;
    }
    HIP_TRY(launch_finalize(fa, s), "finalize");
    double *hd = reinterpret_cast<double *>(static_cast<char *>(ctx->pinned) + 256);
    int32_t *hn = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 512);
    HIP_TRY(hipMemcpyAsync(hd, w.sums, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "sums");
    HIP_TRY(hipMemcpyAsync(hn, w.nex, sizeof(int32_t), hipMemcpyDeviceToHost, s), "nex");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    res->n_exemplars = *hn;
    if (*hn == 0) {
        res->dpsim = res->expref = res->netsim = NAN;
    } else {
        res->dpsim = hd[0];
        res->expref = hd[1];
        res->netsim = hd[0] + hd[1];
    }
    res->status = APX_OK;
    return APX_OK;
}

}  // extern "C"

// ---- matrix-free AP ----------------------------------------------------------
// Workspace of ap_solve_mf: the similarity scratch, the run state and message
// state (no n x n buffer), the partials of every panel launch of a pass, and
// two panels (S rows; and rows the implicit passes write only when a list
// overflows, which ends the run).
namespace {
struct MfLayout {
    size_t o_sim, o_t, o_c, o_d, o_p, o_dec, o_e, o_st, o_ex, o_nex, o_con, o_sum, o_imp, o_acol, o_x, o_pan, o_dum,
        bytes;
};
MfLayout mf_layout(int64_t n, int64_t ld, int64_t prows, int64_t nparts) {
    MfLayout o{};
    WsLayout L;
    const int64_t ldp = round4(n);
    o.o_sim = L.take(mf_sim_bytes(n));
    o.o_t = L.take(sizeof(float) * ldp);
    o.o_c = L.take(sizeof(float) * ldp);
    o.o_d = L.take(sizeof(float) * ldp);
    o.o_p = L.take(sizeof(float) * ldp * (size_t)nparts);
    o.o_dec = L.take(sizeof(int32_t) * n);
    o.o_e = L.take((size_t)n);
    o.o_st = L.take(sizeof(ApState));
    o.o_ex = L.take(sizeof(int32_t) * n);
    o.o_nex = L.take(sizeof(int32_t));
    o.o_con = L.take(sizeof(double) * 2 * (size_t)n);
    o.o_sum = L.take(sizeof(double) * 2);
    o.o_imp = L.take(2 * (size_t)imp_layout(n).stride);
    o.o_acol = L.take(4 * sizeof(float) * (size_t)ldp);
    o.o_x = L.take(2 * (size_t)x_layout(n).stride);
    o.o_pan = L.take(sizeof(float) * (size_t)prows * (size_t)ld);
    o.o_dum = L.take(sizeof(float) * (size_t)prows * (size_t)ld);
    o.bytes = L.off;
    return o;
}
int64_t mf_default_rows(int64_t n, int64_t ld, int grid) {
    // panels of at most 1 GiB, at least 8 rows per workgroup of a pass
    int64_t p = ((int64_t)1 << 30) / (4 * ld);
    if (p < 8 * (int64_t)grid) p = 8 * (int64_t)grid;
    return p < n ? p : n;
}
// Plans and panels of a matrix-free solve; false when n is outside the
// implicit passes or the panel holds less than one row per workgroup.
bool mf_shape(int64_t n, int64_t panel_rows, int num_cus, MfShape *sh) {
    if (n < 2 || n > 65536 || !imp_plan(n, num_cus, &sh->ipl) || !ia_plan(n, num_cus, &sh->apl)) return false;
    sh->ld = (n + 63) & ~int64_t(63);
    sh->gmax = sh->ipl.grid > sh->apl.grid ? sh->ipl.grid : sh->apl.grid;
    int64_t P = panel_rows > 0 ? panel_rows : mf_default_rows(n, sh->ld, sh->gmax);
    if (P > n) P = n;
    if (P < sh->gmax) return false;
    sh->P = P;
    sh->Q = (n + P - 1) / P;
    return true;
}
size_t mf_bytes(int64_t n, const MfShape &sh) { return mf_layout(n, sh.ld, sh.P, sh.Q * sh.gmax).bytes; }
}  // namespace

extern "C" apx_status ap_solve_mf(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                                  int32_t pref_mode, const float *pref_vec, float pref_scalar, uint64_t noise_seed,
                                  double noise_rel, int64_t panel_rows, const apx_params *params, int32_t *idx,
                                  apx_result *res, double *pref_out) {
    if (!ctx) return APX_EINVAL;
    if (!X || !idx || !params || !res) return set_err(ctx, APX_EINVAL, "X, params, idx and res must be non-null");
    if (d < 1 || ldx < d) return set_err(ctx, APX_EINVAL, "need d >= 1 and ldx >= d");
    if (pref_mode < APX_PREF_MEDIAN || pref_mode > APX_PREF_VECTOR) return set_err(ctx, APX_EINVAL, "bad pref_mode");
    if (pref_mode == APX_PREF_VECTOR && !pref_vec) return set_err(ctx, APX_EINVAL, "pref_vec is null");
    if (pref_mode == APX_PREF_SCALAR && !std::isfinite(pref_scalar))
        return set_err(ctx, APX_EINVAL, "pref_scalar is not finite");
    if (!(noise_rel >= 0.0) || !std::isfinite(noise_rel)) return set_err(ctx, APX_EINVAL, "bad noise_rel");
    APX_TRY(check_params(ctx, params));
    if (params->flags & (APX_RAW_LABELS | APX_MSG_THRESHOLD))
        return set_err(ctx, APX_ENOTIMPL, "raw labels and the message-change rule need R and A in memory");
    if (panel_rows < 0) return set_err(ctx, APX_EINVAL, "panel_rows < 0");
    MfShape sh;
    if (!mf_shape(n, 0, ctx->num_cus, &sh) || ctx->implicit_k <= 0 || ctx->implicit_a <= 0)
        return set_err(ctx, APX_ENOTIMPL, "n = %lld outside the implicit passes (or they are disabled)", (long long)n);
    if (!mf_shape(n, panel_rows, ctx->num_cus, &sh))
        return set_err(ctx, APX_EINVAL, "panel_rows must be >= %d (one row per workgroup)", sh.gmax);
    const PassPlan ipl = sh.ipl, apl = sh.apl;
    const int64_t ld = sh.ld, P = sh.P, Q = sh.Q;
    const int gmax = sh.gmax;
    const float lam = params->damping;
    DevGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    std::memset(res, 0, sizeof *res);

    const MfLayout o = mf_layout(n, ld, P, Q * gmax);
    APX_TRY(ws_reserve(ctx, ctx->ws_base + o.bytes));
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;
    // non-finite points or preferences are rejected before anything runs
    int32_t *hflag = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 2048);
    HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(ctx->dflag), sizeof(int32_t), 0, s), "finite check");
    HIP_TRY(launch_check_finite(X, n, d, ldx, ctx->dflag, s), "finite check");
    if (pref_mode == APX_PREF_VECTOR) HIP_TRY(launch_check_finite(pref_vec, 1, n, n, ctx->dflag, s), "finite check");
    HIP_TRY(hipMemcpyAsync(hflag, ctx->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "finite check");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (*hflag) return set_err(ctx, APX_EINVAL, "X or pref_vec holds a NaN or infinite value");

    MfSim m{X, n, d, ldx, pref_mode, pref_vec, pref_scalar, noise_seed, noise_rel, b + o.o_sim};
    float *panel = reinterpret_cast<float *>(b + o.o_pan);
    float *dummy = reinterpret_cast<float *>(b + o.o_dum);
    HIP_TRY(mf_sim_setup(m, panel, ld, P, s), "similarity setup");
    {
        double *h = reinterpret_cast<double *>(static_cast<char *>(ctx->pinned) + 1024);
        uint32_t *hk = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->pinned) + 1088);
        HIP_TRY(hipMemcpyAsync(h, mf_sim_pref(m), sizeof(double), hipMemcpyDeviceToHost, s), "pref copy");
        HIP_TRY(hipMemcpyAsync(hk, mf_sim_bounds(m), 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "bounds copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (hk[1] >= 0xff800000u || hk[0] <= 0x007fffffu)
            return set_err(ctx, APX_EINVAL, "similarities overflow FP32");
        if (pref_out) *pref_out = pref_mode == APX_PREF_VECTOR ? NAN : *h;
    }

    IterWs w{};
    w.tcol = reinterpret_cast<float *>(b + o.o_t);
    w.ccol = reinterpret_cast<float *>(b + o.o_c);
    w.rdiag = reinterpret_cast<float *>(b + o.o_d);
    w.partial = reinterpret_cast<float *>(b + o.o_p);
    w.ldp = round4(n);
    w.dec = reinterpret_cast<int32_t *>(b + o.o_dec);
    w.eflag = reinterpret_cast<uint8_t *>(b + o.o_e);
    w.st = reinterpret_cast<ApState *>(b + o.o_st);
    w.ex = reinterpret_cast<int32_t *>(b + o.o_ex);
    w.nex = reinterpret_cast<int32_t *>(b + o.o_nex);
    w.contrib = reinterpret_cast<double *>(b + o.o_con);
    w.sums = reinterpret_cast<double *>(b + o.o_sum);
    w.imp = b + o.o_imp;
    w.imp_stride = imp_layout(n).stride;
    for (int q = 0; q < 2; ++q) {
        w.acol[q] = reinterpret_cast<float *>(b + o.o_acol) + q * w.ldp;
        w.adiag[q] = reinterpret_cast<float *>(b + o.o_acol) + (2 + q) * w.ldp;
    }
    w.xst = b + o.o_x;
    w.xstride = x_layout(n).stride;

    HIP_TRY(launch_state_init(w.st, params->max_iter, params->conv_iter, lam, s, 0, 0.0f, 0), "state init");
    HIP_TRY(launch_fill_u8(w.eflag, n, 0, s), "flags");
    const ImpLayout il = imp_layout(n);
    HIP_TRY(launch_fill_f32_rows(reinterpret_cast<float *>(w.imp + il.beta), 1, n, n, 0.0f, s), "implicit state");
    HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(w.imp + il.cnt), 4 * n, 0, s), "implicit state");
    HIP_TRY(launch_fill_f32_rows(w.acol[0], 1, w.ldp, w.ldp, 0.0f, s), "implicit A");
    HIP_TRY(launch_fill_f32_rows(w.adiag[0], 1, w.ldp, w.ldp, 0.0f, s), "implicit A");
    HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(w.xst + x_layout(n).cnt), 4 * n, 0, s), "implicit A");

    // Rows [p0, p1) of S live in the panel: every kernel of the pass reads
    // row i at S + i * ld, so it gets the panel shifted back by p0 rows (only
    // its own rows are dereferenced).  Each panel launch writes its own rows
    // of partials; the column reduce sums all of them.
    auto shifted = [&](float *base, int64_t p0) { return base - p0 * ld; };
    // R_1 from R_0 = A_0 = 0 (Eq. (2), damped), panel by panel
    for (int64_t q = 0; q < Q; ++q) {
        const int64_t p0 = q * P, p1 = p0 + P < n ? p0 + P : n;
        HIP_TRY(mf_sim_panel(m, panel, ld, p0, p1, nullptr, s), "similarity panel");
        float *buf[2] = {shifted(dummy, p0), shifted(dummy, p0)};
        ImpArgs ia = imp_args(shifted(panel, p0), shifted(dummy, p0), n, ld, lam, w, buf, true, ctx->implicit_k);
        ia.row_begin = p0;
        ia.row_end = p1;
        ia.part0 = q * ipl.grid;
        HIP_TRY(launch_row_imp(ipl, IMP_PRO_COLD, ia, s), "prologue");
    }
    w.nparts = (int)(Q * ipl.grid);
    HIP_TRY(launch_col_reduce(col_args(w, n, nullptr, 0, 0, lam), s), "column reduce");

    int chunk = params->check_every > 0 ? params->check_every : 16;
    ApState *hst = static_cast<ApState *>(ctx->pinned);
    w.nparts = (int)(Q * apl.grid);
    int32_t t = 1;
    bool stop = false;
    while (!stop) {
        const int32_t t_end = t + chunk <= params->max_iter + 1 ? t + chunk : params->max_iter + 1;
        for (; t < t_end; ++t) {
            for (int64_t q = 0; q < Q; ++q) {
                const int64_t p0 = q * P, p1 = p0 + P < n ? p0 + P : n;
                HIP_TRY(mf_sim_panel(m, panel, ld, p0, p1, w.st, s), "similarity panel");
                float *buf[2] = {shifted(dummy, p0), shifted(dummy, p0)};
                ImpArgs ia = imp_args(shifted(panel, p0), shifted(dummy, p0), n, ld, lam, w, buf, false,
                                      ctx->implicit_k, ctx->implicit_a);
                ia.lean = ctx->lean ? 1 : 0;
                ia.row_begin = p0;
                ia.row_end = p1;
                ia.part0 = q * apl.grid;
                HIP_TRY(launch_row_ia(apl, ia, s), "row pass");
            }
            HIP_TRY(launch_col_reduce(col_args(w, n, w.st, 1, t, lam), s), "column reduce");
        }
        HIP_TRY(hipMemcpyAsync(hst, w.st, sizeof(ApState), hipMemcpyDeviceToHost, s), "state copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        if (hst->frozen == 2)
            return set_err(ctx, APX_ENOTIMPL,
                           "a row list overflowed at iteration %d: the matrix-free form needs the implicit "
                           "messages throughout",
                           hst->iter);
        stop = hst->frozen || t > params->max_iter;
    }
    const int32_t T = hst->iter;
    res->iterations = T;
    res->converged = hst->converged;
    ctx->last_imp_iters = T;
    ctx->last_exp_iters = 0;
    ctx->last_ia_iters = T;
    ctx->last_fallback = hst->imp_owner ? APX_NOTE_R_OWNER : 0;
    ctx->last_lean_rescans = hst->lean_rescans;

    // labels: exemplars from the last pass's flags, every row's best
    // exemplar from its panel
    FinalArgs fa{};
    fa.ld = ld;
    fa.n = (int32_t)n;
    fa.eflag = w.eflag;
    fa.ex = w.ex;
    fa.nex = w.nex;
    fa.idx = idx;
    fa.contrib = w.contrib;
    fa.sums = w.sums;
    HIP_TRY(launch_compact(fa, s), "finalize");
    for (int64_t q = 0; q < Q; ++q) {
        const int64_t p0 = q * P, p1 = p0 + P < n ? p0 + P : n;
        HIP_TRY(mf_sim_panel(m, panel, ld, p0, p1, nullptr, s), "similarity panel");
        fa.S = shifted(panel, p0);
        fa.row0 = p0;
        fa.row1 = p1;
        HIP_TRY(launch_labels(fa, s), "labels");
    }
    HIP_TRY(launch_sum2(fa, s), "finalize");
    double *hd = reinterpret_cast<double *>(static_cast<char *>(ctx->pinned) + 256);
    int32_t *hn = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 512);
    HIP_TRY(hipMemcpyAsync(hd, w.sums, 2 * sizeof(double), hipMemcpyDeviceToHost, s), "sums");
    HIP_TRY(hipMemcpyAsync(hn, w.nex, sizeof(int32_t), hipMemcpyDeviceToHost, s), "nex");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    res->n_exemplars = *hn;
    if (*hn == 0) {
        res->dpsim = res->expref = res->netsim = NAN;
    } else {
        res->dpsim = hd[0];
        res->expref = hd[1];
        res->netsim = hd[0] + hd[1];
    }
    res->status = APX_OK;
    return APX_OK;
}

