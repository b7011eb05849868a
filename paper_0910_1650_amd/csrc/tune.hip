// tune.hip -- autotuner of the dense AP iteration (Algorithm 1, Section 2).
//
// Problem sizes are grouped into buckets that share one row-pass shape (the
// number of float4 chunks each thread owns in a row).  For a bucket the
// tuner times every instantiated workgroup size (256, 512, 1024 threads) and
// variant (row values and column partials in LDS, or in registers) on a
// scratch problem with the same row length, and keeps the fastest.  Every
// candidate uses the same row -> workgroup map, so all of them form the
// same sums in the same order: tuning never changes a bit of any result.
// The tuner also sets the host poll interval of the stop flag so that a
// poll costs about 1% of the iterations between polls.  Choices persist as
// a small JSON file (apx_tune_save / apx_tune_load; APX_TUNE_FILE is loaded
// at context creation, APX_AUTOTUNE=1 tunes unseen buckets on first use).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "apx_internal.h"

namespace apx {

int64_t tune_bucket(int64_t n) {
    return n <= 4096 ? (n + 1023) / 1024 : 4 + (n - 4096 + 4095) / 4096;
}

}  // namespace apx

using namespace apx;

namespace {

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)
#define APX_TRY(expr)                        \
    do {                                     \
        const apx_status _s = (expr);        \
        if (_s != APX_OK) return _s;         \
    } while (0)

constexpr int kThreads[3] = {256, 512, 1024};

// Deterministic finite scratch values: v(i,k) = scale * (offset - h(i,k)/1024)
// with h a small integer hash, so rows have no long runs of ties.
__global__ void k_tune_fill(float *p, int64_t rows, int64_t n, int64_t ld, float scale, float offset) {
    for (int64_t i = blockIdx.x; i < rows; i += gridDim.x)
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
            const uint32_t h = (uint32_t)(i * 2654435761u) ^ (uint32_t)(k * 40503u);
            p[i * ld + k] = scale * (offset - (float)((h >> 7) & 1023u) / 1024.0f);
        }
}

struct Scratch {
    float *S = nullptr, *R = nullptr, *A = nullptr, *vec = nullptr, *partial = nullptr;
    ~Scratch() {
        for (float *p : {S, R, A, vec, partial})
            if (p) (void)hipFree(p);
    }
};

apx_status measure(apx_ctx *ctx, int64_t n, TuneEntry *out) {
    hipStream_t s = ctx->stream;
    const PassPlan base = plan_pass(n, ctx->num_cus);
    const int64_t ld = (n + 63) & ~int64_t(63);
    const int64_t ldp = (n + 3) & ~int64_t(3);
    const int64_t rows = n < 4LL * base.grid ? n : 4LL * base.grid;
    Scratch sc;
    HIP_TRY(hipMalloc(&sc.S, sizeof(float) * rows * ld), "tune scratch");
    HIP_TRY(hipMalloc(&sc.R, sizeof(float) * rows * ld), "tune scratch");
    HIP_TRY(hipMalloc(&sc.A, sizeof(float) * rows * ld), "tune scratch");
    HIP_TRY(hipMalloc(&sc.vec, sizeof(float) * 3 * ldp), "tune scratch");
    HIP_TRY(hipMalloc(&sc.partial, sizeof(float) * ldp * base.grid), "tune scratch");
    const unsigned fg = (unsigned)(rows < 4096 ? rows : 4096);
    k_tune_fill<<<fg, 256, 0, s>>>(sc.S, rows, n, ld, 1.0f, 0.0f);
    k_tune_fill<<<fg, 256, 0, s>>>(sc.R, rows, n, ld, 0.5f, 0.5f);
    k_tune_fill<<<fg, 256, 0, s>>>(sc.A, rows, n, ld, 0.25f, 0.0f);
    HIP_TRY(hipGetLastError(), "tune fill");
    HIP_TRY(hipMemsetAsync(sc.vec, 0, sizeof(float) * 3 * ldp, s), "tune vectors");

    PassArgs a{};
    a.S = sc.S;
    a.Rin = sc.R;
    a.Rout = sc.R;
    a.A = sc.A;
    a.ld = ld;
    a.n = (int32_t)n;
    a.lam = 0.9f;
    a.tcol = sc.vec;
    a.ccol = sc.vec + ldp;
    a.rdiag = sc.vec + 2 * ldp;
    a.partial = sc.partial;
    a.ldp = ldp;
    a.row_begin = 0;
    a.row_end = rows;
    ColArgs c{};
    c.partial = sc.partial;
    c.ldp = ldp;
    c.nparts = base.grid;
    c.rdiag = a.rdiag;
    c.tcol = sc.vec;
    c.ccol = sc.vec + ldp;
    c.n = (int32_t)n;

    hipEvent_t ev[3];
    for (hipEvent_t &e : ev) HIP_TRY(hipEventCreate(&e), "tune event");
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int q = 0; q < 3; ++q) (void)hipEventDestroy(e[q]);
        }
    } eg{ev};

    double best = 1e300, col_ms = 0.0;
    TuneEntry pick{};
    for (int ti = 0; ti < 3; ++ti)
        for (int lds = 1; lds >= 0; --lds) {
            const PassPlan pl = plan_pass_variant(n, ctx->num_cus, kThreads[ti], lds != 0);
            if (pl.threads == 0 || (lds && pl.lds_bytes == 0)) continue;
            constexpr int reps = 5;
            for (int w = 0; w < 2; ++w) {
                HIP_TRY(launch_row_pass(pl, PASS_FULL, a, s), "tune pass");
                HIP_TRY(launch_col_reduce(c, s), "tune reduce");
            }
            HIP_TRY(hipEventRecord(ev[0], s), "tune event");
            for (int r = 0; r < reps; ++r) HIP_TRY(launch_row_pass(pl, PASS_FULL, a, s), "tune pass");
            HIP_TRY(hipEventRecord(ev[1], s), "tune event");
            for (int r = 0; r < reps; ++r) HIP_TRY(launch_col_reduce(c, s), "tune reduce");
            HIP_TRY(hipEventRecord(ev[2], s), "tune event");
            HIP_TRY(hipEventSynchronize(ev[2]), "tune sync");
            float p_ms = 0.0f, c_ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&p_ms, ev[0], ev[1]), "tune elapsed");
            HIP_TRY(hipEventElapsedTime(&c_ms, ev[1], ev[2]), "tune elapsed");
            const double per_iter = (double)p_ms / reps * ((double)n / (double)rows) + (double)c_ms / reps;
            if (per_iter < best) {
                best = per_iter;
                col_ms = (double)c_ms / reps;
                pick.threads = pl.threads;
                pick.lds = pl.lds_bytes > 0 ? 1 : 0;
            }
        }
    if (best >= 1e300) return set_err(ctx, APX_ENOTIMPL, "no row-pass variant for n = %lld", (long long)n);
    (void)col_ms;

    // Host poll: a 64-byte state copy and a stream synchronisation.
    HIP_TRY(hipStreamSynchronize(s), "tune sync");
    const auto t0 = std::chrono::steady_clock::now();
    constexpr int polls = 20;
    for (int r = 0; r < polls; ++r) {
        HIP_TRY(hipMemcpyAsync(ctx->pinned, sc.vec, 64, hipMemcpyDeviceToHost, s), "tune poll");
        HIP_TRY(hipStreamSynchronize(s), "tune poll");
    }
    const double poll_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / polls;
    int chunk = (int)std::ceil(100.0 * poll_ms / best);
    chunk = chunk < 2 ? 2 : (chunk > 64 ? 64 : chunk);
    chunk += chunk & 1;

    pick.bucket = tune_bucket(n);
    pick.n = n;
    pick.check_every = chunk;
    pick.ms_per_iter = best;
    *out = pick;
    return APX_OK;
}

TuneEntry *find_entry(apx_ctx *ctx, int64_t n) {
    const int64_t b = tune_bucket(n);
    for (TuneEntry &e : ctx->tune)
        if (e.bucket == b) return &e;
    return nullptr;
}

// Replaces the bucket's entry; unless keep_form is false, a new entry
// without a form keeps the old entry's form and form timings (the two are
// tuned separately).
void put_entry(apx_ctx *ctx, const TuneEntry &e, bool keep_form = true) {
    for (TuneEntry &x : ctx->tune)
        if (x.bucket == e.bucket) {
            const TuneEntry old = x;
            x = e;
            if (keep_form && e.form == 0) {
                x.form = old.form;
                for (int q = 0; q < 3; ++q) x.form_ms[q] = old.form_ms[q];
            }
            return;
        }
    ctx->tune.push_back(e);
}

// Points of a 16-D mixture of 20 unit Gaussians whose centres are spread
// with standard deviation 4 (Box-Muller on a counter hash): the scratch
// problem of the form timing.
__device__ __forceinline__ float tune_u01(uint32_t a, uint32_t b) {
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return ((float)(h >> 8) + 0.5f) * (1.0f / 16777216.0f);
}
__global__ void k_tune_points(float *X, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = (uint32_t)(tune_u01((uint32_t)i, 1u) * 20.0f);
    for (int j = 0; j < 16; ++j) {
        const float u1 = tune_u01(c, 100u + j), u2 = tune_u01(c, 200u + j);
        const float v1 = tune_u01((uint32_t)i, 300u + j), v2 = tune_u01((uint32_t)i, 400u + j);
        const float cz = sqrtf(-2.0f * logf(u1)) * cosf(6.2831853f * u2);
        const float z = sqrtf(-2.0f * logf(v1)) * cosf(6.2831853f * v2);
        X[i * 16 + j] = 4.0f * cz + z;
    }
}

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

}  // namespace

namespace apx {

apx_status ctx_plan(apx_ctx *ctx, int64_t n, PassPlan *pl, int *check_every, bool may_tune, int *form) {
    *pl = plan_pass(n, ctx->num_cus);
    if (check_every) *check_every = 0;
    if (form) *form = 0;
    TuneEntry *e = find_entry(ctx, n);
    // the tuner allocates a scratch problem: never with a caller-set workspace
    if (!e && may_tune && ctx->autotune && !ctx->ws_external) {
        TuneEntry t{};
        const apx_status st = measure(ctx, n, &t);
        if (st != APX_OK) return st;
        put_entry(ctx, t);
        e = find_entry(ctx, n);
    }
    if (e) {
        const PassPlan t = plan_pass_variant(n, ctx->num_cus, e->threads, e->lds != 0);
        if (t.threads != 0) *pl = t;
        if (check_every) *check_every = e->check_every;
        if (form) *form = e->form;
    }
    if (form && ctx->force_form) *form = ctx->force_form;
    return APX_OK;
}

}  // namespace apx

extern "C" {

apx_status apx_autotune(apx_ctx *ctx, int64_t n) {
    if (!ctx) return APX_EINVAL;
    if (n < 2 || n > 65536) return set_err(ctx, APX_EINVAL, "autotune needs 2 <= n <= 65536");
    DevGuard g(ctx->device);
    TuneEntry t{};
    const apx_status st = measure(ctx, n, &t);
    if (st != APX_OK) return st;
    put_entry(ctx, t);
    return APX_OK;
}

apx_status apx_set_autotune(apx_ctx *ctx, int enable) {
    if (!ctx) return APX_EINVAL;
    ctx->autotune = enable != 0;
    return APX_OK;
}

apx_status apx_tune_set(apx_ctx *ctx, int64_t n, int32_t threads, int32_t lds, int32_t check_every) {
    if (!ctx) return APX_EINVAL;
    if (n < 2 || n > 65536) return set_err(ctx, APX_EINVAL, "need 2 <= n <= 65536");
    const PassPlan pl = plan_pass_variant(n, ctx->num_cus, threads, lds != 0);
    if (pl.threads == 0) return set_err(ctx, APX_EINVAL, "no row pass with %d threads for n = %lld", threads, (long long)n);
    if (check_every < 0) return set_err(ctx, APX_EINVAL, "check_every < 0");
    TuneEntry t{};
    t.bucket = tune_bucket(n);
    t.n = n;
    t.threads = threads;
    t.lds = lds != 0 ? 1 : 0;
    t.check_every = check_every;
    t.ms_per_iter = 0.0;
    put_entry(ctx, t);
    return APX_OK;
}

apx_status apx_tune_get(apx_ctx *ctx, int64_t n, int32_t *threads, int32_t *lds, int32_t *check_every,
                        double *ms_per_iter) {
    if (!ctx || !threads || !lds || !check_every || !ms_per_iter) return APX_EINVAL;
    const TuneEntry *e = find_entry(ctx, n);
    if (!e) {
        *threads = *lds = *check_every = 0;
        *ms_per_iter = 0.0;
        return APX_OK;
    }
    // the variant that actually runs at this n (LDS may not fit every n of a bucket)
    const PassPlan pl = plan_pass_variant(n, ctx->num_cus, e->threads, e->lds != 0);
    *threads = e->threads;
    *lds = pl.lds_bytes > 0 ? 1 : 0;
    *check_every = e->check_every;
    *ms_per_iter = e->ms_per_iter;
    return APX_OK;
}

apx_status apx_autotune_form(apx_ctx *ctx, int64_t n, int32_t *form, double *ms) {
    if (!ctx) return APX_EINVAL;
    if (n < 2 || n > 65536) return set_err(ctx, APX_EINVAL, "autotune_form needs 2 <= n <= 65536");
    DevGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    const int64_t ld = (n + 63) & ~int64_t(63);
    Scratch sc;
    HIP_TRY(hipMalloc(&sc.vec, sizeof(float) * 16 * n), "form scratch");
    HIP_TRY(hipMalloc(&sc.S, sizeof(float) * n * ld), "form scratch");
    HIP_TRY(hipMalloc(&sc.R, sizeof(float) * n * ld), "form scratch");
    HIP_TRY(hipMalloc(&sc.A, sizeof(float) * n * ld), "form scratch");
    HIP_TRY(hipMalloc(&sc.partial, sizeof(int32_t) * n), "form scratch");
    k_tune_points<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(sc.vec, n);
    HIP_TRY(hipGetLastError(), "form points");
    apx_status st = ap_similarity(ctx, sc.vec, n, 16, 16, sc.S, ld, APX_PREF_MEDIAN, nullptr, 0.0f, 12345u,
                                  1e-12, nullptr);
    if (st != APX_OK) return st;
    // per-iteration time: the difference of two fixed-length solves (the
    // prologue, the final rebuild of A and R and the finalisation cancel)
    auto run = [&](int f, int32_t iters, double *out_ms) -> apx_status {
        apx_params p{};
        p.damping = 0.9f;
        p.max_iter = iters;
        p.conv_iter = 0;
        p.check_every = iters;
        apx_result r{};
        ctx->force_form = f;
        HIP_TRY(hipStreamSynchronize(s), "form sync");
        const auto t0 = std::chrono::steady_clock::now();
        const apx_status e = ap_solve(ctx, sc.S, n, ld, sc.R, sc.A, APX_COLD, &p,
                                      reinterpret_cast<int32_t *>(sc.partial), &r);
        ctx->force_form = 0;
        if (e != APX_OK) return e;
        HIP_TRY(hipStreamSynchronize(s), "form sync");
        *out_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return APX_OK;
    };
    double fm[3] = {0.0, 0.0, 0.0};
    int pick = 0;
    constexpr int32_t kShort = 8, kLong = 40;
    for (int f = APX_FORM_EXPLICIT; f <= APX_FORM_IMPLICIT_RA; ++f) {
        double t_short = 0.0, t_long = 0.0, best = 1e300;
        // warm-up run, then the best of two pairs
        APX_TRY(run(f, kShort, &t_short));
        for (int rep = 0; rep < 2; ++rep) {
            APX_TRY(run(f, kShort, &t_short));
            APX_TRY(run(f, kLong, &t_long));
            const double per = (t_long - t_short) / (double)(kLong - kShort);
            best = per < best ? per : best;
        }
        fm[f - 1] = best > 0.0 ? best : 1e-9;
        if (pick == 0 || fm[f - 1] < fm[pick - 1]) pick = f;
    }
    TuneEntry *e = find_entry(ctx, n);
    TuneEntry t{};
    if (e) {
        t = *e;
    } else {
        // no row-pass entry yet: the default plan with the default poll interval
        const PassPlan pl = plan_pass(n, ctx->num_cus);
        t.bucket = tune_bucket(n);
        t.n = n;
        t.threads = pl.threads;
        t.lds = pl.lds_bytes > 0 ? 1 : 0;
        t.check_every = 0;
        t.ms_per_iter = 0.0;
    }
    t.form = pick;
    for (int q = 0; q < 3; ++q) t.form_ms[q] = fm[q];
    put_entry(ctx, t);
    if (form) *form = pick;
    if (ms)
        for (int q = 0; q < 3; ++q) ms[q] = fm[q];
    return APX_OK;
}

apx_status apx_tune_set_form(apx_ctx *ctx, int64_t n, int32_t form) {
    if (!ctx) return APX_EINVAL;
    if (n < 2 || n > 65536) return set_err(ctx, APX_EINVAL, "need 2 <= n <= 65536");
    if (form < APX_FORM_DEFAULT || form > APX_FORM_IMPLICIT_RA) return set_err(ctx, APX_EINVAL, "bad form %d", form);
    TuneEntry *e = find_entry(ctx, n);
    if (e) {
        e->form = form;
        return APX_OK;
    }
    const PassPlan pl = plan_pass(n, ctx->num_cus);
    TuneEntry t{};
    t.bucket = tune_bucket(n);
    t.n = n;
    t.threads = pl.threads;
    t.lds = pl.lds_bytes > 0 ? 1 : 0;
    t.form = form;
    put_entry(ctx, t);
    return APX_OK;
}

apx_status apx_tune_get_form(apx_ctx *ctx, int64_t n, int32_t *form, double *ms) {
    if (!ctx || !form) return APX_EINVAL;
    const TuneEntry *e = find_entry(ctx, n);
    *form = e ? e->form : 0;
    if (ms)
        for (int q = 0; q < 3; ++q) ms[q] = e ? e->form_ms[q] : 0.0;
    return APX_OK;
}

apx_status apx_tune_clear(apx_ctx *ctx) {
    if (!ctx) return APX_EINVAL;
    ctx->tune.clear();
    ctx->btune.clear();
    return APX_OK;
}

apx_status apx_tune_save(apx_ctx *ctx, const char *path) {
    if (!ctx || !path) return APX_EINVAL;
    FILE *f = std::fopen(path, "w");
    if (!f) return set_err(ctx, APX_EINVAL, "cannot write %s", path);
    std::fprintf(f, "{\n \"compute_units\": %d,\n \"entries\": [\n", ctx->num_cus);
    for (size_t q = 0; q < ctx->tune.size(); ++q) {
        const TuneEntry &e = ctx->tune[q];
        std::fprintf(f,
                     "  {\"bucket\": %lld, \"n\": %lld, \"threads\": %d, \"lds\": %d, \"check_every\": %d, "
                     "\"ms_per_iter\": %.6f, \"form\": %d, \"form_ms\": [%.6f, %.6f, %.6f]}%s\n",
                     (long long)e.bucket, (long long)e.n, e.threads, e.lds, e.check_every, e.ms_per_iter, e.form,
                     e.form_ms[0], e.form_ms[1], e.form_ms[2], q + 1 < ctx->tune.size() ? "," : "");
    }
    std::fprintf(f, " ]\n}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? APX_OK : set_err(ctx, APX_EINVAL, "cannot write %s", path);
}

apx_status apx_tune_load(apx_ctx *ctx, const char *path) {
    if (!ctx || !path) return APX_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return set_err(ctx, APX_EINVAL, "cannot read %s", path);
    std::vector<TuneEntry> got;
    int cus = -1;
    char line[512];
    bool bad = false;
    while (std::fgets(line, sizeof line, f)) {
        const char *p = std::strstr(line, "\"compute_units\":");
        if (p) cus = std::atoi(p + 16);
        if (!std::strstr(line, "\"bucket\"")) continue;
        long long b = 0, n = 0;
        TuneEntry e{};
        const int got_fields = std::sscanf(
            line,
            " {\"bucket\": %lld, \"n\": %lld, \"threads\": %d, \"lds\": %d, \"check_every\": %d, "
            "\"ms_per_iter\": %lf, \"form\": %d, \"form_ms\": [%lf, %lf, %lf]}",
            &b, &n, &e.threads, &e.lds, &e.check_every, &e.ms_per_iter, &e.form, &e.form_ms[0], &e.form_ms[1],
            &e.form_ms[2]);
        // files written before forms were tuned end after ms_per_iter
        if (got_fields != 10 && got_fields != 6) {
            bad = true;
            break;
        }
        if (got_fields == 6) {
            e.form = 0;
            e.form_ms[0] = e.form_ms[1] = e.form_ms[2] = 0.0;
        }
        if (e.form < 0 || e.form > APX_FORM_IMPLICIT_RA) {
            bad = true;
            break;
        }
        e.bucket = b;
        e.n = n;
        if (n < 2 || n > 65536 || tune_bucket(n) != b || e.check_every < 0 ||
            plan_pass_variant(n, ctx->num_cus, e.threads, e.lds != 0).threads == 0) {
            bad = true;
            break;
        }
        got.push_back(e);
    }
    std::fclose(f);
    if (bad) return set_err(ctx, APX_EINVAL, "%s: malformed tuning entry", path);
    if (cus != ctx->num_cus)
        return set_err(ctx, APX_EINVAL, "%s was tuned for %d compute units, this device has %d", path, cus,
                       ctx->num_cus);
    for (const TuneEntry &e : got) put_entry(ctx, e, false);
    return APX_OK;
}

}  // extern "C"
