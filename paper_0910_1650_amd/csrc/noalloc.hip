// noalloc.hip -- ap_iterate on a fixed device scratch array, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The array below lives in the library's code object: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// Host code never uses the array's name as an address (in host code it is a
// stand-in, not device memory): apx_create looks the address up once per
// context with hipGetSymbolAddress, with the context's device current, and
// the entry point passes that pointer to the kernels.
#include "apx_internal.h"

using namespace apx;

namespace {

// Largest n served, and the scratch size: the column vectors t_k, c_k,
// r(k,k) and the per-workgroup column partials of the row pass (at most
// 2 x 256 workgroups x 4096 columns, or 256 x 8192), each part 256-byte
// aligned.  12 MiB also covers devices with up to 304 compute units.
constexpr int64_t kNoallocMaxN = 8192;
constexpr size_t kScratchBytes = size_t(12) << 20;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

apx_status apx::noalloc_init(apx_ctx *ctx) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        ctx->scratch = nullptr;
        return set_err(ctx, APX_EDEVICE, "scratch array lookup: %s", hipGetErrorString(e));
    }
    ctx->scratch = ptr;
    return APX_OK;
}

extern "C" apx_status ap_iterate_noalloc(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R,
                                         float *A, float damping, int32_t n_iter, int32_t *decision) {
    apx_status st = check_iterate(ctx, S, n, ld, R, A, damping, n_iter);
    if (st != APX_OK) return st;
    if (n > kNoallocMaxN)
        return set_err(ctx, APX_EINVAL, "ap_iterate_noalloc serves n <= %lld (n = %lld); use ap_iterate",
                       (long long)kNoallocMaxN, (long long)n);
    if (ctx->scratch == nullptr) return set_err(ctx, APX_EDEVICE, "the fixed scratch array is not available");
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    // the plan of ap_iterate (a tuned entry if one exists), never tuning here
    PassPlan pl{};
    st = ctx_plan(ctx, n, &pl, nullptr, false);
    if (st == APX_OK) {
        const int64_t ldp = (n + 3) & ~int64_t(3);
        const size_t vec = align256(sizeof(float) * (size_t)ldp);
        const size_t need = 3 * vec + align256(sizeof(float) * (size_t)ldp * (size_t)pl.grid);
        if (need > kScratchBytes) {
            st = set_err(ctx, APX_EINVAL, "n = %lld needs %zu bytes of scratch on this device (%zu fixed)",
                         (long long)n, need, kScratchBytes);
        } else {
            // Every part is written before it is read (the row pass writes all
            // partials and r(k,k), the column reduce t and c), so nothing is
            // cleared between calls.
            char *b = static_cast<char *>(ctx->scratch);
            float *tcol = reinterpret_cast<float *>(b);
            float *ccol = reinterpret_cast<float *>(b + vec);
            float *rdiag = reinterpret_cast<float *>(b + 2 * vec);
            float *partial = reinterpret_cast<float *>(b + 3 * vec);
            const hipError_t e = iterate_passes(pl, S, n, ld, R, A, damping, n_iter, decision, tcol, ccol, rdiag,
                                                partial, ctx->stream);
            if (e != hipSuccess) st = hip_err(ctx, e, "ap_iterate_noalloc passes");
        }
    }
    if (cur >= 0 && cur != ctx->device) (void)hipSetDevice(cur);
    return st;
}
