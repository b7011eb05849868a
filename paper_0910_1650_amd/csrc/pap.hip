// pap.hip -- batched solves and partition affinity propagation.
//
// Algorithm 2 (Section 3): split the points into k parts, run AP on every
// diagonal block S_jj (which keeps the global preferences on its diagonal),
// place the resulting availabilities A_jj block-diagonally in A' with zeros
// elsewhere, and run AP on the whole S from A' (R_0 = 0).  The k sub-problems
// run together as one batch; the gather of S_jj and the scatter of A_jj
// follow the part's permutation.
#include <cstring>
#include <vector>

#include "apx_internal.h"

using namespace apx;

namespace {

// S_jj(a, b) = S[perm[o_j + a]][perm[o_j + b]]: one workgroup per row of a block.
struct GatherArgs {
    const float *S;
    int64_t ld;
    const int64_t *perm;     // device
    const int64_t *off;      // device, k+1
    float *const *sub;       // device array of k block pointers
    const int64_t *subld;    // device, k
    int32_t k;
};

__global__ void k_pap_gather(GatherArgs g, const int32_t *row_part) {
    const int32_t j = row_part[blockIdx.x];
    const int64_t a = (int64_t)blockIdx.x - g.off[j];
    const int64_t o = g.off[j], nj = g.off[j + 1] - o;
    const float *src = g.S + g.perm[o + a] * g.ld;
    float *dst = g.sub[j] + a * g.subld[j];
    for (int64_t b = threadIdx.x; b < nj; b += blockDim.x) dst[b] = src[g.perm[o + b]];
}

// A[perm[o_j + a]][perm[o_j + b]] = A_jj(a, b) (A holds zeros elsewhere).
__global__ void k_pap_scatter(GatherArgs g, const int32_t *row_part, float *A) {
    const int32_t j = row_part[blockIdx.x];
    const int64_t a = (int64_t)blockIdx.x - g.off[j];
    const int64_t o = g.off[j], nj = g.off[j + 1] - o;
    float *dst = A + g.perm[o + a] * g.ld;
    const float *src = g.sub[j] + a * g.subld[j];
    for (int64_t b = threadIdx.x; b < nj; b += blockDim.x) dst[g.perm[o + b]] = src[b];
}

__global__ void k_zero_rows(float *M, int64_t rows, int64_t cols, int64_t ld) {
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
        for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) M[r * ld + c] = 0.0f;
}

int64_t round4(int64_t v) { return (v + 3) & ~int64_t(3); }

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)

apx_status check_params(apx_ctx *ctx, const apx_params *p) {
    if (!p) return set_err(ctx, APX_EINVAL, "params is null");
    if (!(p->damping >= 0.0f && p->damping < 1.0f)) return set_err(ctx, APX_EINVAL, "damping must be in [0,1)");
    if (p->max_iter < 1 || p->conv_iter < 0) return set_err(ctx, APX_EINVAL, "max_iter must be >= 1 and conv_iter >= 0");
    return APX_OK;
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" apx_status ap_solve_batched(apx_ctx *ctx, int32_t count, const apx_instance *inst,
                                       int32_t warm, const apx_params *params, apx_result *res) {
    if (!ctx) return APX_EINVAL;
    if (count < 1 || !inst || !res) return set_err(ctx, APX_EINVAL, "need count >= 1, inst and res");
    apx_status st = check_params(ctx, params);
    if (st != APX_OK) return st;
    if (warm < APX_COLD || warm > APX_WARM_AR) return set_err(ctx, APX_EINVAL, "bad warm mode %d", warm);
    std::vector<BatchSpec> spec(count);
    for (int j = 0; j < count; ++j) {
        const apx_instance &I = inst[j];
        if (I.n < 2) return set_err(ctx, APX_EINVAL, "instance %d: n must be >= 2", j);
        if (I.ld < I.n || I.ld % 4) return set_err(ctx, APX_EINVAL, "instance %d: bad ld", j);
        if (!I.S || !I.R || !I.A || !I.idx) return set_err(ctx, APX_EINVAL, "instance %d: null pointer", j);
        if (!aligned16(I.S) || !aligned16(I.R) || !aligned16(I.A))
            return set_err(ctx, APX_EINVAL, "instance %d: matrices must be 16-byte aligned", j);
        spec[j] = BatchSpec{I.n, I.ld, I.S, I.R, I.A, I.idx};
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    ctx->ws_base = 0;
    return batched_solve(ctx, count, spec.data(), warm, params, res);
}

extern "C" apx_status pap_solve(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *R, float *A,
                                int32_t k, const int64_t *perm, const int64_t *offsets,
                                const apx_params *params, int32_t *idx, apx_result *res,
                                apx_result *sub) {
    if (!ctx) return APX_EINVAL;
    if (!S || !R || !A || !idx || !res) return set_err(ctx, APX_EINVAL, "null argument");
    if (n < 2 || ld < n || ld % 4) return set_err(ctx, APX_EINVAL, "need n >= 2, ld >= n, ld % 4 == 0");
    if (!aligned16(S) || !aligned16(R) || !aligned16(A)) return set_err(ctx, APX_EINVAL, "matrices must be 16-byte aligned");
    if (k < 1 || k > n) return set_err(ctx, APX_EINVAL, "need 1 <= k <= n");
    apx_status st = check_params(ctx, params);
    if (st != APX_OK) return st;

    // Step 1: the partition (the paper's even split unless given).
    std::vector<int64_t> off(k + 1), pm(n);
    if (offsets) {
        for (int j = 0; j <= k; ++j) off[j] = offsets[j];
        if (off[0] != 0 || off[k] != n) return set_err(ctx, APX_EINVAL, "offsets must run from 0 to n");
        for (int j = 0; j < k; ++j)
            if (off[j + 1] - off[j] < 1) return set_err(ctx, APX_EINVAL, "part %d is empty", j);
    } else {
        const int64_t m = n / k;
        for (int j = 0; j < k; ++j) off[j] = j * m;
        off[k] = n;
    }
    if (perm) {
        std::vector<char> seen(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) return set_err(ctx, APX_EINVAL, "perm is not a permutation");
            seen[perm[i]] = 1;
            pm[i] = perm[i];
        }
    } else {
        for (int64_t i = 0; i < n; ++i) pm[i] = i;
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    hipStream_t s = ctx->stream;

    // Workspace: [tables | S_jj | R_jj | A_jj | idx_jj] then the batch solver's slice;
    // the final full solve reuses the workspace from 0.
    WsLayout L;
    const size_t o_perm = L.take(sizeof(int64_t) * n);
    const size_t o_off = L.take(sizeof(int64_t) * (k + 1));
    const size_t o_ptr = L.take(sizeof(float *) * k);
    const size_t o_ld = L.take(sizeof(int64_t) * k);
    const size_t o_rp = L.take(sizeof(int32_t) * n);
    std::vector<size_t> o_s(k), o_r(k), o_a(k), o_i(k);
    std::vector<int64_t> nj(k), ldj(k);
    for (int j = 0; j < k; ++j) {
        nj[j] = off[j + 1] - off[j];
        ldj[j] = round4(nj[j]);
        o_s[j] = L.take(sizeof(float) * nj[j] * ldj[j]);
        o_r[j] = L.take(sizeof(float) * nj[j] * ldj[j]);
        o_a[j] = L.take(sizeof(float) * nj[j] * ldj[j]);
        o_i[j] = L.take(sizeof(int32_t) * nj[j]);
    }
    const size_t head = L.off;
    // sizes of the batch solve and of the full solve
    std::vector<BatchSpec> spec(k);
    for (int j = 0; j < k; ++j) spec[j] = BatchSpec{nj[j], ldj[j], nullptr, nullptr, nullptr, nullptr};
    bool batch_sub = true;
    for (int j = 0; j < k; ++j) batch_sub = batch_sub && nj[j] >= 2;
    const size_t bbytes = batch_sub ? batched_ws_bytes(k, spec.data(), ctx->num_cus) : 0;
    const size_t fbytes = solve_ws_bytes(n, ld, ctx->num_cus);
    ctx->ws_base = 0;
    st = ws_reserve(ctx, head + bbytes > fbytes ? head + bbytes : fbytes);
    if (st != APX_OK) return st;
    char *b = static_cast<char *>(ctx->ws);

    std::vector<float *> subp(k);
    for (int j = 0; j < k; ++j) subp[j] = reinterpret_cast<float *>(b + o_s[j]);
    std::vector<int32_t> rowpart(n);
    for (int j = 0; j < k; ++j)
        for (int64_t a = off[j]; a < off[j + 1]; ++a) rowpart[a] = j;
    HIP_TRY(hipMemcpyAsync(b + o_perm, pm.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s), "perm");
    HIP_TRY(hipMemcpyAsync(b + o_off, off.data(), sizeof(int64_t) * (k + 1), hipMemcpyHostToDevice, s), "offsets");
    HIP_TRY(hipMemcpyAsync(b + o_ptr, subp.data(), sizeof(float *) * k, hipMemcpyHostToDevice, s), "blocks");
    HIP_TRY(hipMemcpyAsync(b + o_ld, ldj.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s), "lds");
    HIP_TRY(hipMemcpyAsync(b + o_rp, rowpart.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s), "rows");
    HIP_TRY(hipStreamSynchronize(s), "sync");

    GatherArgs g{S, ld, reinterpret_cast<int64_t *>(b + o_perm), reinterpret_cast<int64_t *>(b + o_off),
                 reinterpret_cast<float *const *>(b + o_ptr), reinterpret_cast<int64_t *>(b + o_ld), k};
    const int32_t *rp = reinterpret_cast<int32_t *>(b + o_rp);
    k_pap_gather<<<(unsigned)n, 256, 0, s>>>(g, rp);
    HIP_TRY(hipGetLastError(), "gather");

    // Step 2: AP on every block, all blocks in one batch.
    std::vector<apx_result> subres(k);
    if (batch_sub) {
        for (int j = 0; j < k; ++j)
            spec[j] = BatchSpec{nj[j], ldj[j], subp[j], reinterpret_cast<float *>(b + o_r[j]),
                                reinterpret_cast<float *>(b + o_a[j]), reinterpret_cast<int32_t *>(b + o_i[j])};
        ctx->ws_base = head;
        st = batched_solve(ctx, k, spec.data(), APX_COLD, params, subres.data());
        ctx->ws_base = 0;
        if (st != APX_OK) return st;
    } else {
        // a single-point block has no messages: its availability stays 0
        for (int j = 0; j < k; ++j) {
            std::memset(&subres[j], 0, sizeof subres[j]);
            k_zero_rows<<<(unsigned)(nj[j] > 0 ? nj[j] : 1), 256, 0, s>>>(reinterpret_cast<float *>(b + o_a[j]), nj[j], nj[j], ldj[j]);
            HIP_TRY(hipGetLastError(), "zero");
        }
        for (int j = 0; j < k; ++j) {
            if (nj[j] < 2) { subres[j].converged = 1; subres[j].n_exemplars = 1; continue; }
            BatchSpec one{nj[j], ldj[j], subp[j], reinterpret_cast<float *>(b + o_r[j]),
                          reinterpret_cast<float *>(b + o_a[j]), reinterpret_cast<int32_t *>(b + o_i[j])};
            ctx->ws_base = head;
            st = batched_solve(ctx, 1, &one, APX_COLD, params, &subres[j]);
            ctx->ws_base = 0;
            if (st != APX_OK) return st;
        }
    }
    if (sub) std::memcpy(sub, subres.data(), sizeof(apx_result) * k);

    // Step 3: A' = blockdiag(A_jj), zeros elsewhere.
    k_zero_rows<<<(unsigned)(n < 8192 ? n : 8192), 256, 0, s>>>(A, n, n, ld);
    HIP_TRY(hipGetLastError(), "zero A");
    for (int j = 0; j < k; ++j) subp[j] = reinterpret_cast<float *>(b + o_a[j]);
    HIP_TRY(hipMemcpyAsync(b + o_ptr, subp.data(), sizeof(float *) * k, hipMemcpyHostToDevice, s), "blocks");
    k_pap_scatter<<<(unsigned)n, 256, 0, s>>>(g, rp, A);
    HIP_TRY(hipGetLastError(), "scatter");
    HIP_TRY(hipStreamSynchronize(s), "sync");

    // Step 4: AP on the whole S from A' (R_0 = 0).
    return ap_solve(ctx, S, n, ld, R, A, APX_WARM_A, params, idx, res);
}
