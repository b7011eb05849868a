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

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

namespace {

// Workspace of pap_solve for parts of sizes nj: [tables | S_jj R_jj A_jj idx_jj]
// followed by the batch solver's slice, or the full solve's from 0.
struct PapLayout {
    size_t o_perm, o_off, o_ptr, o_ld, o_rp, head, bbytes, fbytes, blk_bytes;
    std::vector<size_t> o_s, o_r, o_a, o_i;
    std::vector<int64_t> ldj;
    bool batch_sub;
    size_t total() const { return head + bbytes > fbytes ? head + bbytes : fbytes; }
};

PapLayout pap_layout(int64_t n, int64_t ld, int32_t k, const std::vector<int64_t> &nj, int num_cus) {
    PapLayout P;
    WsLayout L;
    P.o_perm = L.take(sizeof(int64_t) * n);
    P.o_off = L.take(sizeof(int64_t) * (k + 1));
    P.o_ptr = L.take(sizeof(float *) * k);
    P.o_ld = L.take(sizeof(int64_t) * k);
    P.o_rp = L.take(sizeof(int32_t) * n);
    P.o_s.resize(k);
    P.o_r.resize(k);
    P.o_a.resize(k);
    P.o_i.resize(k);
    P.ldj.resize(k);
    for (int j = 0; j < k; ++j) {
        P.ldj[j] = round4(nj[j]);
        P.o_s[j] = L.take(sizeof(float) * nj[j] * P.ldj[j]);
        P.o_r[j] = L.take(sizeof(float) * nj[j] * P.ldj[j]);
        P.o_a[j] = L.take(sizeof(float) * nj[j] * P.ldj[j]);
        P.o_i[j] = L.take(sizeof(int32_t) * nj[j]);
    }
    P.head = L.off;
    std::vector<BatchSpec> spec(k);
    P.batch_sub = true;
    for (int j = 0; j < k; ++j) {
        spec[j] = BatchSpec{nj[j], P.ldj[j], nullptr, nullptr, nullptr, nullptr};
        P.batch_sub = P.batch_sub && nj[j] >= 2;
    }
    if (P.batch_sub) {
        P.bbytes = batched_ws_bytes(k, spec.data(), num_cus);
    } else {
        // parts solved one at a time: the largest part's slice
        P.bbytes = 0;
        for (int j = 0; j < k; ++j)
            if (nj[j] >= 2) {
                const size_t b = batched_ws_bytes(1, &spec[j], num_cus);
                P.bbytes = b > P.bbytes ? b : P.bbytes;
            }
    }
    // Step 4: the per-row block table, then the full solve's workspace
    P.blk_bytes = (sizeof(int32_t) * 2 * (size_t)n + 255) & ~(size_t)255;
    P.fbytes = P.blk_bytes + solve_ws_bytes(n, ld, num_cus);
    return P;
}

std::vector<int64_t> even_sizes(int64_t n, int32_t k) {
    const int64_t m = n / k;
    std::vector<int64_t> nj(k, m);
    nj[k - 1] = n - m * (k - 1);
    return nj;
}

}  // namespace

namespace apx {
size_t pap_ws_bytes(int64_t n, int64_t ld, int32_t k, const int64_t *sizes, int num_cus) {
    std::vector<int64_t> nj = sizes ? std::vector<int64_t>(sizes, sizes + k) : even_sizes(n, k);
    int64_t tot = 0;
    for (int j = 0; j < k; ++j) {
        if (nj[j] < 1) return 0;
        tot += nj[j];
    }
    if (tot != n) return 0;
    return pap_layout(n, ld, k, nj, num_cus).total();
}
}  // namespace apx

extern "C" apx_status ap_solve_batched(apx_ctx *ctx, int32_t count, const apx_instance *inst,
                                       int32_t warm, const apx_params *params, apx_result *res) {
    if (!ctx) return APX_EINVAL;
    if (count < 1 || !inst || !res) return set_err(ctx, APX_EINVAL, "need count >= 1, inst and res");
    apx_status st = check_params(ctx, params);
    if (st != APX_OK) return st;
    if (warm < APX_COLD || warm > APX_WARM_AR) return set_err(ctx, APX_EINVAL, "bad warm mode %d", warm);
    if (params->flags & (APX_RAW_LABELS | APX_MSG_THRESHOLD))
        return set_err(ctx, APX_ENOTIMPL, "ap_solve_batched supports only the APX_CHECK_FINITE flag");
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
    if (params->flags & APX_CHECK_FINITE)
        for (int j = 0; j < count; ++j) {
            st = check_finite(ctx, spec[j].S, spec[j].n, spec[j].ld, "an instance's S");
            if (st != APX_OK) return st;
        }
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
    const apx_params *const orig_params = params;

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
    if (params->flags & APX_CHECK_FINITE) {
        st = check_finite(ctx, S, n, ld, "S");
        if (st != APX_OK) return st;
    }

    // Workspace: [tables | S_jj | R_jj | A_jj | idx_jj] then the batch solver's slice;
    // the final full solve reuses the workspace from 0.
    std::vector<int64_t> nj(k);
    for (int j = 0; j < k; ++j) nj[j] = off[j + 1] - off[j];
    const PapLayout P = pap_layout(n, ld, k, nj, ctx->num_cus);
    const size_t o_perm = P.o_perm, o_off = P.o_off, o_ptr = P.o_ptr, o_ld = P.o_ld, o_rp = P.o_rp;
    const size_t head = P.head;
    const std::vector<size_t> &o_s = P.o_s, &o_r = P.o_r, &o_a = P.o_a, &o_i = P.o_i;
    const std::vector<int64_t> &ldj = P.ldj;
    const bool batch_sub = P.batch_sub;
    std::vector<BatchSpec> spec(k);
    ctx->ws_base = 0;
    st = ws_reserve(ctx, P.total());
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

    // Step 2: AP on every block, all blocks in one batch (the flags apply to
    // Step 4 only; S was checked above).
    std::vector<apx_result> subres(k);
    apx_params sp = *params;
    sp.flags = 0;
    params = &sp;
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

    // Step 4: AP on the whole S from A' (R_0 = 0).  With contiguous parts
    // the solve is told each row's block of A', so its availabilities can
    // stay implicit (A' enters as lambda^t a'(i,k) inside the blocks); the
    // 1024-thread passes keep a row's block chunks in at most three float4
    // registers per thread, which bounds a part to 2 * 4096 - 3 points.
    apx_params fp = *orig_params;
    fp.flags &= ~(uint32_t)APX_CHECK_FINITE;
    bool contiguous = true;
    for (int64_t i = 0; i < n && contiguous; ++i) contiguous = pm[i] == i;
    int64_t maxpart = 0;
    for (int j = 0; j < k; ++j) maxpart = nj[j] > maxpart ? nj[j] : maxpart;
    const bool blocks = contiguous && k >= 2 && n > 4096 && maxpart <= 2 * 4096 - 3;
    if (blocks) {
        std::vector<int32_t> hb(2 * (size_t)n);
        for (int j = 0; j < k; ++j)
            for (int64_t i = off[j]; i < off[j + 1]; ++i) {
                hb[2 * i] = (int32_t)off[j];
                hb[2 * i + 1] = (int32_t)off[j + 1];
            }
        HIP_TRY(hipMemcpyAsync(b, hb.data(), sizeof(int32_t) * 2 * (size_t)n, hipMemcpyHostToDevice, s), "blocks");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        ctx->warm_blk = reinterpret_cast<const int32_t *>(b);
        ctx->ws_base = P.blk_bytes;
    }
    st = ap_solve(ctx, S, n, ld, R, A, APX_WARM_A, &fp, idx, res);
    ctx->warm_blk = nullptr;
    ctx->ws_base = 0;
    return st;
}
