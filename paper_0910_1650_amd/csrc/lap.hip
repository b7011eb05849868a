// lap.hip -- landmark affinity propagation (Section 4, Algorithm 3, Steps 1-2).
//
// Step 1: AP on a uniform random sample M of landmark points (similarity
// built on matrix cores, median preference, tie noise).  Step 2 (without the
// per-class distance threshold): every point goes to the exemplar at the
// least squared Euclidean distance; exemplars label themselves.  The full
// n x n similarity matrix is never formed.
//
// Assignment is exact: squared distances are first computed in FP32 (direct
// difference form), and a point whose best and runner-up distances are not
// separated by more than the FP32 error bound gamma_{d+2} * (d1 + d_e) has all
// candidates inside that window recomputed in FP64 in ascending coordinate
// order; ties go to the lowest exemplar index.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "apx_internal.h"

using namespace apx;

namespace {

constexpr int PT = 64;        // points per workgroup
constexpr int NG = 4;         // exemplar groups per point (256 threads)

__global__ void k_gather_rows(const float *X, int64_t ldx, int64_t d, const int64_t *rows,
                              int64_t m, float *out, int64_t ldo) {
    for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
        const float *src = X + rows[r] * ldx;
        for (int64_t j = threadIdx.x; j < d; j += blockDim.x) out[r * ldo + j] = src[j];
    }
}

// Compact the landmark-level exemplar flags into ascending global indices.
__global__ void k_lap_exemplars(const int32_t *lab, const int64_t *landmarks, int64_t m,
                                int64_t *ex, int32_t *count) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t c = 0;
    for (int64_t i = 0; i < m; ++i)
        if (lab[i] == i) ex[c++] = landmarks[i];
    // ascending global order (landmarks are sorted ascending by the host)
    *count = c;
}

__device__ __forceinline__ double sqdist64(const float *x, const float *y, int64_t d) {
    double acc = 0.0;
    for (int64_t j = 0; j < d; ++j) {
        const double diff = __dsub_rn((double)x[j], (double)y[j]);
        acc = __dadd_rn(acc, __dmul_rn(diff, diff));
    }
    return acc;
}

struct AssignArgs {
    const float *X;
    int64_t n, d, ldx;
    const int64_t *ex;       // exemplar global indices, ascending
    const float *EX;         // exemplar coordinates, m x ldE
    int64_t ldE;
    const int32_t *m_dev;    // number of exemplars
    const uint8_t *is_ex;    // n flags
    int32_t *idx;
    double *dist;            // FP64 distance of each point to its exemplar (0 for exemplars)
    double gamma;            // FP32 error factor of one squared distance
};

// One workgroup: 64 points x 4 exemplar groups.  Exemplar coordinates are
// streamed through LDS in chunks; each thread keeps the best two FP32
// distances of its group; groups are merged in a fixed order.
__global__ __launch_bounds__(256) void k_lap_assign(AssignArgs a) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    const int p = tid % PT, g = tid / PT;
    const int64_t i = (int64_t)blockIdx.x * PT + p;
    const int m = *a.m_dev;
    const int64_t d = a.d;
    const int ldl = (int)d + 1;                 // padded row in LDS
    float *xs = lds;                            // PT x ldl points
    float *es = lds + PT * ldl;                 // chunk of exemplars, ECH x ldl
    const int ECH = 64;
    for (int e = tid; e < PT * (int)d; e += blockDim.x) {
        const int pp = e / (int)d, j = e % (int)d;
        const int64_t ii = (int64_t)blockIdx.x * PT + pp;
        xs[pp * ldl + j] = ii < a.n ? a.X[ii * a.ldx + j] : 0.0f;
    }
    float d1 = INFINITY, d2 = INFINITY;
    int e1 = INT32_MAX;
    for (int e0 = 0; e0 < m; e0 += ECH) {
        const int ne = (m - e0) < ECH ? (m - e0) : ECH;
        __syncthreads();
        for (int e = tid; e < ne * (int)d; e += blockDim.x) {
            const int q = e / (int)d, j = e % (int)d;
            es[q * ldl + j] = a.EX[(int64_t)(e0 + q) * a.ldE + j];
        }
        __syncthreads();
        for (int q = g; q < ne; q += NG) {
            float acc = 0.0f;
            const float *xp = xs + p * ldl;
            const float *ep = es + q * ldl;
            for (int j = 0; j < (int)d; ++j) {
                const float diff = xp[j] - ep[j];
                acc = fmaf(diff, diff, acc);
            }
            const int ei = e0 + q;   // exemplars are visited in ascending order per thread
            if (acc < d1) {
                d2 = d1;
                d1 = acc;
                e1 = ei;
            } else {
                d2 = fminf(d2, acc);
            }
        }
    }
    // merge the 4 groups of each point (fixed order g = 0..3)
    __syncthreads();
    float *md1 = lds, *md2 = lds + 256;
    int *me1 = reinterpret_cast<int *>(lds + 512);
    md1[tid] = d1;
    md2[tid] = d2;
    me1[tid] = e1;
    __syncthreads();
    if (g != 0 || i >= a.n) return;
    for (int gg = 1; gg < NG; ++gg) {
        const float od1 = md1[gg * PT + p], od2 = md2[gg * PT + p];
        const int oe1 = me1[gg * PT + p];
        const bool take = od1 < d1 || (od1 == d1 && oe1 < e1);
        const float nd2 = take ? fminf(od2, d1) : fminf(d2, od1);
        d1 = take ? od1 : d1;
        e1 = take ? oe1 : e1;
        d2 = nd2;
    }
    const float *xi = a.X + i * a.ldx;
    if (a.is_ex[i]) {
        a.idx[i] = (int32_t)i;
        a.dist[i] = 0.0;
        return;
    }
    if (m == 0) {
        a.idx[i] = -1;
        a.dist[i] = 0.0;
        return;
    }
    // Certified when every other exemplar is farther than the FP32 error window.
    const double w = a.gamma * 2.0 * ((double)d1 + (double)d2);
    int best = e1;
    double bestd;
    if ((double)d2 - (double)d1 > w) {
        bestd = sqdist64(xi, a.EX + (int64_t)e1 * a.ldE, d);
    } else {
        // FP64 recheck of every candidate whose FP32 distance is within the
        // window (ascending exemplar index: strict improvement keeps the
        // lowest index on exact ties).
        bestd = INFINITY;
        best = -1;
        for (int e = 0; e < m; ++e) {
            const float *ep = a.EX + (int64_t)e * a.ldE;
            float acc = 0.0f;
            for (int64_t j = 0; j < d; ++j) {
                const float diff = xi[j] - ep[j];
                acc = fmaf(diff, diff, acc);
            }
            if ((double)acc - (double)d1 > a.gamma * 2.0 * ((double)acc + (double)d1)) continue;
            const double dd = sqdist64(xi, ep, d);
            if (dd < bestd) {
                bestd = dd;
                best = e;
            }
        }
    }
    a.idx[i] = (int32_t)a.ex[best];
    a.dist[i] = bestd;
}

// Deterministic FP64 sum of n values (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_sum_f64(const double *v, int64_t n, double *out) {
    __shared__ double sh[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_clear_flags(uint8_t *flags, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        flags[i] = 0;
}
__global__ void k_flag_exemplars(uint8_t *flags, const int64_t *ex, int32_t m) {
    for (int e = threadIdx.x; e < m; e += blockDim.x) flags[ex[e]] = 1;
}

// SplitMix64 stream for host-side landmark sampling when none are given.
uint64_t splitmix_next(uint64_t &state) {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int64_t round64(int64_t v) { return (v + 63) & ~int64_t(63); }

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)

}  // namespace

namespace {

// Workspace of lap_solve: [landmark tables, X_M, S_M, R_M, A_M, exemplars,
// flags, distances] then the slice of the landmark similarity and solve.
struct LapLayout {
    size_t o_lm, o_xm, o_S, o_R, o_A, o_lab, o_ex, o_m, o_EX, o_flag, o_dist, o_sum, head, tail;
};
LapLayout lap_layout(int64_t n, int64_t d, int64_t L, int num_cus) {
    const int64_t ldL = round64(L), ldm = d;
    WsLayout W;
    LapLayout o{};
    o.o_lm = W.take(sizeof(int64_t) * L);
    o.o_xm = W.take(sizeof(float) * L * ldm);
    o.o_S = W.take(sizeof(float) * L * ldL);
    o.o_R = W.take(sizeof(float) * L * ldL);
    o.o_A = W.take(sizeof(float) * L * ldL);
    o.o_lab = W.take(sizeof(int32_t) * L);
    o.o_ex = W.take(sizeof(int64_t) * L);
    o.o_m = W.take(sizeof(int32_t) * 4);
    o.o_EX = W.take(sizeof(float) * L * ldm);
    o.o_flag = W.take((size_t)n);
    o.o_dist = W.take(sizeof(double) * n);
    o.o_sum = W.take(sizeof(double) * 2);
    o.head = W.off;
    const size_t sim = similarity_ws_bytes(L), sol = solve_ws_bytes(L, ldL, num_cus);
    o.tail = sim > sol ? sim : sol;
    return o;
}

}  // namespace

size_t apx::lap_ws_bytes(int64_t n, int64_t d, int64_t L, int num_cus) {
    const LapLayout o = lap_layout(n, d, L, num_cus);
    return o.head + o.tail;
}

extern "C" apx_status lap_solve(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                                int64_t n_landmarks, const int64_t *landmarks, uint64_t seed,
                                double noise_rel, int32_t pref_mode, float pref_scalar,
                                const apx_params *params, int32_t *idx, apx_result *res,
                                int64_t *exemplars_out) {
    if (!ctx) return APX_EINVAL;
    if (!X || !idx || !res || !params) return set_err(ctx, APX_EINVAL, "null argument");
    if (n < 2 || d < 1 || ldx < d) return set_err(ctx, APX_EINVAL, "need n >= 2, d >= 1, ldx >= d");
    if (n_landmarks < 2 || n_landmarks > n) return set_err(ctx, APX_EINVAL, "need 2 <= n_landmarks <= n");
    if (d > 4096) return set_err(ctx, APX_ENOTIMPL, "d > 4096");
    {
        const apx_status ps = check_params(ctx, params);
        if (ps != APX_OK) return ps;
    }
    if (params->flags & APX_RAW_LABELS)
        return set_err(ctx, APX_EINVAL, "APX_RAW_LABELS does not apply to lap_solve (labels are assignments)");
    if (pref_mode != APX_PREF_MEDIAN && pref_mode != APX_PREF_SCALAR)
        return set_err(ctx, APX_EINVAL, "lap_solve takes APX_PREF_MEDIAN or APX_PREF_SCALAR");
    if (pref_mode == APX_PREF_SCALAR && !std::isfinite(pref_scalar))
        return set_err(ctx, APX_EINVAL, "pref_scalar is not finite");
    const int64_t L = n_landmarks;
    std::vector<int64_t> lm(L);
    if (landmarks) {
        std::vector<char> seen(n, 0);
        for (int64_t i = 0; i < L; ++i) {
            if (landmarks[i] < 0 || landmarks[i] >= n || seen[landmarks[i]])
                return set_err(ctx, APX_EINVAL, "landmarks must be distinct indices in [0, n)");
            seen[landmarks[i]] = 1;
            lm[i] = landmarks[i];
        }
    } else {
        // Algorithm 3, Step 1: uniform sample without replacement (partial
        // Fisher-Yates driven by a SplitMix64 stream from `seed`).
        std::vector<int64_t> pool(n);
        for (int64_t i = 0; i < n; ++i) pool[i] = i;
        uint64_t state = seed;
        for (int64_t i = 0; i < L; ++i) {
            const int64_t j = i + (int64_t)(splitmix_next(state) % (uint64_t)(n - i));
            std::swap(pool[i], pool[j]);
            lm[i] = pool[i];
        }
    }
    std::sort(lm.begin(), lm.end());
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    hipStream_t s = ctx->stream;

    const int64_t ldL = round64(L), ldm = d;
    const LapLayout LL = lap_layout(n, d, L, ctx->num_cus);
    const size_t o_lm = LL.o_lm, o_xm = LL.o_xm, o_S = LL.o_S, o_R = LL.o_R, o_A = LL.o_A, o_lab = LL.o_lab,
                 o_ex = LL.o_ex, o_m = LL.o_m, o_EX = LL.o_EX, o_flag = LL.o_flag, o_dist = LL.o_dist,
                 o_sum = LL.o_sum, head = LL.head;
    ctx->ws_base = 0;
    apx_status st = ws_reserve(ctx, head + LL.tail);
    if (st != APX_OK) return st;
    char *b = static_cast<char *>(ctx->ws);
    int64_t *dlm = reinterpret_cast<int64_t *>(b + o_lm);
    float *XM = reinterpret_cast<float *>(b + o_xm);
    float *SL = reinterpret_cast<float *>(b + o_S);
    float *RL = reinterpret_cast<float *>(b + o_R);
    float *AL = reinterpret_cast<float *>(b + o_A);
    int32_t *lab = reinterpret_cast<int32_t *>(b + o_lab);
    int64_t *ex = reinterpret_cast<int64_t *>(b + o_ex);
    int32_t *dm = reinterpret_cast<int32_t *>(b + o_m);
    float *EX = reinterpret_cast<float *>(b + o_EX);
    uint8_t *flag = reinterpret_cast<uint8_t *>(b + o_flag);
    double *dist = reinterpret_cast<double *>(b + o_dist);
    double *dsum = reinterpret_cast<double *>(b + o_sum);

    HIP_TRY(hipMemcpyAsync(dlm, lm.data(), sizeof(int64_t) * L, hipMemcpyHostToDevice, s), "landmarks");
    k_gather_rows<<<(unsigned)(L < 8192 ? L : 8192), 128, 0, s>>>(X, ldx, d, dlm, L, XM, ldm);
    HIP_TRY(hipGetLastError(), "gather");

    // Step 1: AP on the landmarks.
    ctx->ws_base = head;
    double pref = NAN;
    st = ap_similarity(ctx, XM, L, d, ldm, SL, ldL, pref_mode, nullptr, pref_scalar, seed, noise_rel, &pref);
    if (st == APX_OK) st = ap_solve(ctx, SL, L, ldL, RL, AL, APX_COLD, params, lab, res);
    ctx->ws_base = 0;
    if (st != APX_OK) return st;

    // Step 2: nearest exemplar for every point.
    k_lap_exemplars<<<1, 64, 0, s>>>(lab, dlm, L, ex, dm);
    HIP_TRY(hipGetLastError(), "exemplars");
    int32_t hm = 0;
    HIP_TRY(hipMemcpyAsync(&hm, dm, sizeof(int32_t), hipMemcpyDeviceToHost, s), "count");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (hm > 0) {
        k_gather_rows<<<(unsigned)(hm < 8192 ? hm : 8192), 128, 0, s>>>(X, ldx, d, ex, hm, EX, ldm);
        HIP_TRY(hipGetLastError(), "gather exemplars");
    }
    k_clear_flags<<<256, 256, 0, s>>>(flag, n);
    if (hm > 0) k_flag_exemplars<<<1, 256, 0, s>>>(flag, ex, hm);
    HIP_TRY(hipGetLastError(), "flags");
    AssignArgs aa{};
    aa.X = X;
    aa.n = n;
    aa.d = d;
    aa.ldx = ldx;
    aa.ex = ex;
    aa.EX = EX;
    aa.ldE = ldm;
    aa.m_dev = dm;
    aa.is_ex = flag;
    aa.idx = idx;
    aa.dist = dist;
    const double u = std::ldexp(1.0, -24);
    aa.gamma = (double)(d + 2) * u / (1.0 - (double)(d + 2) * u);
    const size_t lds = sizeof(float) * (size_t)(PT + 64) * (size_t)(d + 1);
    if (lds > 160 * 1024 - 1024) return set_err(ctx, APX_ENOTIMPL, "d too large for the assignment tile");
    HIP_TRY(hipFuncSetAttribute((const void *)k_lap_assign, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(lds > 3 * 1024 ? lds : 3 * 1024)), "lds");
    k_lap_assign<<<(unsigned)((n + PT - 1) / PT), 256, lds > 3 * 1024 ? lds : 3 * 1024, s>>>(aa);
    HIP_TRY(hipGetLastError(), "assign");
    k_sum_f64<<<1, 1024, 0, s>>>(dist, n, dsum);
    HIP_TRY(hipGetLastError(), "sum");
    double hs = 0.0;
    HIP_TRY(hipMemcpyAsync(&hs, dsum, sizeof(double), hipMemcpyDeviceToHost, s), "sum");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (exemplars_out && hm > 0)
        HIP_TRY(hipMemcpy(exemplars_out, ex, sizeof(int64_t) * hm, hipMemcpyDeviceToHost), "exemplars");
    res->n_exemplars = hm;
    if (hm == 0) {
        res->dpsim = res->expref = res->netsim = NAN;
    } else {
        res->dpsim = -hs;
        res->expref = pref * hm;
        res->netsim = res->dpsim + res->expref;
    }
    return APX_OK;
}
