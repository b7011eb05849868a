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
    const int64_t *pts;      // nullable: point i is X row pts[i] (else row i)
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
        xs[pp * ldl + j] = ii < a.n ? a.X[(a.pts ? a.pts[ii] : ii) * a.ldx + j] : 0.0f;
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
    const int64_t gi = a.pts ? a.pts[i] : i;    // the point's row (global index)
    const float *xi = a.X + gi * a.ldx;
    if (a.is_ex != nullptr && a.is_ex[gi]) {
        a.idx[i] = (int32_t)gi;
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
    int best = e1 < m ? e1 : -1;
    double bestd;
    if (best >= 0 && (double)d2 - (double)d1 > w) {
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
    if (best < 0 || best >= m) {   // no finite distance (non-finite input)
        a.idx[i] = -1;
        a.dist[i] = NAN;
        return;
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

namespace {
// APX_EINVAL unless every coordinate of X is finite (every point takes part
// in an assignment); synchronises the stream.
apx_status check_points_finite(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx) {
    hipStream_t s = ctx->stream;
    int32_t *hflag = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 2048);
    HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(ctx->dflag), sizeof(int32_t), 0, s), "finite check");
    HIP_TRY(launch_check_finite(X, n, d, ldx, ctx->dflag, s), "finite check");
    HIP_TRY(hipMemcpyAsync(hflag, ctx->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "finite check");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (*hflag) return set_err(ctx, APX_EINVAL, "X holds a NaN or infinite value");
    return APX_OK;
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
    {
        const apx_status fs = check_points_finite(ctx, X, n, d, ldx);
        if (fs != APX_OK) return fs;
    }

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

// ===========================================================================
// Algorithm 3, Steps 1-4 (lap_full_solve).
//
// Step 1  AP on the landmarks M: centres C1, each landmark's class.
// Step 2  max_distance(c): the largest FP64 squared distance of a landmark of
//         class c to c.  Every other point goes to its nearest centre c
//         (certified, lowest index on ties) if its distance is strictly below
//         max_distance(c); the rest, U, stay unassigned.
// Step 3  |U| <= m0: AP on U; |U| > m0: the whole method on U, with
//         min(L, m0) landmarks drawn from U.  Their centres join C1.
// Step 4  Every point of the level goes to its nearest merged centre; each
//         class's centre becomes its medoid (the member of least summed FP64
//         squared distance to the class, Section 2's energy for fixed
//         classes; lowest index on ties); the refined centres are returned.
// The top level finally gives every point its nearest refined centre.
// Every AP after the top-level landmark AP uses that AP's preference p.
// The per-level device buffers are shared (levels run one after another;
// the host keeps each level's point and centre lists).
// ===========================================================================
namespace {

__global__ void k_fill_labels(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// FP64 squared distance of point pairs (a[i], b[i]).
__global__ void k_pair_dist(const float *X, int64_t ldx, int64_t d, const int64_t *a, const int64_t *b, int64_t m,
                            double *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = sqdist64(X + a[i] * ldx, X + b[i] * ldx, d);
}

// Step 2's test: flag[i] = 1 when point i stays unassigned, i.e. its distance
// to its nearest centre lab[i] is not below that centre's max_distance
// (centres: ascending global indices, maxd in the same order).
__global__ void k_lap_threshold(const int32_t *lab, const double *dist, int64_t m, const int64_t *cent, int32_t nc,
                                const double *maxd, uint8_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = lab[i];
        int lo = 0, hi = nc;   // lower bound of c in cent
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cent[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        flag[i] = (lo < nc && cent[lo] == c && dist[i] < maxd[lo]) ? 0 : 1;
    }
}

// Summed FP64 squared distance of candidate q (a member of its class) to
// every member of the class: one workgroup per candidate, members split over
// the threads in a fixed way and reduced in a fixed order.
__global__ __launch_bounds__(256) void k_medoid_sums(const float *X, int64_t ldx, int64_t d, const int64_t *members,
                                                     const int64_t *offsets, const int32_t *cls, double *tot) {
    __shared__ double sh[256];
    const int64_t q = blockIdx.x;
    const int32_t c = cls[q];
    const int64_t b0 = offsets[c], b1 = offsets[c + 1];
    const float *xq = X + members[q] * ldx;
    double acc = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) acc = __dadd_rn(acc, sqdist64(X + members[i] * ldx, xq, d));
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = __dadd_rn(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[q] = sh[0];
}

// The medoid of each class: least summed distance, lowest member on ties
// (members ascending within a class).  One wavefront per class.
__global__ __launch_bounds__(64) void k_medoid_pick(const int64_t *members, const int64_t *offsets, const double *tot,
                                                    int32_t nclass, int64_t *med) {
    const int c = blockIdx.x;
    if (c >= nclass) return;
    const int64_t b0 = offsets[c], b1 = offsets[c + 1];
    double best = INFINITY;
    int64_t bq = -1;
    for (int64_t q = b0 + threadIdx.x; q < b1; q += 64) {
        if (tot[q] < best) {   // ascending q within a lane: a tie keeps the lower member
            best = tot[q];
            bq = q;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int64_t oq = __shfl_xor(bq, off, 64);
        if (ob < best || (ob == best && oq >= 0 && (bq < 0 || oq < bq))) {
            best = ob;
            bq = oq;
        }
    }
    if (threadIdx.x == 0) med[c] = bq >= 0 ? members[bq] : -1;
}

struct LapFull {
    apx_ctx *ctx;
    hipStream_t s;
    const float *X;
    int64_t n, d, ldx, L, m0, amax, lda;
    uint64_t seed;
    double noise_rel;
    apx_params prm;
    double p;              // the top-level landmark AP's preference
    int32_t pref_mode;     // of the top-level landmark AP
    // device buffers (workspace head)
    int64_t *dpts, *dlist2, *dmem, *doff;
    int32_t *dlab, *dcls, *dapidx, *dcount;
    double *ddist, *dtot, *dmaxd, *dsum;
    uint8_t *dflag, *dexf;
    int64_t *dcent, *dmed;
    float *dEX, *dXS, *dS, *dR, *dA;
    size_t head;
    // statistics of the top level
    apx_lap_stats st;
    apx_result top;
    int depth;
};

size_t lapf_head(int64_t n, int64_t d, int64_t L, int64_t m0, int64_t *amax_out, int64_t *lda_out) {
    const int64_t amax = L > m0 ? L : m0;
    const int64_t lda = round64(amax);
    const int64_t cmax = n;               // centres at any level (recursion can add up)
    WsLayout W;
    W.take(sizeof(int64_t) * n);          // dpts
    W.take(sizeof(int64_t) * n);          // dlist2
    W.take(sizeof(int64_t) * n);          // dmem
    W.take(sizeof(int64_t) * (n + 1));    // doff
    W.take(sizeof(int32_t) * n);          // dlab
    W.take(sizeof(int32_t) * n);          // dcls
    W.take(sizeof(int32_t) * amax);       // dapidx
    W.take(sizeof(int32_t) * 4);          // dcount
    W.take(sizeof(double) * n);           // ddist
    W.take(sizeof(double) * n);           // dtot
    W.take(sizeof(double) * cmax);        // dmaxd
    W.take(sizeof(double) * 2);           // dsum
    W.take((size_t)n);                    // dflag
    W.take((size_t)n);                    // dexf
    W.take(sizeof(int64_t) * cmax);       // dcent
    W.take(sizeof(int64_t) * cmax);       // dmed
    W.take(sizeof(float) * cmax * d);     // dEX
    W.take(sizeof(float) * amax * d);     // dXS
    W.take(sizeof(float) * amax * lda);   // dS
    W.take(sizeof(float) * amax * lda);   // dR
    W.take(sizeof(float) * amax * lda);   // dA
    *amax_out = amax;
    *lda_out = lda;
    return W.off;
}

void lapf_carve(LapFull &F, char *b) {
    WsLayout W;
    auto take = [&](size_t bytes) { return b + W.take(bytes); };
    const int64_t n = F.n, d = F.d, amax = F.amax, lda = F.lda, cmax = n;
    F.dpts = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * n));
    F.dlist2 = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * n));
    F.dmem = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * n));
    F.doff = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * (n + 1)));
    F.dlab = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * n));
    F.dcls = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * n));
    F.dapidx = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * amax));
    F.dcount = reinterpret_cast<int32_t *>(take(sizeof(int32_t) * 4));
    F.ddist = reinterpret_cast<double *>(take(sizeof(double) * n));
    F.dtot = reinterpret_cast<double *>(take(sizeof(double) * n));
    F.dmaxd = reinterpret_cast<double *>(take(sizeof(double) * cmax));
    F.dsum = reinterpret_cast<double *>(take(sizeof(double) * 2));
    F.dflag = reinterpret_cast<uint8_t *>(take((size_t)n));
    F.dexf = reinterpret_cast<uint8_t *>(take((size_t)n));
    F.dcent = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * cmax));
    F.dmed = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * cmax));
    F.dEX = reinterpret_cast<float *>(take(sizeof(float) * cmax * d));
    F.dXS = reinterpret_cast<float *>(take(sizeof(float) * amax * d));
    F.dS = reinterpret_cast<float *>(take(sizeof(float) * amax * lda));
    F.dR = reinterpret_cast<float *>(take(sizeof(float) * amax * lda));
    F.dA = reinterpret_cast<float *>(take(sizeof(float) * amax * lda));
}

#define LF_HIP(expr, what)                                            \
    do {                                                              \
        hipError_t _e = (expr);                                       \
        if (_e != hipSuccess) return hip_err(F.ctx, _e, what);        \
    } while (0)
#define LF_TRY(expr)                       \
    do {                                   \
        apx_status _st = (expr);           \
        if (_st != APX_OK) return _st;     \
    } while (0)

int grid_of(int64_t m) { return (int)(m / 256 + 1 < 4096 ? m / 256 + 1 : 4096); }

// AP on the points `pts` (ascending global indices, at least two): centres
// (ascending) and, if cls is given, each point's centre (Algorithm 1's
// labels).  pref_mode / pref_scalar as ap_similarity; *pref receives p.
apx_status lapf_ap(LapFull &F, const std::vector<int64_t> &pts, int32_t pref_mode, float pref_scalar, uint64_t seed,
                   std::vector<int64_t> &centres, std::vector<int64_t> *cls, double *pref, apx_result *res) {
    const int64_t m = (int64_t)pts.size();
    hipStream_t s = F.s;
    LF_HIP(hipMemcpyAsync(F.dpts, pts.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s), "point list");
    k_gather_rows<<<(unsigned)(m < 8192 ? m : 8192), 128, 0, s>>>(F.X, F.ldx, F.d, F.dpts, m, F.dXS, F.d);
    LF_HIP(hipGetLastError(), "gather");
    F.ctx->ws_base = F.head;
    double pv = NAN;
    apx_status st = ap_similarity(F.ctx, F.dXS, m, F.d, F.d, F.dS, F.lda, pref_mode, nullptr, pref_scalar, seed,
                                  F.noise_rel, &pv);
    apx_result r{};
    if (st == APX_OK) st = ap_solve(F.ctx, F.dS, m, F.lda, F.dR, F.dA, APX_COLD, &F.prm, F.dapidx, &r);
    F.ctx->ws_base = 0;
    if (st != APX_OK) return st;
    std::vector<int32_t> lab(m);
    LF_HIP(hipMemcpyAsync(lab.data(), F.dapidx, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s), "labels");
    LF_HIP(hipStreamSynchronize(s), "sync");
    centres.clear();
    for (int64_t i = 0; i < m; ++i)
        if (lab[i] == i) centres.push_back(pts[i]);
    if (cls) {
        cls->resize(m);
        for (int64_t i = 0; i < m; ++i) (*cls)[i] = lab[i] >= 0 ? pts[lab[i]] : -1;
    }
    if (pref) *pref = pv;
    if (res) *res = r;
    return APX_OK;
}

// Nearest centre (certified, lowest index on ties) of m points: the points
// are X rows dpts[0..m) (or rows 0..m-1 when dpts is null); centres
// ascending global indices; with `own` the centres label themselves.
// Results in out_lab (global centre index) and F.ddist (FP64 distance).
apx_status lapf_assign(LapFull &F, const int64_t *dpts, int64_t m, const std::vector<int64_t> &cent, bool own,
                       int32_t *out_lab) {
    hipStream_t s = F.s;
    const int32_t nc = (int32_t)cent.size();
    LF_HIP(hipMemcpyAsync(F.dcent, cent.data(), sizeof(int64_t) * nc, hipMemcpyHostToDevice, s), "centres");
    LF_HIP(hipMemcpyAsync(F.dcount, &nc, sizeof(int32_t), hipMemcpyHostToDevice, s), "count");
    k_gather_rows<<<(unsigned)(nc < 8192 ? (nc > 0 ? nc : 1) : 8192), 128, 0, s>>>(F.X, F.ldx, F.d, F.dcent, nc, F.dEX,
                                                                                   F.d);
    LF_HIP(hipGetLastError(), "gather centres");
    if (own) {
        k_clear_flags<<<256, 256, 0, s>>>(F.dexf, F.n);
        k_flag_exemplars<<<1, 256, 0, s>>>(F.dexf, F.dcent, nc);
        LF_HIP(hipGetLastError(), "centre flags");
    }
    AssignArgs aa{};
    aa.X = F.X;
    aa.n = m;
    aa.d = F.d;
    aa.ldx = F.ldx;
    aa.pts = dpts;
    aa.ex = F.dcent;
    aa.EX = F.dEX;
    aa.ldE = F.d;
    aa.m_dev = F.dcount;
    aa.is_ex = own ? F.dexf : nullptr;
    aa.idx = out_lab;
    aa.dist = F.ddist;
    const double u = std::ldexp(1.0, -24);
    aa.gamma = (double)(F.d + 2) * u / (1.0 - (double)(F.d + 2) * u);
    const size_t lds = sizeof(float) * (size_t)(PT + 64) * (size_t)(F.d + 1);
    const size_t ldsx = lds > 3 * 1024 ? lds : 3 * 1024;
    LF_HIP(hipFuncSetAttribute((const void *)k_lap_assign, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsx),
           "lds");
    k_lap_assign<<<(unsigned)((m + PT - 1) / PT), 256, ldsx, s>>>(aa);
    LF_HIP(hipGetLastError(), "assign");
    return APX_OK;
}

// Step 4's refinement on the level's points P (sorted; identity when null
// and |P| = n) and merged centres C: classes by nearest centre, then each
// class's medoid.  E receives the medoids, ascending.
apx_status lapf_refine(LapFull &F, const std::vector<int64_t> *P, const std::vector<int64_t> &C,
                       std::vector<int64_t> &E) {
    hipStream_t s = F.s;
    const int64_t m = P ? (int64_t)P->size() : F.n;
    if (P) LF_HIP(hipMemcpyAsync(F.dpts, P->data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s), "points");
    LF_TRY(lapf_assign(F, P ? F.dpts : nullptr, m, C, true, F.dlab));
    std::vector<int32_t> lab(m);
    LF_HIP(hipMemcpyAsync(lab.data(), F.dlab, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s), "labels");
    LF_HIP(hipStreamSynchronize(s), "sync");
    // members by class (classes in the order of C, members ascending)
    const int32_t nc = (int32_t)C.size();
    std::vector<int64_t> off(nc + 1, 0), mem(m);
    std::vector<int32_t> cpos(m), cls(m);
    for (int64_t i = 0; i < m; ++i) {
        cpos[i] = (int32_t)(std::lower_bound(C.begin(), C.end(), (int64_t)lab[i]) - C.begin());
        off[cpos[i] + 1] += 1;
    }
    for (int32_t c = 0; c < nc; ++c) off[c + 1] += off[c];
    {
        std::vector<int64_t> fill(off.begin(), off.end() - 1);
        for (int64_t i = 0; i < m; ++i) {
            const int64_t q = fill[cpos[i]]++;
            mem[q] = P ? (*P)[i] : i;
            cls[q] = cpos[i];
        }
    }
    LF_HIP(hipMemcpyAsync(F.dmem, mem.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, s), "members");
    LF_HIP(hipMemcpyAsync(F.doff, off.data(), sizeof(int64_t) * (nc + 1), hipMemcpyHostToDevice, s), "offsets");
    LF_HIP(hipMemcpyAsync(F.dcls, cls.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, s), "classes");
    k_medoid_sums<<<(unsigned)m, 256, 0, s>>>(F.X, F.ldx, F.d, F.dmem, F.doff, F.dcls, F.dtot);
    LF_HIP(hipGetLastError(), "medoid sums");
    k_medoid_pick<<<(unsigned)nc, 64, 0, s>>>(F.dmem, F.doff, F.dtot, nc, F.dmed);
    LF_HIP(hipGetLastError(), "medoid pick");
    E.resize(nc);
    LF_HIP(hipMemcpyAsync(E.data(), F.dmed, sizeof(int64_t) * nc, hipMemcpyDeviceToHost, s), "medoids");
    LF_HIP(hipStreamSynchronize(s), "sync");
    std::sort(E.begin(), E.end());
    E.erase(std::unique(E.begin(), E.end()), E.end());
    return APX_OK;
}

// Uniform sample of `count` of m positions (ascending): the first `count`
// slots of a Fisher-Yates shuffle driven by the SplitMix64 stream.
std::vector<int64_t> sample_positions(int64_t m, int64_t count, uint64_t seed) {
    std::vector<int64_t> pool(m);
    for (int64_t i = 0; i < m; ++i) pool[i] = i;
    uint64_t state = seed;
    for (int64_t i = 0; i < count; ++i) {
        const int64_t j = i + (int64_t)(splitmix_next(state) % (uint64_t)(m - i));
        std::swap(pool[i], pool[j]);
    }
    std::vector<int64_t> out(pool.begin(), pool.begin() + count);
    std::sort(out.begin(), out.end());
    return out;
}

// One level of the method on points P (ascending; all n points at the top)
// with landmarks M (ascending, a subset of P): its refined centres.
apx_status lapf_level(LapFull &F, const std::vector<int64_t> *P, const std::vector<int64_t> &M, int lev,
                      std::vector<int64_t> &E) {
    if (lev >= 64) return set_err(F.ctx, APX_ENOTIMPL, "LAP recursion deeper than 64 levels");
    F.depth = lev + 1 > F.depth ? lev + 1 : F.depth;
    hipStream_t s = F.s;
    const uint64_t sd = F.seed + 3ull * (uint64_t)lev;
    // Step 1
    std::vector<int64_t> C1, cls;
    apx_result r1{};
    if (lev == 0) {
        double p = NAN;
        LF_TRY(lapf_ap(F, M, F.pref_mode, (float)F.p, sd, C1, &cls, &p, &r1));
        F.p = p;
        F.top = r1;
    } else {
        LF_TRY(lapf_ap(F, M, APX_PREF_SCALAR, (float)F.p, sd, C1, &cls, nullptr, &r1));
    }
    // Step 2: the points of P that are not landmarks
    std::vector<int64_t> Q;
    {
        const int64_t np = P ? (int64_t)P->size() : F.n;
        Q.reserve(np - (int64_t)M.size());
        size_t mi = 0;
        for (int64_t q = 0; q < np; ++q) {
            const int64_t g = P ? (*P)[q] : q;
            while (mi < M.size() && M[mi] < g) ++mi;
            if (mi < M.size() && M[mi] == g) continue;
            Q.push_back(g);
        }
    }
    std::vector<int64_t> U;
    int64_t assigned = 0;
    if (!C1.empty() && !Q.empty()) {
        // max_distance per class from the landmarks' FP64 distances
        const int64_t mL = (int64_t)M.size();
        LF_HIP(hipMemcpyAsync(F.dpts, M.data(), sizeof(int64_t) * mL, hipMemcpyHostToDevice, s), "landmarks");
        LF_HIP(hipMemcpyAsync(F.dlist2, cls.data(), sizeof(int64_t) * mL, hipMemcpyHostToDevice, s), "classes");
        k_pair_dist<<<grid_of(mL), 256, 0, s>>>(F.X, F.ldx, F.d, F.dpts, F.dlist2, mL, F.dtot);
        LF_HIP(hipGetLastError(), "landmark distances");
        std::vector<double> dl(mL);
        LF_HIP(hipMemcpyAsync(dl.data(), F.dtot, sizeof(double) * mL, hipMemcpyDeviceToHost, s), "distances");
        LF_HIP(hipStreamSynchronize(s), "sync");
        std::vector<double> maxd(C1.size(), 0.0);
        for (int64_t i = 0; i < mL; ++i) {
            const size_t c = (size_t)(std::lower_bound(C1.begin(), C1.end(), cls[i]) - C1.begin());
            if (c < C1.size() && C1[c] == cls[i] && dl[i] > maxd[c]) maxd[c] = dl[i];
        }
        // nearest centre of every other point, then the threshold
        const int64_t mq = (int64_t)Q.size();
        LF_HIP(hipMemcpyAsync(F.dlist2, Q.data(), sizeof(int64_t) * mq, hipMemcpyHostToDevice, s), "points");
        LF_TRY(lapf_assign(F, F.dlist2, mq, C1, false, F.dlab));
        LF_HIP(hipMemcpyAsync(F.dmaxd, maxd.data(), sizeof(double) * maxd.size(), hipMemcpyHostToDevice, s), "maxd");
        k_lap_threshold<<<grid_of(mq), 256, 0, s>>>(F.dlab, F.ddist, mq, F.dcent, (int32_t)C1.size(), F.dmaxd,
                                                   F.dflag);
        LF_HIP(hipGetLastError(), "threshold");
        std::vector<uint8_t> fl(mq);
        LF_HIP(hipMemcpyAsync(fl.data(), F.dflag, (size_t)mq, hipMemcpyDeviceToHost, s), "flags");
        LF_HIP(hipStreamSynchronize(s), "sync");
        for (int64_t q = 0; q < mq; ++q) {
            if (fl[q]) U.push_back(Q[q]);
            else ++assigned;
        }
    } else {
        U = Q;
    }
    // Step 3
    std::vector<int64_t> C3;
    int mode = 0;
    if (U.size() == 1) {
        C3 = U;
        mode = 1;
    } else if (U.size() >= 2 && (int64_t)U.size() <= F.m0) {
        LF_TRY(lapf_ap(F, U, APX_PREF_SCALAR, (float)F.p, sd + 1, C3, nullptr, nullptr, nullptr));
        mode = 1;
    } else if ((int64_t)U.size() > F.m0) {
        const int64_t Lr = F.L < F.m0 ? F.L : F.m0;
        std::vector<int64_t> pos = sample_positions((int64_t)U.size(), Lr, F.seed + 3ull * (uint64_t)(lev + 1));
        std::vector<int64_t> Mr(Lr);
        for (int64_t i = 0; i < Lr; ++i) Mr[i] = U[pos[i]];
        LF_TRY(lapf_level(F, &U, Mr, lev + 1, C3));
        mode = 2;
    }
    std::vector<int64_t> C;
    std::set_union(C1.begin(), C1.end(), C3.begin(), C3.end(), std::back_inserter(C));
    if (lev == 0) {
        F.st.step1_centres = (int32_t)C1.size();
        F.st.assigned = assigned;
        F.st.unassigned = (int64_t)U.size();
        F.st.merged_centres = (int32_t)C.size();
        F.st.step3_mode = mode;
    }
    // Step 4
    if (C.empty()) {
        E.clear();
        return APX_OK;
    }
    return lapf_refine(F, P, C, E);
}

}  // namespace

size_t apx::lap_full_ws_bytes(int64_t n, int64_t d, int64_t L, int64_t m0, int num_cus) {
    int64_t amax = 0, lda = 0;
    const size_t head = lapf_head(n, d, L, m0, &amax, &lda);
    const size_t sim = similarity_ws_bytes(amax), sol = solve_ws_bytes(amax, lda, num_cus);
    return head + (sim > sol ? sim : sol);
}

extern "C" apx_status lap_full_solve(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                                     int64_t n_landmarks, const int64_t *landmarks, uint64_t seed, double noise_rel,
                                     int32_t pref_mode, float pref_scalar, int64_t m0, const apx_params *params,
                                     int32_t *idx, apx_result *res, apx_lap_stats *stats, int64_t *exemplars_out) {
    if (!ctx) return APX_EINVAL;
    if (!X || !idx || !res || !params) return set_err(ctx, APX_EINVAL, "null argument");
    if (n < 2 || d < 1 || ldx < d) return set_err(ctx, APX_EINVAL, "need n >= 2, d >= 1, ldx >= d");
    if (n_landmarks < 2 || n_landmarks > n) return set_err(ctx, APX_EINVAL, "need 2 <= n_landmarks <= n");
    if (m0 < 2) return set_err(ctx, APX_EINVAL, "need m0 >= 2");
    if (n > ((int64_t)1 << 31) - 1) return set_err(ctx, APX_ENOTIMPL, "n too large");
    if (d > 300) return set_err(ctx, APX_ENOTIMPL, "d > 300 (assignment tile)");
    {
        const apx_status ps = check_params(ctx, params);
        if (ps != APX_OK) return ps;
    }
    if (params->flags & APX_RAW_LABELS)
        return set_err(ctx, APX_EINVAL, "APX_RAW_LABELS does not apply to lap_full_solve (labels are assignments)");
    if (pref_mode != APX_PREF_MEDIAN && pref_mode != APX_PREF_SCALAR)
        return set_err(ctx, APX_EINVAL, "lap_full_solve takes APX_PREF_MEDIAN or APX_PREF_SCALAR");
    if (pref_mode == APX_PREF_SCALAR && !std::isfinite(pref_scalar))
        return set_err(ctx, APX_EINVAL, "pref_scalar is not finite");
    const int64_t L = n_landmarks;
    std::vector<int64_t> M;
    if (landmarks) {
        std::vector<char> seen(n, 0);
        M.assign(landmarks, landmarks + L);
        for (int64_t v : M) {
            if (v < 0 || v >= n || seen[v]) return set_err(ctx, APX_EINVAL, "landmarks must be distinct indices in [0, n)");
            seen[v] = 1;
        }
        std::sort(M.begin(), M.end());
    } else {
        M = sample_positions(n, L, seed);
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);

    LapFull F{};
    F.ctx = ctx;
    F.s = ctx->stream;
    F.X = X;
    F.n = n;
    F.d = d;
    F.ldx = ldx;
    F.L = L;
    F.m0 = m0;
    F.seed = seed;
    F.noise_rel = noise_rel;
    F.prm = *params;
    F.prm.flags &= ~(uint32_t)APX_CHECK_FINITE;
    F.head = lapf_head(n, d, L, m0, &F.amax, &F.lda);
    const size_t sim = similarity_ws_bytes(F.amax), sol = solve_ws_bytes(F.amax, F.lda, ctx->num_cus);
    ctx->ws_base = 0;
    apx_status st = ws_reserve(ctx, F.head + (sim > sol ? sim : sol));
    if (st != APX_OK) return st;
    lapf_carve(F, static_cast<char *>(ctx->ws));
    // every point takes part in the assignments: non-finite X is rejected first
    st = check_points_finite(ctx, X, n, d, ldx);
    if (st != APX_OK) return st;
    F.pref_mode = pref_mode;
    F.p = pref_scalar;
    std::vector<int64_t> E;
    st = lapf_level(F, nullptr, M, 0, E);
    ctx->ws_base = 0;
    if (st != APX_OK) return st;
    F.st.levels = F.depth;
    F.st.refined_centres = (int32_t)E.size();
    hipStream_t s = F.s;
    std::memset(res, 0, sizeof *res);
    res->iterations = F.top.iterations;
    res->converged = F.top.converged;
    res->n_exemplars = (int32_t)E.size();
    res->status = APX_OK;
    if (E.empty()) {
        k_fill_labels<<<grid_of(n), 256, 0, s>>>(idx, n, -1);
        HIP_TRY(hipGetLastError(), "labels");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        res->dpsim = res->expref = res->netsim = NAN;
    } else {
        // every point to its nearest refined centre
        st = lapf_assign(F, nullptr, n, E, true, idx);
        if (st != APX_OK) return st;
        k_sum_f64<<<1, 1024, 0, s>>>(F.ddist, n, F.dsum);
        HIP_TRY(hipGetLastError(), "sum");
        double hs = 0.0;
        HIP_TRY(hipMemcpyAsync(&hs, F.dsum, sizeof(double), hipMemcpyDeviceToHost, s), "sum");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        res->dpsim = -hs;
        res->expref = F.p * (double)E.size();
        res->netsim = res->dpsim + res->expref;
    }
    if (exemplars_out && !E.empty()) std::memcpy(exemplars_out, E.data(), sizeof(int64_t) * E.size());
    if (stats) {
        *stats = F.st;
        stats->preference = F.p;
    }
    return APX_OK;
}

// Landmark set for Step 1 of Algorithm 3 from given points (a previous run's
// exemplars, say) plus a uniform sample of the others (host only).
extern "C" apx_status apx_lap_landmarks(int64_t n, int64_t n_landmarks, const int64_t *keep, int64_t n_keep,
                                        uint64_t seed, int64_t *out) {
    if (n < 1 || n_landmarks < 1 || n_landmarks > n || n_keep < 0 || n_keep > n_landmarks || !out ||
        (n_keep > 0 && !keep))
        return APX_EINVAL;
    std::vector<char> kept(n, 0);
    for (int64_t i = 0; i < n_keep; ++i) {
        if (keep[i] < 0 || keep[i] >= n || kept[keep[i]]) return APX_EINVAL;
        kept[keep[i]] = 1;
    }
    std::vector<int64_t> rest;
    rest.reserve(n - n_keep);
    for (int64_t i = 0; i < n; ++i)
        if (!kept[i]) rest.push_back(i);
    const std::vector<int64_t> pos = sample_positions((int64_t)rest.size(), n_landmarks - n_keep, seed);
    std::vector<int64_t> M(keep, keep + n_keep);
    for (int64_t p : pos) M.push_back(rest[p]);
    std::sort(M.begin(), M.end());
    std::memcpy(out, M.data(), sizeof(int64_t) * (size_t)n_landmarks);
    return APX_OK;
}
