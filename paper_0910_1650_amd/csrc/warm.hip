// warm.hip -- learned warm start for Algorithm 1 (Section 2).
//
// Algorithm 1 starts from zero availabilities (Eq. (1)); the paper's only warm
// start is PAP's merge of sub-problem availabilities (Section 3, Algorithm 2,
// steps 3-4).  This file replaces that merge with a prediction made per point
// from its row of S:
//
//   features   16 numbers per point: order statistics of the off-diagonal row
//              (1st..32nd largest, their top-32 mean, five quantiles),
//              s(k,k) against the row median and the top-32 mean, the share
//              of the row above s(k,k), ln(n)/10; similarities are divided
//              by sigma, the magnitude of the median of the row medians.
//   network    16 -> 128 -> 128 -> 2 with GELU; bf16 weights and activations
//              on the matrix cores with FP32 accumulation; FP32 backward with
//              fixed-order reductions; Adam on FP32 master weights.
//   targets    the column quantities of Eqs. (3)-(4) of a converged run,
//              t_k = r(k,k) + c_k and c_k = sum_{i != k} max(0, r(i,k)),
//              divided by sigma.
//   A_0        a(i,k) = min(0, sigma y0_k) off the diagonal and
//              a(k,k) = max(0, sigma y1_k): Eqs. (3)-(4) with the predicted
//              column quantities.  R_0 = one undamped Eq. (2) step from A_0.
//
// Order statistics are exact: a most-significant-digit radix select over the
// order-preserving integer image of the FP32 values (8-bit digits, four
// passes) serves all eleven ranks of a row at once.
#include <cmath>
#include <cstring>

#include "apx_internal.h"

using namespace apx;

namespace {

constexpr int NF = APX_MLP_FEATURES;   // 16
constexpr int NH = 128;
constexpr int NO = 2;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + NF * NH;
constexpr int OFF_W2 = OFF_B1 + NH;
constexpr int OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH;
constexpr int OFF_B3 = OFF_W3 + NH * NO;
constexpr int NPARAM = OFF_B3 + NO;
static_assert(NPARAM == APX_MLP_PARAMS, "parameter layout");

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)
#define APX_TRY(expr)                       \
    do {                                    \
        apx_status _st = (expr);            \
        if (_st != APX_OK) return _st;      \
    } while (0)

// ---------------------------------------------------------------------------
// Exact multi-rank selection
// ---------------------------------------------------------------------------
constexpr int SEL_T = 1024;
constexpr int NTGT = 11;               // 6 descending ranks + 5 quantiles
constexpr int TOP = 32;

__device__ __forceinline__ uint32_t fkey(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float keyf(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

struct SelShared {
    uint32_t hist[NTGT][256];
    uint32_t pref[NTGT];       // key digits found so far
    int32_t rank[NTGT];        // rank still to find among keys with that prefix
    int32_t slot[NTGT];        // histogram each target reads
    uint32_t slot_pref[NTGT];  // prefix counted by each histogram
    int32_t nslots;
};

// On entry sm.rank[t] (t < ntgt) holds the ascending rank wanted; on return
// sm.pref[t] is the key of that order statistic.  Targets whose prefixes
// agree share a histogram; prefixes of one pass have equal length, so each
// element feeds at most one histogram.  get(j) returns the key of element j
// of [0, count).  Called by every thread of the block.
template <class Get>
__device__ void radix_select(SelShared &sm, int64_t count, int ntgt, Get get) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    if (tid < ntgt) {
        sm.pref[tid] = 0;
        sm.slot[tid] = 0;
    }
    if (tid == 0) {
        sm.nslots = 1;
        sm.slot_pref[0] = 0;
    }
    __syncthreads();
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        const int ns = sm.nslots;
        for (int e = tid; e < ns * 256; e += blockDim.x) (&sm.hist[0][0])[e] = 0u;
        __syncthreads();
        for (int64_t j = tid; j < count; j += blockDim.x) {
            const uint32_t key = get(j);
            int s = 0;
            if (pass > 0) {
                const uint32_t hi = key >> (shift + 8);
                s = -1;
                for (int q = 0; q < ns; ++q)
                    if (sm.slot_pref[q] == hi) s = q;
            }
            if (s >= 0) atomicAdd(&sm.hist[s][(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        for (int t = wave; t < ntgt; t += nwaves) {
            const uint32_t *h = sm.hist[sm.slot[t]];
            uint32_t c[4], tot = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = h[4 * lane + q];
                tot += c[q];
            }
            uint32_t inc = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t o = __shfl_up(inc, off, 64);
                if (lane >= off) inc += o;
            }
            const uint32_t before = inc - tot;
            const uint32_t r = (uint32_t)sm.rank[t];
            if (r >= before && r < inc) {
                uint32_t acc = before;
                int d = 0;
                while (d < 3 && r >= acc + c[d]) acc += c[d++];
                sm.pref[t] = (sm.pref[t] << 8) | (uint32_t)(4 * lane + d);
                sm.rank[t] = (int32_t)(r - acc);
            }
        }
        __syncthreads();
        if (tid == 0) {
            int n2 = 0;
            for (int t = 0; t < ntgt; ++t) {
                int s = -1;
                for (int q = 0; q < n2; ++q)
                    if (sm.slot_pref[q] == sm.pref[t]) s = q;
                if (s < 0) {
                    s = n2++;
                    sm.slot_pref[s] = sm.pref[t];
                }
                sm.slot[t] = s;
            }
            sm.nslots = n2;
        }
        __syncthreads();
    }
}

// Per-row statistics (64 bytes).
struct RowStats {
    float v[NTGT];      // 1st, 2nd, 4th, 8th, 16th, 32nd largest; quantiles 1, 10, 25, 50, 75 %
    float diag;         // s(k,k)
    int32_t above;      // #{j != k : s(k,j) > s(k,k)}
    int32_t pad;
    double top_sum;     // sum of the min(32, n-1) largest
};
static_assert(sizeof(RowStats) == 64, "RowStats layout");
constexpr int Q50 = 9;  // index of the median in RowStats::v

__constant__ int kDesc[6] = {0, 1, 3, 7, 15, 31};
__constant__ int kQuant[5] = {1, 10, 25, 50, 75};

__global__ __launch_bounds__(SEL_T) void k_row_stats(const float *S, int64_t ld, int32_t n,
                                                     RowStats *out) {
    __shared__ SelShared sm;
    __shared__ double wsum[SEL_T / 64];
    __shared__ int32_t wcnt[SEL_T / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t m = n - 1;
    for (int64_t k = blockIdx.x; k < n; k += gridDim.x) {
        const float *row = S + k * ld;
        if (tid < NTGT) {
            int64_t r;
            if (tid < 6) {
                const int64_t j = kDesc[tid];
                r = m - 1 - (j < m - 1 ? j : m - 1);
            } else {
                r = ((int64_t)kQuant[tid - 6] * (m - 1)) / 100;
            }
            sm.rank[tid] = (int32_t)r;
        }
        radix_select(sm, m, NTGT, [&](int64_t j) { return fkey(row[j < k ? j : j + 1]); });
        // Elements above the 32nd largest, and elements above the diagonal.
        const uint32_t key32 = sm.pref[5];
        const float dg = row[k];
        double s = 0.0;
        int32_t gt = 0, above = 0;
        for (int64_t j = tid; j < m; j += blockDim.x) {
            const float v = row[j < k ? j : j + 1];
            if (fkey(v) > key32) {
                s += (double)v;
                ++gt;
            }
            above += (v > dg) ? 1 : 0;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            s += __shfl_down(s, off, 64);
            gt += __shfl_down(gt, off, 64);
            above += __shfl_down(above, off, 64);
        }
        if (lane == 0) {
            wsum[wave] = s;
            wcnt[wave][0] = gt;
            wcnt[wave][1] = above;
        }
        __syncthreads();
        if (tid == 0) {
            double tot = 0.0;
            int32_t g = 0, a = 0;
            for (int w = 0; w < SEL_T / 64; ++w) {
                tot += wsum[w];
                g += wcnt[w][0];
                a += wcnt[w][1];
            }
            const int32_t cnt = m < TOP ? (int32_t)m : TOP;
            RowStats r;
            for (int t = 0; t < NTGT; ++t) r.v[t] = keyf(sm.pref[t]);
            r.diag = dg;
            r.above = a;
            r.pad = 0;
            r.top_sum = tot + (double)(cnt - g) * (double)keyf(key32);
            out[k] = r;
        }
        __syncthreads();
    }
}

// sigma = |lower median of the row medians| (1 if that is 0 or not finite).
__global__ __launch_bounds__(SEL_T) void k_sigma(const RowStats *st, int32_t n, float *sigma) {
    __shared__ SelShared sm;
    if (threadIdx.x == 0) sm.rank[0] = (n - 1) / 2;
    radix_select(sm, n, 1, [&](int64_t j) { return fkey(st[j].v[Q50]); });
    if (threadIdx.x == 0) {
        float s = fabsf(keyf(sm.pref[0]));
        if (!(s > 0.0f) || !(s < INFINITY)) s = 1.0f;
        *sigma = s;
    }
}

__global__ void k_features(const RowStats *st, int32_t n, const float *sigma, float ln_n_10, float *F) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const RowStats r = st[k];
    const double sg = (double)*sigma;
    const int64_t m = n - 1;
    const double tm = r.top_sum / (double)(m < TOP ? m : TOP);
    float f[NF];
    for (int t = 0; t < 6; ++t) f[t] = (float)((double)r.v[t] / sg);
    f[6] = (float)(tm / sg);
    for (int q = 0; q < 5; ++q) f[7 + q] = (float)((double)r.v[6 + q] / sg);
    f[12] = (float)(((double)r.diag - (double)r.v[Q50]) / sg);
    f[13] = (float)(((double)r.diag - tm) / sg);
    f[14] = (float)((double)r.above / (double)m);
    f[15] = ln_n_10;
    float4 *o = reinterpret_cast<float4 *>(F + k * NF);
    for (int q = 0; q < 4; ++q) o[q] = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// Network
// ---------------------------------------------------------------------------
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// gfx950's 32x32x16 bf16 matrix op (FP32 accumulate): lane l holds row (or
// column) l mod 32 and k = 8 (l / 32) .. + 7 of its operand.  The two halves
// of an operand come from 8-byte aligned LDS rows (their padding keeps the
// 8-byte loads free of bank conflicts).
__device__ __forceinline__ v16f mfma16(v4s a0, v4s a1, v4s b0, v4s b1, v16f c) {
    const v8s a = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
    const v8s b = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

__device__ __forceinline__ v16f zero16() {
    v16f z;
#pragma unroll
    for (int q = 0; q < 16; ++q) z[q] = 0.0f;
    return z;
}

// Round to bfloat16, nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t bf16_bits(float x) {
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x40u);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// GELU z Phi(z) and its derivative Phi(z) + z phi(z).
__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * expf(-0.5f * z * z);
}

constexpr int FW_T = 256;           // 4 waves
constexpr int FW_P = 128;           // points per block, 32 per wave
constexpr int LW1 = NF + 4;         // padded row of W1^T in LDS (bf16)
constexpr int LW2 = NH + 4;         // padded row of W2^T and of the activations

struct FwdShared {
    uint16_t w1t[NH * LW1];         // W1^T [unit][feature]
    uint16_t w2t[NH * LW2];         // W2^T [unit out][unit in]
    uint16_t h[FW_P * LW2];         // activations [point][unit]
    float w3[NH * NO];              // bf16-rounded W3 [unit][output]
    float b1[NH], b2[NH], b3[4];
};

struct FwdArgs {
    const float *theta;             // FP32 master parameters
    const float *F;                 // features, count x 16
    const int64_t *rows;            // nullable: point p of the batch is rows[p]
    int64_t count;
    float *Y;                       // count x 2
    float *Z1, *Z2;                 // nullable stash: pre-activations, count x 128
    uint16_t *H1, *H2;              // stash: bf16 activations, count x 128
};

// Bias, GELU and bf16 rounding of one 32 x 128 layer output held in MFMA
// accumulators; lane l holds column (l % 32) of each 32 x 32 tile and rows
// 8 (v / 4) + 4 (l / 32) + v % 4 for v < 16.
template <bool STASH>
__device__ __forceinline__ void layer_epilogue(const v16f (&acc)[4], const float *bias, uint16_t *hw,
                                               float *Z, uint16_t *H, int64_t p0, int64_t count,
                                               int lane) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int j = 32 * nt + (lane & 31);
        const float bj = bias[j];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const float z = acc[nt][v] + bj;
            const uint16_t hb = bf16_bits(gelu(z));
            hw[r * LW2 + j] = hb;
            if (STASH && p0 + r < count) {
                Z[(p0 + r) * NH + j] = z;
                H[(p0 + r) * NH + j] = hb;
            }
        }
    }
}

template <bool STASH>
__global__ __launch_bounds__(FW_T) void k_mlp_fwd(FwdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    FwdShared &sh = *reinterpret_cast<FwdShared *>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < NF * NH; e += FW_T)
        sh.w1t[(e % NH) * LW1 + e / NH] = bf16_bits(a.theta[OFF_W1 + e]);
    for (int e = tid; e < NH * NH; e += FW_T)
        sh.w2t[(e % NH) * LW2 + e / NH] = bf16_bits(a.theta[OFF_W2 + e]);
    for (int e = tid; e < NH * NO; e += FW_T) sh.w3[e] = bf16_val(bf16_bits(a.theta[OFF_W3 + e]));
    for (int e = tid; e < NH; e += FW_T) {
        sh.b1[e] = a.theta[OFF_B1 + e];
        sh.b2[e] = a.theta[OFF_B2 + e];
    }
    if (tid < NO) sh.b3[tid] = a.theta[OFF_B3 + tid];
    __syncthreads();

    const int64_t p0 = (int64_t)blockIdx.x * FW_P + wave * 32;
    const int li = lane & 31, lk = (lane >> 5) * 8;
    uint16_t *hw = sh.h + (wave * 32) * LW2;

    // Layer 1 (K = 16, one matrix op per 32 units): A operand = bf16
    // features of point p0 + li, k = lk .. lk + 7.
    v4s xa[2];
    {
        const int64_t p = p0 + li;
        const int64_t src = p < a.count ? (a.rows ? a.rows[p] : p) : -1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float4 f = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (src >= 0) f = *reinterpret_cast<const float4 *>(a.F + src * NF + lk + 4 * h);
            xa[h] = v4s{(short)bf16_bits(f.x), (short)bf16_bits(f.y), (short)bf16_bits(f.z),
                        (short)bf16_bits(f.w)};
        }
    }
    v16f acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const uint16_t *w = sh.w1t + (32 * nt + li) * LW1 + lk;
        acc[nt] = mfma16(xa[0], xa[1], *reinterpret_cast<const v4s *>(w), *reinterpret_cast<const v4s *>(w + 4),
                         zero16());
    }
    layer_epilogue<STASH>(acc, sh.b1, hw, a.Z1, a.H1, p0, a.count, lane);
    __syncthreads();

    // Layer 2: 32 points x 128 units, K = 128 in 8 steps of 16.
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = zero16();
#pragma unroll 4
    for (int ks = 0; ks < 8; ++ks) {
        const uint16_t *hr = hw + li * LW2 + 16 * ks + lk;
        const v4s a0 = *reinterpret_cast<const v4s *>(hr), a1 = *reinterpret_cast<const v4s *>(hr + 4);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const uint16_t *w = sh.w2t + (32 * nt + li) * LW2 + 16 * ks + lk;
            acc[nt] = mfma16(a0, a1, *reinterpret_cast<const v4s *>(w), *reinterpret_cast<const v4s *>(w + 4),
                             acc[nt]);
        }
    }
    __syncthreads();
    layer_epilogue<STASH>(acc, sh.b2, hw, a.Z2, a.H2, p0, a.count, lane);
    __syncthreads();

    // Layer 3 (128 -> 2) on the vector units: lane -> (point li, output lane / 32).
    {
        const int o = lane >> 5;
        float y = 0.0f;
        const uint16_t *hr = hw + li * LW2;
        for (int j = 0; j < NH; ++j) y = fmaf(bf16_val(hr[j]), sh.w3[j * NO + o], y);
        y += sh.b3[o];
        if (p0 + li < a.count) a.Y[(p0 + li) * NO + o] = y;
    }
}

// Backward of one block of BW_P points; writes this block's partial gradient.
constexpr int BW_T = 256;
constexpr int BW_P = 64;

struct BwdShared {
    float dz2[BW_P][NH + 1];        // gradient at the second pre-activation
    uint16_t h1[BW_P][NH + 2];      // bf16 first activations
    uint16_t w2[NH][NH + 2];        // bf16 W2 [in][out]
    float x[BW_P][NF + 1];          // bf16-rounded features
    float dw1[NH][NF + 1];          // second half of the dW1 partial
    float db1[NH];
    float dy[BW_P][NO];
    float w3[NH][NO];
    double red[BW_T / 64];
};

struct BwdArgs {
    const float *theta;
    const float *F, *T, *w;         // features (count x 16), targets (count x 2), weights (count)
    const int64_t *rows;            // nullable batch indices into F, T, w
    int64_t count;
    const float *Y, *Z1, *Z2;       // from the stashing forward pass
    const uint16_t *H1, *H2;
    float *gpart;                   // [gridDim.x][NPARAM]
    double *lpart;                  // [gridDim.x]
};

__global__ __launch_bounds__(BW_T) void k_mlp_bwd(BwdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    BwdShared &sh = *reinterpret_cast<BwdShared *>(smem);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p0 = (int64_t)blockIdx.x * BW_P;
    float *g = a.gpart + (int64_t)blockIdx.x * NPARAM;

    for (int e = tid; e < NH * NH; e += BW_T) sh.w2[e / NH][e % NH] = bf16_bits(a.theta[OFF_W2 + e]);
    for (int e = tid; e < NH * NO; e += BW_T) sh.w3[e / NO][e % NO] = bf16_val(bf16_bits(a.theta[OFF_W3 + e]));
    for (int e = tid; e < BW_P * NF; e += BW_T) {
        const int p = e / NF, f = e % NF;
        float v = 0.0f;
        if (p0 + p < a.count) {
            const int64_t src = a.rows ? a.rows[p0 + p] : p0 + p;
            v = bf16_val(bf16_bits(a.F[src * NF + f]));
        }
        sh.x[p][f] = v;
    }
    for (int e = tid; e < BW_P * NH; e += BW_T) {
        const int p = e / NH, j = e % NH;
        sh.h1[p][j] = p0 + p < a.count ? a.H1[(p0 + p) * NH + j] : (uint16_t)0;
    }
    // Loss and its gradient at the outputs: w_p * Huber(y - t), delta 1.
    double lsum = 0.0;
    if (tid < BW_P * NO) {
        const int p = tid / NO, o = tid % NO;
        float d = 0.0f;
        if (p0 + p < a.count) {
            const int64_t src = a.rows ? a.rows[p0 + p] : p0 + p;
            const float e = a.Y[(p0 + p) * NO + o] - a.T[src * NO + o];
            const float wp = a.w[src];
            d = wp * fminf(1.0f, fmaxf(-1.0f, e));
            const double ae = fabs((double)e);
            lsum = (double)wp * (ae <= 1.0 ? 0.5 * (double)e * (double)e : ae - 0.5);
        }
        sh.dy[p][o] = d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    if (lane == 0) sh.red[wave] = lsum;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < BW_T / 64; ++w) t += sh.red[w];
        a.lpart[blockIdx.x] = t;
    }

    // Output layer: dW3[j][o] = sum_p h2[p][j] dy[p][o]; db3.
    {
        const int j = tid >> 1, o = tid & 1;
        float acc = 0.0f;
        for (int p = 0; p < BW_P && p0 + p < a.count; ++p)
            acc = fmaf(bf16_val(a.H2[(p0 + p) * NH + j]), sh.dy[p][o], acc);
        g[OFF_W3 + j * NO + o] = acc;
        if (tid < NO) {
            float b = 0.0f;
            for (int p = 0; p < BW_P; ++p) b += sh.dy[p][tid];
            g[OFF_B3 + tid] = b;
        }
    }
    // dz2 = (W3 dy) * GELU'(z2)
    for (int e = tid; e < BW_P * NH; e += BW_T) {
        const int p = e / NH, j = e % NH;
        float v = 0.0f;
        if (p0 + p < a.count) {
            const float dh = fmaf(sh.w3[j][0], sh.dy[p][0], sh.w3[j][1] * sh.dy[p][1]);
            v = dh * gelu_grad(a.Z2[(p0 + p) * NH + j]);
        }
        sh.dz2[p][j] = v;
    }
    __syncthreads();

    // dW2[i][j] = sum_p h1[p][i] dz2[p][j]; thread -> column j, 64 rows i.
    {
        const int j = tid & (NH - 1), i0 = (tid >> 7) * 64;
        float acc[64];
#pragma unroll
        for (int q = 0; q < 64; ++q) acc[q] = 0.0f;
        for (int p = 0; p < BW_P; ++p) {
            const float dz = sh.dz2[p][j];
#pragma unroll
            for (int q = 0; q < 64; ++q) acc[q] = fmaf(bf16_val(sh.h1[p][i0 + q]), dz, acc[q]);
        }
#pragma unroll
        for (int q = 0; q < 64; ++q) g[OFF_W2 + (i0 + q) * NH + j] = acc[q];
        if (tid < NH) {
            float b = 0.0f;
            for (int p = 0; p < BW_P; ++p) b += sh.dz2[p][tid];
            g[OFF_B2 + tid] = b;
        }
    }

    // dz1 = (W2 dz2) * GELU'(z1); dW1[f][i] = sum_p x[p][f] dz1[p][i]; db1.
    // Thread -> unit i and one half of the points; halves added in order.
    {
        const int i = tid & (NH - 1), half = tid >> 7;
        float dw[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) dw[f] = 0.0f;
        float db = 0.0f;
        for (int p = half * (BW_P / 2); p < (half + 1) * (BW_P / 2); ++p) {
            if (p0 + p >= a.count) break;
            float dh = 0.0f;
            for (int j = 0; j < NH; ++j) dh = fmaf(bf16_val(sh.w2[i][j]), sh.dz2[p][j], dh);
            const float dz = dh * gelu_grad(a.Z1[(p0 + p) * NH + i]);
            db += dz;
#pragma unroll
            for (int f = 0; f < NF; ++f) dw[f] = fmaf(sh.x[p][f], dz, dw[f]);
        }
        if (half == 1) {
#pragma unroll
            for (int f = 0; f < NF; ++f) sh.dw1[i][f] = dw[f];
            sh.db1[i] = db;
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int f = 0; f < NF; ++f) g[OFF_W1 + f * NH + i] = dw[f] + sh.dw1[i][f];
            g[OFF_B1 + i] = db + sh.db1[i];
        }
    }
}

// grad[e] = sum over blocks of the partials, in block order (FP64).
__global__ void k_mlp_reduce(const float *gpart, const double *lpart, int32_t nblk, float *grad,
                             double *loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < NPARAM) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += (double)gpart[(int64_t)b * NPARAM + e];
        grad[e] = (float)s;
    }
    if (loss && e == 0) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += lpart[b];
        *loss = s;
    }
}

// Adam (Kingma and Ba, 2015) with bias correction factors c1 = 1/(1-beta1^t),
// c2 = 1/(1-beta2^t).
__global__ void k_adam(float *theta, float *m, float *v, const float *g, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    theta[e] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ---------------------------------------------------------------------------
// Targets and A_0
// ---------------------------------------------------------------------------
// 64 columns x 16 row slices per block; slices combined in order (FP64).
__global__ __launch_bounds__(1024) void k_targets(const float *R, int64_t ld, int32_t n,
                                                  const float *sigma, float *Y) {
    __shared__ double part[16][64];
    const int c = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int64_t k = (int64_t)blockIdx.x * 64 + c;
    double s = 0.0;
    if (k < n)
        for (int64_t i = sl; i < n; i += 16)
            if (i != k) s += (double)fmaxf(0.0f, R[i * ld + k]);
    part[sl][c] = s;
    __syncthreads();
    if (sl == 0 && k < n) {
        double cs = 0.0;
        for (int q = 0; q < 16; ++q) cs += part[q][c];
        const double sg = (double)*sigma;
        Y[k * NO + 0] = (float)(((double)R[k * ld + k] + cs) / sg);
        Y[k * NO + 1] = (float)(cs / sg);
    }
}

__device__ __forceinline__ float a0_value(const float *Y, float sg, int64_t i, int64_t k) {
    return k == i ? fmaxf(0.0f, sg * Y[i * NO + 1]) : fminf(0.0f, sg * Y[k * NO]);
}

__global__ void k_warm_a0(const float *Y, const float *sigma, int32_t n, float *A, int64_t ld) {
    const float sg = *sigma;
    const int64_t n4 = n & ~3;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        float *row = A + i * ld;
        for (int64_t k = 4 * threadIdx.x; k < n4; k += 4 * blockDim.x) {
            const float4 o = make_float4(a0_value(Y, sg, i, k), a0_value(Y, sg, i, k + 1),
                                         a0_value(Y, sg, i, k + 2), a0_value(Y, sg, i, k + 3));
            *reinterpret_cast<float4 *>(row + k) = o;
        }
        for (int64_t k = n4 + threadIdx.x; k < n; k += blockDim.x) row[k] = a0_value(Y, sg, i, k);
    }
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

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

apx_status check_sq(apx_ctx *ctx, const float *M, const char *name, int64_t n, int64_t ld) {
    if (M == nullptr) return set_err(ctx, APX_EINVAL, "%s is null", name);
    if (!aligned16(M)) return set_err(ctx, APX_EINVAL, "%s is not 16-byte aligned", name);
    if (ld < n || ld % 4 != 0) return set_err(ctx, APX_EINVAL, "%s: need ld >= n and ld %% 4 == 0", name);
    return APX_OK;
}

unsigned grid_rows(int64_t n, int num_cus) {
    const int64_t g = (int64_t)num_cus * 2;
    return (unsigned)(n < g ? n : g);
}

// Features into F using `stats` (n RowStats) and `sigma` (device float).
apx_status run_features(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, RowStats *stats,
                        float *F, float *sigma) {
    hipStream_t s = ctx->stream;
    k_row_stats<<<grid_rows(n, ctx->num_cus), SEL_T, 0, s>>>(S, ld, (int32_t)n, stats);
    HIP_TRY(hipGetLastError(), "row statistics");
    k_sigma<<<1, SEL_T, 0, s>>>(stats, (int32_t)n, sigma);
    HIP_TRY(hipGetLastError(), "sigma");
    const float ln10 = (float)(std::log((double)n) / 10.0);
    k_features<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(stats, (int32_t)n, sigma, ln10, F);
    HIP_TRY(hipGetLastError(), "features");
    return APX_OK;
}

apx_status run_forward(apx_ctx *ctx, const FwdArgs &fa, bool stash) {
    const size_t lds = sizeof(FwdShared);
    const unsigned grid = (unsigned)((fa.count + FW_P - 1) / FW_P);
    if (stash) {
        HIP_TRY(hipFuncSetAttribute((const void *)k_mlp_fwd<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds), "lds");
        k_mlp_fwd<true><<<grid, FW_T, lds, ctx->stream>>>(fa);
    } else {
        HIP_TRY(hipFuncSetAttribute((const void *)k_mlp_fwd<false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds), "lds");
        k_mlp_fwd<false><<<grid, FW_T, lds, ctx->stream>>>(fa);
    }
    HIP_TRY(hipGetLastError(), "network forward");
    return APX_OK;
}

int64_t round64(int64_t v) { return (v + 63) & ~int64_t(63); }

struct BwdLayout {
    size_t o_y, o_z1, o_z2, o_h1, o_h2, o_gp, o_lp, bytes;
};
BwdLayout bwd_layout(int64_t count) {
    const int64_t nblk = (count + BW_P - 1) / BW_P;
    WsLayout W;
    BwdLayout o{};
    o.o_y = W.take(sizeof(float) * NO * (size_t)count);
    o.o_z1 = W.take(sizeof(float) * NH * (size_t)count);
    o.o_z2 = W.take(sizeof(float) * NH * (size_t)count);
    o.o_h1 = W.take(sizeof(uint16_t) * NH * (size_t)count);
    o.o_h2 = W.take(sizeof(uint16_t) * NH * (size_t)count);
    o.o_gp = W.take(sizeof(float) * NPARAM * (size_t)nblk);
    o.o_lp = W.take(sizeof(double) * (size_t)nblk);
    o.bytes = W.off;
    return o;
}

struct WarmLayout {
    size_t o_st, o_f, o_y, o_s, head;
};
WarmLayout warm_layout(int64_t n) {
    WsLayout W;
    WarmLayout o{};
    o.o_st = W.take(sizeof(RowStats) * (size_t)n);
    o.o_f = W.take(sizeof(float) * NF * (size_t)n);
    o.o_y = W.take(sizeof(float) * NO * (size_t)n);
    o.o_s = W.take(sizeof(float) * 4);
    o.head = W.off;
    return o;
}

}  // namespace

namespace apx {
size_t features_ws_bytes(int64_t n) {
    WsLayout W;
    W.take(sizeof(RowStats) * (size_t)n);
    return W.off;
}
size_t mlp_backward_ws_bytes(int64_t count) { return bwd_layout(count).bytes; }
size_t warmstart_ws_bytes(int64_t n, int64_t ld, int num_cus) {
    return warm_layout(n).head + resp_step_ws_bytes(n, ld, num_cus);
}
}  // namespace apx

extern "C" {

apx_status apx_features(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, float *F, float *sigma) {
    if (!ctx) return APX_EINVAL;
    if (n < 2) return set_err(ctx, APX_EINVAL, "apx_features needs n >= 2");
    if (n > 65536) return set_err(ctx, APX_ENOTIMPL, "n = %lld exceeds 65536", (long long)n);
    APX_TRY(check_sq(ctx, S, "S", n, ld));
    if (!F || !aligned16(F) || !sigma) return set_err(ctx, APX_EINVAL, "F (16-byte aligned) and sigma are required");
    DevGuard g(ctx->device);
    WsLayout W;
    const size_t o_st = W.take(sizeof(RowStats) * (size_t)n);
    APX_TRY(ws_reserve(ctx, ctx->ws_base + W.off));
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;
    return run_features(ctx, S, n, ld, reinterpret_cast<RowStats *>(b + o_st), F, sigma);
}

apx_status apx_mlp_forward(apx_ctx *ctx, const float *theta, const float *F, int64_t count, float *Y) {
    if (!ctx) return APX_EINVAL;
    if (!theta || !F || !Y || !aligned16(F)) return set_err(ctx, APX_EINVAL, "null or misaligned argument");
    if (count < 0) return set_err(ctx, APX_EINVAL, "count < 0");
    if (count == 0) return APX_OK;
    DevGuard g(ctx->device);
    FwdArgs fa{};
    fa.theta = theta;
    fa.F = F;
    fa.count = count;
    fa.Y = Y;
    return run_forward(ctx, fa, false);
}

apx_status apx_mlp_backward(apx_ctx *ctx, const float *theta, const float *F, const float *T,
                            const float *w, const int64_t *rows, int64_t count, float *grad,
                            double *loss) {
    if (!ctx) return APX_EINVAL;
    if (!theta || !F || !T || !w || !grad || !aligned16(F))
        return set_err(ctx, APX_EINVAL, "null or misaligned argument");
    if (count < 1) return set_err(ctx, APX_EINVAL, "count must be >= 1");
    DevGuard g(ctx->device);
    const int64_t nblk = (count + BW_P - 1) / BW_P;
    const BwdLayout BL = bwd_layout(count);
    const size_t o_y = BL.o_y, o_z1 = BL.o_z1, o_z2 = BL.o_z2, o_h1 = BL.o_h1, o_h2 = BL.o_h2, o_gp = BL.o_gp,
                 o_lp = BL.o_lp;
    APX_TRY(ws_reserve(ctx, ctx->ws_base + BL.bytes));
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;
    FwdArgs fa{};
    fa.theta = theta;
    fa.F = F;
    fa.rows = rows;
    fa.count = count;
    fa.Y = reinterpret_cast<float *>(b + o_y);
    fa.Z1 = reinterpret_cast<float *>(b + o_z1);
    fa.Z2 = reinterpret_cast<float *>(b + o_z2);
    fa.H1 = reinterpret_cast<uint16_t *>(b + o_h1);
    fa.H2 = reinterpret_cast<uint16_t *>(b + o_h2);
    APX_TRY(run_forward(ctx, fa, true));
    BwdArgs ba{};
    ba.theta = theta;
    ba.F = F;
    ba.T = T;
    ba.w = w;
    ba.rows = rows;
    ba.count = count;
    ba.Y = fa.Y;
    ba.Z1 = fa.Z1;
    ba.Z2 = fa.Z2;
    ba.H1 = fa.H1;
    ba.H2 = fa.H2;
    ba.gpart = reinterpret_cast<float *>(b + o_gp);
    ba.lpart = reinterpret_cast<double *>(b + o_lp);
    const size_t lds = sizeof(BwdShared);
    HIP_TRY(hipFuncSetAttribute((const void *)k_mlp_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds), "lds");
    k_mlp_bwd<<<(unsigned)nblk, BW_T, lds, ctx->stream>>>(ba);
    HIP_TRY(hipGetLastError(), "network backward");
    k_mlp_reduce<<<(NPARAM + 255) / 256, 256, 0, ctx->stream>>>(ba.gpart, ba.lpart, (int32_t)nblk, grad, loss);
    HIP_TRY(hipGetLastError(), "gradient reduce");
    return APX_OK;
}

apx_status apx_mlp_adam(apx_ctx *ctx, float *theta, float *m, float *v, const float *grad,
                        int64_t count, int32_t step, float lr, float beta1, float beta2, float eps) {
    if (!ctx) return APX_EINVAL;
    if (!theta || !m || !v || !grad) return set_err(ctx, APX_EINVAL, "null argument");
    if (count < 0 || step < 1) return set_err(ctx, APX_EINVAL, "need count >= 0 and step >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return set_err(ctx, APX_EINVAL, "need 0 <= beta < 1 and eps > 0");
    if (count == 0) return APX_OK;
    DevGuard g(ctx->device);
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    k_adam<<<(unsigned)((count + 255) / 256), 256, 0, ctx->stream>>>(theta, m, v, grad, count, lr, beta1,
                                                                    beta2, eps, c1, c2);
    HIP_TRY(hipGetLastError(), "adam");
    return APX_OK;
}

apx_status apx_targets(apx_ctx *ctx, const float *R, int64_t n, int64_t ld, const float *sigma, float *Y) {
    if (!ctx) return APX_EINVAL;
    if (n < 1) return set_err(ctx, APX_EINVAL, "n must be >= 1");
    APX_TRY(check_sq(ctx, R, "R", n, ld));
    if (!sigma || !Y) return set_err(ctx, APX_EINVAL, "null argument");
    DevGuard g(ctx->device);
    k_targets<<<(unsigned)((n + 63) / 64), 1024, 0, ctx->stream>>>(R, ld, (int32_t)n, sigma, Y);
    HIP_TRY(hipGetLastError(), "targets");
    return APX_OK;
}

apx_status apx_warm_a0(apx_ctx *ctx, const float *Y, const float *sigma, int64_t n, float *A, int64_t ld) {
    if (!ctx) return APX_EINVAL;
    if (n < 1) return set_err(ctx, APX_EINVAL, "n must be >= 1");
    APX_TRY(check_sq(ctx, A, "A", n, ld));
    if (!sigma || !Y) return set_err(ctx, APX_EINVAL, "null argument");
    DevGuard g(ctx->device);
    k_warm_a0<<<grid_rows(n, ctx->num_cus * 4), 256, 0, ctx->stream>>>(Y, sigma, (int32_t)n, A, ld);
    HIP_TRY(hipGetLastError(), "A_0");
    return APX_OK;
}

apx_status ap_warmstart(apx_ctx *ctx, const float *S, int64_t n, int64_t ld, const float *theta,
                        float *R, float *A, float *sigma) {
    if (!ctx) return APX_EINVAL;
    if (n < 2) return set_err(ctx, APX_EINVAL, "ap_warmstart needs n >= 2");
    if (n > 65536) return set_err(ctx, APX_ENOTIMPL, "n = %lld exceeds 65536", (long long)n);
    APX_TRY(check_sq(ctx, S, "S", n, ld));
    APX_TRY(check_sq(ctx, R, "R", n, ld));
    APX_TRY(check_sq(ctx, A, "A", n, ld));
    if (!theta) return set_err(ctx, APX_EINVAL, "theta is null");
    DevGuard g(ctx->device);
    const WarmLayout WL = warm_layout(n);
    const size_t o_st = WL.o_st, o_f = WL.o_f, o_y = WL.o_y, o_s = WL.o_s, head = WL.head;
    const size_t base = ctx->ws_base;
    APX_TRY(ws_reserve(ctx, base + head + resp_step_ws_bytes(n, ld, ctx->num_cus)));
    char *b = static_cast<char *>(ctx->ws) + base;
    RowStats *stats = reinterpret_cast<RowStats *>(b + o_st);
    float *F = reinterpret_cast<float *>(b + o_f);
    float *Yp = reinterpret_cast<float *>(b + o_y);
    float *sg = sigma ? sigma : reinterpret_cast<float *>(b + o_s);
    APX_TRY(run_features(ctx, S, n, ld, stats, F, sg));
    FwdArgs fa{};
    fa.theta = theta;
    fa.F = F;
    fa.count = n;
    fa.Y = Yp;
    APX_TRY(run_forward(ctx, fa, false));
    k_warm_a0<<<grid_rows(n, ctx->num_cus * 4), 256, 0, ctx->stream>>>(Yp, sg, (int32_t)n, A, ld);
    HIP_TRY(hipGetLastError(), "A_0");
    // R_0 = one undamped responsibility step (Eq. (2)) from A_0.
    ctx->ws_base = base + head;
    const apx_status st = resp_step(ctx, S, n, ld, R, A);
    ctx->ws_base = base;
    return st;
}

}  // extern "C"
