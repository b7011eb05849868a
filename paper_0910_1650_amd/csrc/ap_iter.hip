// ap_iter.hip -- the dense affinity-propagation iteration on gfx950.
//
// One iteration of Algorithm 1 (Section 2) is two launches:
//
//   row pass   (one workgroup streams whole rows; every element of S, R, A is
//               touched once): availabilities A_t by Eqs. (3)/(4) with
//               damping, the exemplar decision argmax_k a(i,k)+r(i,k), the
//               top-2 of a(i,k)+s(i,k), then R_{t+1} by Eq. (2) with damping,
//               and per-workgroup column partials of max(0, r_{t+1}(i,k)).
//   col reduce (sums the partials in FP64 in a fixed order into the column
//               vectors c_k and t_k = r(k,k) + c_k; applies the stop rule).
//
// Each thread owns the same columns in every row (float4 chunks strided by
// the workgroup size), so the row values needed after the top-2 reduction
// (u = lambda*r + (1-lambda)*s) and the column partials stay in registers;
// HBM traffic per element and iteration is read S, R, A and write A, R.
#include "apx_internal.h"

#include <cfloat>

namespace apx {
namespace {

constexpr float kNegInf = -INFINITY;

struct Top2 {
    float v1;   // largest a+s
    int k1;     // its column (lowest on ties)
    float v2;   // largest over the other columns
};

struct ArgMax {
    float v;
    int k;
};

__device__ __forceinline__ void top2_push(Top2 &t, float v, int k) {
    // columns arrive in ascending order within a thread: a tie keeps k1
    if (v > t.v1) {
        t.v2 = t.v1;
        t.v1 = v;
        t.k1 = k;
    } else {
        t.v2 = fmaxf(t.v2, v);
    }
}

__device__ __forceinline__ void top2_merge(Top2 &t, float ov1, int ok1, float ov2) {
    bool take = (ov1 > t.v1) || (ov1 == t.v1 && ok1 < t.k1);
    float nv2 = take ? fmaxf(ov2, t.v1) : fmaxf(t.v2, ov1);
    if (take) {
        t.v1 = ov1;
        t.k1 = ok1;
    }
    t.v2 = nv2;
}

__device__ __forceinline__ void argmax_merge(ArgMax &m, float ov, int ok) {
    if (ov > m.v || (ov == m.v && ok < m.k)) {
        m.v = ov;
        m.k = ok;
    }
}

__device__ __forceinline__ float f4get(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
__device__ __forceinline__ void f4set(float4 &v, int e, float x) {
    if (e == 0) v.x = x;
    else if (e == 1) v.y = x;
    else if (e == 2) v.z = x;
    else v.w = x;
}

// Availability update of one element (Eqs. (3), (4), damping).
__device__ __forceinline__ float avail(float a, float r, float t, float ci, bool diag, float lam,
                                       float oml) {
#pragma clang fp contract(off)
    float upd = diag ? ci : fminf(0.0f, t - fmaxf(0.0f, r));
    return lam * a + oml * upd;
}

template <int T, int J, int MODE>
__global__ __launch_bounds__(T) void k_row_pass(PassArgs p) {
    // Every product is rounded before it is added: with u = lambda*r +
    // (1-lambda)*s and the subtraction of (1-lambda)*max below, an exact tie
    // s(i,k) = max then cancels to exactly zero, as in Eq. (2).
#pragma clang fp contract(off)
    if (p.st != nullptr && p.st->frozen) return;
    constexpr int NW = T / 64;
    __shared__ float sh_f[2][NW][3];
    __shared__ int sh_i[2][NW][2];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n = p.n;
    const int64_t ld = p.ld;
    const float lam = p.lam;
    const float oml = 1.0f - lam;
    const int64_t nrows = p.row_end - p.row_begin;
    const int64_t r0 = p.row_begin + (int64_t)blockIdx.x * nrows / gridDim.x;
    const int64_t r1 = p.row_begin + (int64_t)(blockIdx.x + 1) * nrows / gridDim.x;

    float4 part[J];
    float4 tv[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        part[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int c = (j * T + tid) * 4;
        if (MODE != PASS_R_ONLY && c < n) tv[j] = *reinterpret_cast<const float4 *>(p.tcol + c);
        else tv[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    int my_nex = 0, my_changed = 0;

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const float *Srow = p.S + i * ld;
        const float *Rin = p.Rin + i * ld;
        float *Rout = p.Rout + i * ld;
        float *Arow = p.A + i * ld;
        const float ci = (MODE != PASS_R_ONLY) ? p.ccol[ii] : 0.0f;

        float4 u[J];
        Top2 t2{kNegInf, n, kNegInf};
        ArgMax dm{kNegInf, n};
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = (j * T + tid) * 4;
            u[j] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (c < n) {
                float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (MODE != PASS_A_ONLY) s4 = *reinterpret_cast<const float4 *>(Srow + c);
                float4 r4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (p.load_r) r4 = *reinterpret_cast<const float4 *>(Rin + c);
                float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (p.load_a) a4 = *reinterpret_cast<const float4 *>(Arow + c);
                const bool full = c + 3 < n;
                if (MODE != PASS_R_ONLY) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = c + e;
                        if (k < n) {
                            float an = avail(f4get(a4, e), f4get(r4, e), f4get(tv[j], e), ci,
                                             k == ii, lam, oml);
                            f4set(a4, e, an);
                            float dvv = an + f4get(r4, e);
                            if (dvv > dm.v) {
                                dm.v = dvv;
                                dm.k = k;
                            }
                        }
                    }
                    if (full) {
                        *reinterpret_cast<float4 *>(Arow + c) = a4;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (c + e < n) Arow[c + e] = f4get(a4, e);
                    }
                }
                if (MODE != PASS_A_ONLY) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = c + e;
                        if (k < n) {
                            top2_push(t2, f4get(a4, e) + f4get(s4, e), k);
                            f4set(u[j], e, lam * f4get(r4, e) + oml * f4get(s4, e));
                        }
                    }
                }
            }
        }

        // ---- workgroup reduction of the decision and the top-2 ----------
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            if (MODE != PASS_A_ONLY) {
                float ov1 = __shfl_xor(t2.v1, off, 64);
                int ok1 = __shfl_xor(t2.k1, off, 64);
                float ov2 = __shfl_xor(t2.v2, off, 64);
                top2_merge(t2, ov1, ok1, ov2);
            }
            if (MODE != PASS_R_ONLY) {
                float odv = __shfl_xor(dm.v, off, 64);
                int odk = __shfl_xor(dm.k, off, 64);
                argmax_merge(dm, odv, odk);
            }
        }
        const int slot = (int)(i & 1);
        if (lane == 0) {
            sh_f[slot][wave][0] = t2.v1;
            sh_f[slot][wave][1] = t2.v2;
            sh_f[slot][wave][2] = dm.v;
            sh_i[slot][wave][0] = t2.k1;
            sh_i[slot][wave][1] = dm.k;
        }
        __syncthreads();
        Top2 bt{sh_f[slot][0][0], sh_i[slot][0][0], sh_f[slot][0][1]};
        ArgMax bd{sh_f[slot][0][2], sh_i[slot][0][1]};
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            top2_merge(bt, sh_f[slot][w][0], sh_i[slot][w][0], sh_f[slot][w][1]);
            argmax_merge(bd, sh_f[slot][w][2], sh_i[slot][w][1]);
        }

        if (MODE != PASS_R_ONLY && tid == 0) {
            if (p.dec) p.dec[ii] = bd.k;
            if (p.eflag) {
                const uint8_t e = (uint8_t)(bd.k == ii);
                if (p.eflag[ii] != e) my_changed = 1;
                p.eflag[ii] = e;
                my_nex += e;
            }
        }

        // ---- responsibilities R_{t+1} and column partials ----------------
        if (MODE != PASS_A_ONLY) {
            const float m_other = oml * bt.v1;   // (1-lambda) * max over k' != k, k != k1
            const float m_self = oml * bt.v2;    // at k = k1
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int c = (j * T + tid) * 4;
                if (c < n) {
                    float4 rn;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = c + e;
                        const float v = f4get(u[j], e) - (k == bt.k1 ? m_self : m_other);
                        f4set(rn, e, v);
                        if (k < n) {
                            if (k == ii) p.rdiag[ii] = v;
                            else f4set(part[j], e, f4get(part[j], e) + fmaxf(0.0f, v));
                        }
                    }
                    if (c + 3 < n) {
                        *reinterpret_cast<float4 *>(Rout + c) = rn;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (c + e < n) Rout[c + e] = f4get(rn, e);
                    }
                }
            }
        }
    }

    if (MODE != PASS_A_ONLY) {
        float *P = p.partial + (int64_t)blockIdx.x * p.ldp;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = (j * T + tid) * 4;
            if (c < n) *reinterpret_cast<float4 *>(P + c) = part[j];
        }
    }
    if (MODE != PASS_R_ONLY && tid == 0 && p.st != nullptr) {
        if (my_nex) atomicAdd(&p.st->nex, my_nex);
        if (my_changed) atomicOr(&p.st->changed, 1);
    }
}

__global__ void k_col_reduce(ColArgs a) {
    if (a.st != nullptr && a.st->frozen) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < a.n) {
        double c = 0.0;
        const float *P = a.partial + k;
        for (int g = 0; g < a.nparts; ++g) c += (double)P[(int64_t)g * a.ldp];
        a.tcol[k] = (float)((double)a.rdiag[k] + c);
        a.ccol[k] = (float)c;
    }
    if (a.bookkeep && a.st != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        ApState *st = a.st;
        const int t = st->iter + 1;
        const int same = (t > 1) && (st->changed == 0);
        const int run = same ? st->run + 1 : 1;
        st->iter = t;
        st->run = run;
        st->last_nex = st->nex;
        if (st->conv_iter > 0 && run >= st->conv_iter && st->nex > 0) {
            st->converged = 1;
            st->frozen = 1;
        } else if (t >= st->max_iter) {
            st->frozen = 1;
        }
        st->nex = 0;
        st->changed = 0;
    }
}

__global__ void k_state_init(ApState *st, int32_t max_iter, int32_t conv_iter) {
    if (threadIdx.x == 0) {
        ApState s{};
        s.max_iter = max_iter;
        s.conv_iter = conv_iter;
        *st = s;
    }
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_rows(float *p, int64_t rows, int64_t cols, int64_t ld, float v) {
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x)
        for (int64_t c = threadIdx.x; c < cols; c += blockDim.x) p[r * ld + c] = v;
}

__global__ void k_copy_rows(float *dst, const float *src, int64_t rows, int64_t cols, int64_t ld) {
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const float4 *s4 = reinterpret_cast<const float4 *>(src + r * ld);
        float4 *d4 = reinterpret_cast<float4 *>(dst + r * ld);
        const int64_t c4 = cols / 4;
        for (int64_t c = threadIdx.x; c < c4; c += blockDim.x) d4[c] = s4[c];
        for (int64_t c = c4 * 4 + threadIdx.x; c < cols; c += blockDim.x) dst[r * ld + c] = src[r * ld + c];
    }
}

// ---- finalize ------------------------------------------------------------
// Exemplar list in ascending order (one workgroup, ballot + prefix).
__global__ __launch_bounds__(1024) void k_compact(const uint8_t *eflag, int32_t n, int32_t *ex,
                                                  int32_t *nex) {
    __shared__ int wcount[16];
    __shared__ int base;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += 1024) {
        const int k = k0 + tid;
        const bool e = (k < n) && eflag[k];
        const unsigned long long m = __ballot(e);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wcount[w];
        if (e) ex[off + before] = k;
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wcount[w];
            base += tot;
        }
        __syncthreads();
    }
    if (tid == 0) *nex = base;
}

// One wavefront per row: label = best exemplar by s(i,k), lowest k on ties.
__global__ __launch_bounds__(256) void k_labels(FinalArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= a.n) return;
    const int m = *a.nex;
    const float *Srow = a.S + i * a.ld;
    double dp = 0.0, ep = 0.0;
    int lab;
    if (m == 0) {
        lab = -1;
    } else if (a.eflag[i]) {
        lab = (int)i;
        ep = (double)Srow[i];
    } else {
        float bv = kNegInf;
        int bk = INT32_MAX;
        for (int j = lane; j < m; j += 64) {
            const int k = a.ex[j];
            const float v = Srow[k];
            if (v > bv || (v == bv && k < bk)) {
                bv = v;
                bk = k;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            float ov = __shfl_xor(bv, off, 64);
            int ok = __shfl_xor(bk, off, 64);
            if (ov > bv || (ov == bv && ok < bk)) {
                bv = ov;
                bk = ok;
            }
        }
        lab = bk;
        dp = (double)bv;
    }
    if (lane == 0) {
        a.idx[i] = lab;
        a.contrib[i] = dp;
        a.contrib[a.n + i] = ep;
    }
}

// Deterministic FP64 sums of the per-row contributions (fixed order).
__global__ __launch_bounds__(1024) void k_sum2(const double *contrib, int32_t n, double *sums) {
    __shared__ double sh[2][1024];
    const int tid = threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (int i = tid; i < n; i += 1024) {
        s0 += contrib[i];
        s1 += contrib[n + i];
    }
    sh[0][tid] = s0;
    sh[1][tid] = s1;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) {
            sh[0][tid] += sh[0][tid + w];
            sh[1][tid] += sh[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        sums[0] = sh[0][0];
        sums[1] = sh[1][0];
    }
}

template <int T, int J>
hipError_t launch_t(int mode, const PassArgs &a, int grid, hipStream_t s) {
    switch (mode) {
    case PASS_FULL: k_row_pass<T, J, PASS_FULL><<<grid, T, 0, s>>>(a); break;
    case PASS_R_ONLY: k_row_pass<T, J, PASS_R_ONLY><<<grid, T, 0, s>>>(a); break;
    default: k_row_pass<T, J, PASS_A_ONLY><<<grid, T, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

}  // namespace

PassPlan plan_pass(int64_t n, int num_cus) {
    PassPlan pl{};
    const int64_t q = (n + 3) / 4;   // float4 chunks per row
    if (n <= 4096) {
        pl.threads = 256;
        pl.chunks = (int)((q + 255) / 256);
        int64_t g = 2LL * num_cus;
        pl.grid = (int)(n < g ? n : g);
    } else {
        pl.threads = 1024;
        pl.chunks = (int)((q + 1023) / 1024);
        pl.grid = (int)(n < num_cus ? n : num_cus);
    }
    return pl;
}

hipError_t launch_row_pass(const PassPlan &pl, int mode, const PassArgs &a, hipStream_t s) {
    if (pl.threads == 256) {
        switch (pl.chunks) {
        case 1: return launch_t<256, 1>(mode, a, pl.grid, s);
        case 2: return launch_t<256, 2>(mode, a, pl.grid, s);
        case 3: return launch_t<256, 3>(mode, a, pl.grid, s);
        case 4: return launch_t<256, 4>(mode, a, pl.grid, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (pl.chunks) {
    case 1: return launch_t<1024, 1>(mode, a, pl.grid, s);
    case 2: return launch_t<1024, 2>(mode, a, pl.grid, s);
    case 3: return launch_t<1024, 3>(mode, a, pl.grid, s);
    case 4: return launch_t<1024, 4>(mode, a, pl.grid, s);
    case 5: return launch_t<1024, 5>(mode, a, pl.grid, s);
    case 6: return launch_t<1024, 6>(mode, a, pl.grid, s);
    case 7: return launch_t<1024, 7>(mode, a, pl.grid, s);
    case 8: return launch_t<1024, 8>(mode, a, pl.grid, s);
    case 9: return launch_t<1024, 9>(mode, a, pl.grid, s);
    case 10: return launch_t<1024, 10>(mode, a, pl.grid, s);
    case 11: return launch_t<1024, 11>(mode, a, pl.grid, s);
    case 12: return launch_t<1024, 12>(mode, a, pl.grid, s);
    case 13: return launch_t<1024, 13>(mode, a, pl.grid, s);
    case 14: return launch_t<1024, 14>(mode, a, pl.grid, s);
    case 15: return launch_t<1024, 15>(mode, a, pl.grid, s);
    case 16: return launch_t<1024, 16>(mode, a, pl.grid, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_col_reduce(const ColArgs &a, hipStream_t s) {
    const int threads = 256;
    const int grid = (a.n + threads - 1) / threads;
    k_col_reduce<<<grid, threads, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_state_init(ApState *st, int32_t max_iter, int32_t conv_iter, hipStream_t s) {
    k_state_init<<<1, 64, 0, s>>>(st, max_iter, conv_iter);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    k_fill_u8<<<(int)(g < 4096 ? (g > 0 ? g : 1) : 4096), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32_rows(float *p, int64_t rows, int64_t cols, int64_t ld, float v,
                                hipStream_t s) {
    int g = (int)(rows < 8192 ? rows : 8192);
    k_fill_rows<<<g > 0 ? g : 1, 256, 0, s>>>(p, rows, cols, ld, v);
    return hipGetLastError();
}

hipError_t launch_copy_rows(float *dst, const float *src, int64_t rows, int64_t cols, int64_t ld,
                            hipStream_t s) {
    int g = (int)(rows < 8192 ? rows : 8192);
    k_copy_rows<<<g > 0 ? g : 1, 256, 0, s>>>(dst, src, rows, cols, ld);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs &a, hipStream_t s) {
    k_compact<<<1, 1024, 0, s>>>(a.eflag, a.n, a.ex, a.nex);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_labels<<<(a.n + 3) / 4, 256, 0, s>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum2<<<1, 1024, 0, s>>>(a.contrib, a.n, a.sums);
    return hipGetLastError();
}

}  // namespace apx
