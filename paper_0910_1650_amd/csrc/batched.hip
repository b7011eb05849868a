// batched.hip -- many independent AP instances of uneven size in one launch
// per half-iteration (Algorithm 1 run on each instance; the sub-problems of
// partition AP, Algorithm 2 Step 2, are such a batch).
//
// Every launch walks a ragged work table: a work item is a contiguous block
// of rows of one instance.  A full row pass and a column reduce per iteration
// cover every active instance; each instance keeps its own stop-rule state,
// and a frozen (stopped) instance's work items exit at once.  All instances
// share one iteration counter, so the parity of t picks the responsibility
// buffer for all of them.
#include <cstring>
#include <vector>

#include "apx_internal.h"

namespace apx {
namespace {

constexpr float kNegInf = -INFINITY;
constexpr int BT = 256;   // threads per work item

struct InstDesc {
    const float *S;
    float *R[2];          // R_t lives in R[t & 1]
    float *A;
    int64_t ld;
    int32_t n;
    int32_t nparts;       // work items (= partial rows) of this instance
    float *partial;       // [nparts][ldp]
    int64_t ldp;
    float *tcol, *ccol, *rdiag;
    uint8_t *eflag;
    int32_t *dec;
    ApState *st;
    int32_t *idx;         // labels (caller's)
    int32_t *ex;          // exemplar list scratch (n)
    double *sums;         // [dpsim, expref]
    int32_t *nex_out;
    int32_t pad;
};

struct WorkItem {
    int32_t inst;
    int32_t row0, row1;
    int32_t part;         // partial row of this item
};

struct ColBlock {
    int32_t inst;
    int32_t col0;
};

__device__ __forceinline__ float f4get(const float4 &v, int e) {
    return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
}
__device__ __forceinline__ void f4set(float4 &v, int e, float x) {
    if (e == 0) v.x = x;
    else if (e == 1) v.y = x;
    else if (e == 2) v.z = x;
    else v.w = x;
}

__device__ __forceinline__ void top2_merge(float &v1, int &k1, float &v2, float ov1, int ok1, float ov2) {
    const bool take = (ov1 > v1) || (ov1 == v1 && ok1 < k1);
    const float nv2 = take ? fmaxf(ov2, v1) : fmaxf(v2, ov1);
    v1 = take ? ov1 : v1;
    k1 = take ? ok1 : k1;
    v2 = nv2;
}
__device__ __forceinline__ void argmax_merge(float &v, int &k, float ov, int ok) {
    const bool take = ov > v || (ov == v && ok < k);
    v = take ? ov : v;
    k = take ? ok : k;
}

// Batched row pass: same arithmetic as the single-instance pass (Eqs. (2)-(4)
// with damping, decision, column partials), one work item per workgroup.
// MODE: PASS_FULL, PASS_R_ONLY, PASS_R_COLD (also writes A_0 = 0).
template <int J, int MODE>
__global__ __launch_bounds__(BT) void k_batch_row_pass(const InstDesc *descs, const WorkItem *items,
                                                       float lam, int32_t t) {
#pragma clang fp contract(off)
    constexpr bool DO_A = (MODE == PASS_FULL);
    constexpr bool LD_RA = (MODE != PASS_R_COLD);
    constexpr int NW = BT / 64;
    const WorkItem wi = items[blockIdx.x];
    const InstDesc d = descs[wi.inst];
    if (d.st->frozen) return;
    __shared__ float sh_f[2][NW][3];
    __shared__ int sh_i[2][NW][2];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = d.n;
    const int64_t ld = d.ld;
    const float oml = 1.0f - lam;
    const float *Rin = d.R[t & 1];
    float *Rout = d.R[(t + 1) & 1];
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);

    float4 part[J];
#pragma unroll
    for (int j = 0; j < J; ++j) part[j] = z4;
    int my_nex = 0, my_changed = 0;

    for (int i = wi.row0; i < wi.row1; ++i) {
        const float *Srow = d.S + (int64_t)i * ld;
        const float *Rrow = Rin + (int64_t)i * ld;
        float *Arow = d.A + (int64_t)i * ld;
        float *Orow = Rout + (int64_t)i * ld;
        const float ci = DO_A ? d.ccol[i] : 0.0f;
        float v1 = kNegInf, v2 = kNegInf, dv = kNegInf;
        int k1 = INT32_MAX, dk = INT32_MAX;
        float4 u[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = (j * BT + tid) * 4;
            u[j] = z4;
            if (c >= n) continue;
            const bool full = c + 3 < n;
            const float4 s4 = *reinterpret_cast<const float4 *>(Srow + c);
            float4 r4 = z4, a4 = z4;
            if constexpr (LD_RA) {
                r4 = *reinterpret_cast<const float4 *>(Rrow + c);
                a4 = *reinterpret_cast<const float4 *>(Arow + c);
            }
            float4 t4 = z4;
            if constexpr (DO_A) t4 = *reinterpret_cast<const float4 *>(d.tcol + c);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = c + e;
                if (!(full || k < n)) continue;
                float a = f4get(a4, e);
                const float r = f4get(r4, e);
                if constexpr (DO_A) {
                    const float upd = (k == i) ? ci : fminf(0.0f, f4get(t4, e) - fmaxf(0.0f, r));
                    a = lam * a + oml * upd;
                    f4set(a4, e, a);
                    const float dvv = a + r;
                    const bool gt = dvv > dv;
                    dk = gt ? k : dk;
                    dv = gt ? dvv : dv;
                }
                const float v = a + f4get(s4, e);
                const bool gt = v > v1;
                v2 = gt ? v1 : fmaxf(v2, v);
                k1 = gt ? k : k1;
                v1 = gt ? v : v1;
                f4set(u[j], e, lam * r + oml * f4get(s4, e));
            }
            if constexpr (DO_A || MODE == PASS_R_COLD) {
                if (full) {
                    *reinterpret_cast<float4 *>(Arow + c) = a4;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (c + e < n) Arow[c + e] = f4get(a4, e);
                }
            }
        }
        // workgroup reduction (wavefront butterflies, then across wavefronts)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            top2_merge(v1, k1, v2, __shfl_xor(v1, off, 64), __shfl_xor(k1, off, 64),
                       __shfl_xor(v2, off, 64));
            if constexpr (DO_A) argmax_merge(dv, dk, __shfl_xor(dv, off, 64), __shfl_xor(dk, off, 64));
        }
        const int slot = i & 1;
        if (lane == 0) {
            sh_f[slot][wave][0] = v1;
            sh_f[slot][wave][1] = v2;
            sh_f[slot][wave][2] = dv;
            sh_i[slot][wave][0] = k1;
            sh_i[slot][wave][1] = dk;
        }
        __syncthreads();
        v1 = sh_f[slot][0][0];
        v2 = sh_f[slot][0][1];
        dv = sh_f[slot][0][2];
        k1 = sh_i[slot][0][0];
        dk = sh_i[slot][0][1];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            top2_merge(v1, k1, v2, sh_f[slot][w][0], sh_i[slot][w][0], sh_f[slot][w][1]);
            if constexpr (DO_A) argmax_merge(dv, dk, sh_f[slot][w][2], sh_i[slot][w][1]);
        }
        if constexpr (DO_A) {
            if (tid == 0) {
                d.dec[i] = dk;
                const uint8_t e = (uint8_t)(dk == i);
                if (d.eflag[i] != e) my_changed = 1;
                d.eflag[i] = e;
                my_nex += e;
            }
        }
        const float m_other = oml * v1, m_self = oml * v2;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = (j * BT + tid) * 4;
            if (c >= n) continue;
            const bool full = c + 3 < n;
            float4 rn;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = c + e;
                const float v = f4get(u[j], e) - (k == k1 ? m_self : m_other);
                f4set(rn, e, v);
                if (k < n) {
                    if (k == i) d.rdiag[i] = v;
                    else f4set(part[j], e, f4get(part[j], e) + fmaxf(0.0f, v));
                }
            }
            if (full) {
                *reinterpret_cast<float4 *>(Orow + c) = rn;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c + e < n) Orow[c + e] = f4get(rn, e);
            }
        }
    }
    float *P = d.partial + (int64_t)wi.part * d.ldp;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = (j * BT + tid) * 4;
        if (c < n) *reinterpret_cast<float4 *>(P + c) = part[j];
    }
    if constexpr (DO_A) {
        if (tid == 0) {
            if (my_nex) atomicAdd(&d.st->nex, my_nex);
            if (my_changed) atomicOr(&d.st->changed, 1);
        }
    }
}

// Column sums per instance (FP64, fixed order over the instance's work items)
// and, for the block holding column 0, the stop rule of that instance.
__global__ __launch_bounds__(256) void k_batch_col_reduce(const InstDesc *descs, const ColBlock *blocks,
                                                          int bookkeep) {
    const ColBlock cb = blocks[blockIdx.x];
    const InstDesc d = descs[cb.inst];
    if (d.st->frozen) return;
    const int k = cb.col0 + threadIdx.x;
    if (k < d.n) {
        double c = 0.0;
        for (int g = 0; g < d.nparts; ++g) c += (double)d.partial[(int64_t)g * d.ldp + k];
        d.tcol[k] = (float)((double)d.rdiag[k] + c);
        d.ccol[k] = (float)c;
    }
    if (bookkeep && cb.col0 == 0 && threadIdx.x == 0) {
        ApState *st = d.st;
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

__global__ void k_batch_init(const InstDesc *descs, int count, int32_t max_iter, int32_t conv_iter) {
    const int j = blockIdx.x;
    if (j >= count) return;
    const InstDesc d = descs[j];
    if (threadIdx.x == 0) {
        ApState s{};
        s.max_iter = max_iter;
        s.conv_iter = conv_iter;
        *d.st = s;
    }
    for (int i = threadIdx.x; i < d.n; i += blockDim.x) d.eflag[i] = 0;
}

// R_T into the caller's buffer when T is odd (R_T then lives in R[1]).
__global__ void k_batch_fix_r(const InstDesc *descs) {
    const InstDesc d = descs[blockIdx.y];
    if ((d.st->iter & 1) == 0) return;
    for (int64_t i = blockIdx.x; i < d.n; i += gridDim.x) {
        const float *src = d.R[1] + i * d.ld;
        float *dst = d.R[0] + i * d.ld;
        for (int c = threadIdx.x; c < d.n; c += blockDim.x) dst[c] = src[c];
    }
}

// Zero A (A_0 = 0) or R (R_0 = 0) of every instance.
__global__ void k_batch_zero(const InstDesc *descs, int which) {
    const InstDesc d = descs[blockIdx.y];
    float *M = which == 0 ? d.A : d.R[0];
    for (int64_t i = blockIdx.x; i < d.n; i += gridDim.x)
        for (int c = threadIdx.x; c < d.n; c += blockDim.x) M[i * d.ld + c] = 0.0f;
}

// Labels and FP64 net similarity, one workgroup per instance: exemplar list
// (ascending), then each non-exemplar takes the exemplar of largest s(i,k)
// (lowest k on ties); sums formed in a fixed order.
__global__ __launch_bounds__(1024) void k_batch_finalize(const InstDesc *descs) {
    const InstDesc d = descs[blockIdx.x];
    __shared__ int wcount[16];
    __shared__ int base;
    __shared__ double red[2][1024];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int k0 = 0; k0 < d.n; k0 += 1024) {
        const int k = k0 + tid;
        const bool e = (k < d.n) && d.eflag[k];
        const unsigned long long m = __ballot(e);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int w = 0; w < wave; ++w) off += wcount[w];
        if (e) d.ex[off + before] = k;
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < 16; ++w) tot += wcount[w];
            base += tot;
        }
        __syncthreads();
    }
    const int m = base;
    double dp = 0.0, ep = 0.0;
    // one wavefront per row
    for (int i = wave; i < d.n; i += 16) {
        const float *Srow = d.S + (int64_t)i * d.ld;
        int lab;
        if (m == 0) {
            lab = -1;
        } else if (d.eflag[i]) {
            lab = i;
            if (lane == 0) ep += (double)Srow[i];
        } else {
            float bv = kNegInf;
            int bk = INT32_MAX;
            for (int j = lane; j < m; j += 64) {
                const int k = d.ex[j];
                const float v = Srow[k];
                if (v > bv || (v == bv && k < bk)) {
                    bv = v;
                    bk = k;
                }
            }
            for (int o = 32; o >= 1; o >>= 1) {
                const float ov = __shfl_xor(bv, o, 64);
                const int ok = __shfl_xor(bk, o, 64);
                if (ov > bv || (ov == bv && ok < bk)) {
                    bv = ov;
                    bk = ok;
                }
            }
            lab = bk;
            if (lane == 0) dp += (double)bv;
        }
        if (lane == 0) d.idx[i] = lab;
    }
    red[0][tid] = dp;
    red[1][tid] = ep;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        d.sums[0] = red[0][0];
        d.sums[1] = red[1][0];
        *d.nex_out = m;
    }
}

template <int J>
hipError_t launch_batch_pass(int mode, const InstDesc *descs, const WorkItem *items, int nitems,
                             float lam, int32_t t, hipStream_t s) {
    switch (mode) {
    case PASS_FULL: k_batch_row_pass<J, PASS_FULL><<<nitems, BT, 0, s>>>(descs, items, lam, t); break;
    case PASS_R_ONLY: k_batch_row_pass<J, PASS_R_ONLY><<<nitems, BT, 0, s>>>(descs, items, lam, t); break;
    default: k_batch_row_pass<J, PASS_R_COLD><<<nitems, BT, 0, s>>>(descs, items, lam, t); break;
    }
    return hipGetLastError();
}

hipError_t batch_pass(int J, int mode, const InstDesc *descs, const WorkItem *items, int nitems,
                      float lam, int32_t t, hipStream_t s) {
    switch (J) {
    case 1: return launch_batch_pass<1>(mode, descs, items, nitems, lam, t, s);
    case 2: return launch_batch_pass<2>(mode, descs, items, nitems, lam, t, s);
    case 3: return launch_batch_pass<3>(mode, descs, items, nitems, lam, t, s);
    case 4: return launch_batch_pass<4>(mode, descs, items, nitems, lam, t, s);
    case 5: return launch_batch_pass<5>(mode, descs, items, nitems, lam, t, s);
    case 6: return launch_batch_pass<6>(mode, descs, items, nitems, lam, t, s);
    case 7: return launch_batch_pass<7>(mode, descs, items, nitems, lam, t, s);
    case 8: return launch_batch_pass<8>(mode, descs, items, nitems, lam, t, s);
    case 9: return launch_batch_pass<9>(mode, descs, items, nitems, lam, t, s);
    case 10: return launch_batch_pass<10>(mode, descs, items, nitems, lam, t, s);
    case 11: return launch_batch_pass<11>(mode, descs, items, nitems, lam, t, s);
    case 12: return launch_batch_pass<12>(mode, descs, items, nitems, lam, t, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

namespace {

struct BatchPlan {
    int J;
    std::vector<WorkItem> items;
    std::vector<int32_t> nparts;
    std::vector<ColBlock> cblocks;
    // workspace offsets (relative to the plan's base)
    std::vector<size_t> o_r2, o_part, o_t, o_c, o_d, o_e, o_dec, o_ex;
    size_t o_st, o_sum, o_nex, o_desc, o_items, o_cb, bytes;
};

BatchPlan make_plan(int32_t count, const BatchSpec *spec, int num_cus) {
    BatchPlan P;
    int64_t max_n = 0, total = 0;
    for (int j = 0; j < count; ++j) {
        max_n = spec[j].n > max_n ? spec[j].n : max_n;
        total += spec[j].n * spec[j].n;
    }
    P.J = (int)((max_n + 4 * BT - 1) / (4 * BT));
    // Work items: about 4 per CU in total, at least one per instance, rows
    // split so that items carry similar element counts.
    const int64_t target = total / (4LL * num_cus) + 1;
    P.nparts.resize(count);
    for (int j = 0; j < count; ++j) {
        const int64_t n = spec[j].n;
        int64_t rows = target / (n > 0 ? n : 1);
        if (rows < 1) rows = 1;
        if (rows > n) rows = n;
        int32_t p = 0;
        for (int64_t r = 0; r < n; r += rows, ++p)
            P.items.push_back(WorkItem{j, (int32_t)r, (int32_t)(r + rows < n ? r + rows : n), p});
        P.nparts[j] = p;
        for (int64_t c = 0; c < n; c += 256) P.cblocks.push_back(ColBlock{j, (int32_t)c});
    }
    WsLayout L;
    P.o_r2.resize(count); P.o_part.resize(count); P.o_t.resize(count); P.o_c.resize(count);
    P.o_d.resize(count); P.o_e.resize(count); P.o_dec.resize(count); P.o_ex.resize(count);
    for (int j = 0; j < count; ++j) {
        const int64_t n = spec[j].n, ldp = (n + 3) & ~int64_t(3);
        P.o_r2[j] = L.take(sizeof(float) * (size_t)n * (size_t)spec[j].ld);
        P.o_part[j] = L.take(sizeof(float) * (size_t)ldp * P.nparts[j]);
        P.o_t[j] = L.take(sizeof(float) * ldp);
        P.o_c[j] = L.take(sizeof(float) * ldp);
        P.o_d[j] = L.take(sizeof(float) * ldp);
        P.o_e[j] = L.take((size_t)n);
        P.o_dec[j] = L.take(sizeof(int32_t) * n);
        P.o_ex[j] = L.take(sizeof(int32_t) * n);
    }
    P.o_st = L.take(sizeof(ApState) * count);
    P.o_sum = L.take(sizeof(double) * 2 * count);
    P.o_nex = L.take(sizeof(int32_t) * count);
    P.o_desc = L.take(sizeof(InstDesc) * count);
    P.o_items = L.take(sizeof(WorkItem) * P.items.size());
    P.o_cb = L.take(sizeof(ColBlock) * P.cblocks.size());
    P.bytes = L.off;
    return P;
}

}  // namespace

size_t batched_ws_bytes(int32_t count, const BatchSpec *spec, int num_cus) {
    return make_plan(count, spec, num_cus).bytes;
}

// Host driver shared by ap_solve_batched and pap_solve (Step 2): the
// workspace slice starts at ctx->ws_base.
apx_status batched_solve(apx_ctx *ctx, int32_t count, const BatchSpec *spec, int32_t warm,
                         const apx_params *params, apx_result *res) {
    hipStream_t s = ctx->stream;
    BatchPlan P = make_plan(count, spec, ctx->num_cus);
    if (P.J > 12) return set_err(ctx, APX_ENOTIMPL, "batched instances are limited to n <= %d", 12 * 4 * BT);
    apx_status st = ws_reserve(ctx, ctx->ws_base + P.bytes);
    if (st != APX_OK) return st;
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;

    ApState *dst = reinterpret_cast<ApState *>(b + P.o_st);
    double *dsum = reinterpret_cast<double *>(b + P.o_sum);
    int32_t *dnex = reinterpret_cast<int32_t *>(b + P.o_nex);
    std::vector<InstDesc> descs(count);
    int64_t max_n = 0;
    for (int j = 0; j < count; ++j) {
        InstDesc &d = descs[j];
        std::memset(&d, 0, sizeof d);
        d.S = spec[j].S;
        d.R[0] = spec[j].R;
        d.R[1] = reinterpret_cast<float *>(b + P.o_r2[j]);
        d.A = spec[j].A;
        d.ld = spec[j].ld;
        d.n = (int32_t)spec[j].n;
        d.nparts = P.nparts[j];
        d.partial = reinterpret_cast<float *>(b + P.o_part[j]);
        d.ldp = (spec[j].n + 3) & ~int64_t(3);
        d.tcol = reinterpret_cast<float *>(b + P.o_t[j]);
        d.ccol = reinterpret_cast<float *>(b + P.o_c[j]);
        d.rdiag = reinterpret_cast<float *>(b + P.o_d[j]);
        d.eflag = reinterpret_cast<uint8_t *>(b + P.o_e[j]);
        d.dec = reinterpret_cast<int32_t *>(b + P.o_dec[j]);
        d.st = dst + j;
        d.idx = spec[j].idx;
        d.ex = reinterpret_cast<int32_t *>(b + P.o_ex[j]);
        d.sums = dsum + 2 * j;
        d.nex_out = dnex + j;
        max_n = spec[j].n > max_n ? spec[j].n : max_n;
    }
    InstDesc *ddesc = reinterpret_cast<InstDesc *>(b + P.o_desc);
    WorkItem *ditems = reinterpret_cast<WorkItem *>(b + P.o_items);
    ColBlock *dcb = reinterpret_cast<ColBlock *>(b + P.o_cb);
    hipError_t e;
    if ((e = hipMemcpyAsync(ddesc, descs.data(), sizeof(InstDesc) * count, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(ditems, P.items.data(), sizeof(WorkItem) * P.items.size(), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(dcb, P.cblocks.data(), sizeof(ColBlock) * P.cblocks.size(), hipMemcpyHostToDevice, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_err(ctx, e, "batch tables");

    const float lam = params->damping;
    const int J = P.J, nitems = (int)P.items.size(), ncb = (int)P.cblocks.size();
    const dim3 zgrid((unsigned)(max_n < 2048 ? max_n : 2048), (unsigned)count);
    k_batch_init<<<count, 256, 0, s>>>(ddesc, count, params->max_iter, params->conv_iter);
    if ((e = hipGetLastError())) return hip_err(ctx, e, "batch init");
    if (warm == APX_COLD) {
        if ((e = batch_pass(J, PASS_R_COLD, ddesc, ditems, nitems, lam, 0, s))) return hip_err(ctx, e, "prologue");
    } else {
        if (warm == APX_WARM_A) {
            k_batch_zero<<<zgrid, 256, 0, s>>>(ddesc, 1);
            if ((e = hipGetLastError())) return hip_err(ctx, e, "R_0");
        }
        if ((e = batch_pass(J, PASS_R_ONLY, ddesc, ditems, nitems, lam, 0, s))) return hip_err(ctx, e, "prologue");
    }
    k_batch_col_reduce<<<ncb, 256, 0, s>>>(ddesc, dcb, 0);
    if ((e = hipGetLastError())) return hip_err(ctx, e, "column reduce");

    const int chunk = params->check_every > 0 ? params->check_every : 16;
    std::vector<ApState> hst(count);
    int32_t t = 1;
    for (;;) {
        int32_t stop_at = t + chunk;
        if (stop_at > params->max_iter + 1) stop_at = params->max_iter + 1;
        for (; t < stop_at; ++t) {
            if ((e = batch_pass(J, PASS_FULL, ddesc, ditems, nitems, lam, t, s))) return hip_err(ctx, e, "row pass");
            k_batch_col_reduce<<<ncb, 256, 0, s>>>(ddesc, dcb, 1);
            if ((e = hipGetLastError())) return hip_err(ctx, e, "column reduce");
        }
        if ((e = hipMemcpyAsync(hst.data(), dst, sizeof(ApState) * count, hipMemcpyDeviceToHost, s)) ||
            (e = hipStreamSynchronize(s)))
            return hip_err(ctx, e, "state");
        bool all = true;
        for (int j = 0; j < count; ++j) all = all && hst[j].frozen;
        if (all || t > params->max_iter) break;
    }
    k_batch_fix_r<<<zgrid, 256, 0, s>>>(ddesc);
    if ((e = hipGetLastError())) return hip_err(ctx, e, "copy R");
    k_batch_finalize<<<count, 1024, 0, s>>>(ddesc);
    if ((e = hipGetLastError())) return hip_err(ctx, e, "finalize");
    std::vector<double> sums(2 * (size_t)count);
    std::vector<int32_t> nex(count);
    if ((e = hipMemcpyAsync(sums.data(), dsum, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s)) ||
        (e = hipMemcpyAsync(nex.data(), dnex, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_err(ctx, e, "results");
    for (int j = 0; j < count; ++j) {
        apx_result &r = res[j];
        std::memset(&r, 0, sizeof r);
        r.iterations = hst[j].iter;
        r.converged = hst[j].converged;
        r.n_exemplars = nex[j];
        if (nex[j] == 0) {
            r.dpsim = r.expref = r.netsim = NAN;
        } else {
            r.dpsim = sums[2 * j];
            r.expref = sums[2 * j + 1];
            r.netsim = r.dpsim + r.expref;
        }
        r.status = APX_OK;
    }
    return APX_OK;
}

}  // namespace apx
