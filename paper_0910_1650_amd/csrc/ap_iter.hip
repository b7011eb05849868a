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
#include <cmath>
#include <cstdlib>

namespace apx {
namespace {

constexpr float kNegInf = -INFINITY;
// Dynamic LDS of the row pass (u and column partials): 160 KB per CU on
// gfx950, minus the static reduction scratch.
constexpr int kMaxDynLds = 160 * 1024 - 1024;
// The implicit pass keeps its row state in static LDS as well.
constexpr int kMaxDynLdsImp = 160 * 1024 - 2048;

struct Top2 {
    float v1;   // largest a+s
    int k1;     // its column (lowest on ties)
    float v2;   // largest over the other columns
};

struct ArgMax {
    float v;
    int k;
};

// All merges are written as selects (no branches): columns arrive in
// ascending order within a thread, so a tie keeps the earlier column.
__device__ __forceinline__ void top2_push(Top2 &t, float v, int k) {
    const bool gt = v > t.v1;
    t.v2 = gt ? t.v1 : fmaxf(t.v2, v);
    t.k1 = gt ? k : t.k1;
    t.v1 = gt ? v : t.v1;
}

__device__ __forceinline__ void top2_merge(Top2 &t, float ov1, int ok1, float ov2) {
    const bool take = (ov1 > t.v1) || (ov1 == t.v1 && ok1 < t.k1);
    const float nv2 = take ? fmaxf(ov2, t.v1) : fmaxf(t.v2, ov1);
    t.v1 = take ? ov1 : t.v1;
    t.k1 = take ? ok1 : t.k1;
    t.v2 = nv2;
}

__device__ __forceinline__ void argmax_merge(ArgMax &m, float ov, int ok) {
    const bool take = ov > m.v || (ov == m.v && ok < m.k);
    m.v = take ? ov : m.v;
    m.k = take ? ok : m.k;
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

// Workgroup barrier that orders LDS only: global loads issued before it stay
// in flight (the next row is prefetched across the reduction).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, const float4 &v) { *reinterpret_cast<float4 *>(p) = v; }

// Row access: every chunk of a row is addressed from a uniform row base (in
// scalar registers) plus one shared per-thread byte offset (tid*16) and a
// compile-time chunk offset (j*T*16).  Plain global loads and stores are
// used: raw buffer-resource loads and stores (descriptor word 3 = 0x00020000)
// gave run-to-run differences in this kernel on gfx950 for rows longer than
// ~12k elements, while global memory operations are exact and reproducible.
typedef const float *rsrc_t;
typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ rsrc_t row_rsrc(const float *base, int64_t) { return base; }
// S, R and A are streamed once per iteration and never re-read in the same
// pass: loads and stores carry the nontemporal hint.
__device__ __forceinline__ float4 bld4(rsrc_t r, int voff, int soff) {
    const v4f v = __builtin_nontemporal_load(
        reinterpret_cast<const v4f *>(reinterpret_cast<const char *>(r) + voff + soff));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void bst4(rsrc_t r, int voff, int soff, const float4 &x) {
    const v4f v = {x.x, x.y, x.z, x.w};
    __builtin_nontemporal_store(
        v, reinterpret_cast<v4f *>(const_cast<char *>(reinterpret_cast<const char *>(r)) + voff + soff));
}

// ---- per-chunk pieces of the row pass ------------------------------------
// Thread tid owns the float4 chunks j = 0..J-1 at columns c_j = 4*(j*T+tid)
// of every row.  Inside a thread, columns are visited in ascending order and
// identified by the local index 4*j+e (a compile-time constant), so ties keep
// the lowest column without any per-element index arithmetic.  A column k
// belongs to thread (k/4) % T, chunk (k/4) / T, element k % 4.
struct ColOwner {
    bool mine;   // this thread owns the column
    int j, e;    // its chunk and element (uniform)
};
template <int T>
__device__ __forceinline__ ColOwner owner_of(int k, int tid) {
    return ColOwner{((k >> 2) % T) == tid, (k >> 2) / T, k & 3};
}
template <int T>
__device__ __forceinline__ int local_to_col(int le, int tid) {
    return ((le >> 2) * T + tid) * 4 + (le & 3);
}

// Availabilities A_t (Eqs. (3), (4), damping) of chunk j, and the running
// decision argmax_k a(i,k)+r(i,k) as a local index.
__device__ __forceinline__ void chunk_avail(float4 &a, const float4 &r, const float4 &t, float ci,
                                            int j, const ColOwner &dg, int c, int n, bool full,
                                            float lam, float oml, float &dv, int &dl) {
#pragma clang fp contract(off)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (full || c + e < n) {
            const bool diag = dg.mine && dg.j == j && dg.e == e;
            const float an = avail(f4get(a, e), f4get(r, e), f4get(t, e), ci, diag, lam, oml);
            f4set(a, e, an);
            const float v = an + f4get(r, e);
            const bool gt = v > dv;
            dl = gt ? 4 * j + e : dl;
            dv = gt ? v : dv;
        }
    }
}

// Top-2 of a(i,k)+s(i,k) (local indices) and u = lambda*r + (1-lambda)*s.
__device__ __forceinline__ float4 chunk_top2(const float4 &a, const float4 &r, const float4 &sv,
                                             int j, int c, int n, bool full, float lam, float oml,
                                             float &v1, int &l1, float &v2) {
#pragma clang fp contract(off)
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if (full || c + e < n) {
            const float v = f4get(a, e) + f4get(sv, e);
            const bool gt = v > v1;
            v2 = gt ? v1 : fmaxf(v2, v);
            l1 = gt ? 4 * j + e : l1;
            v1 = gt ? v : v1;
            f4set(u, e, lam * f4get(r, e) + oml * f4get(sv, e));
        }
    }
    return u;
}

// R_{t+1} (Eq. (2), damping) of chunk j from u; returns max(0, r) for the
// column partials (zero on the diagonal and outside the row).
__device__ __forceinline__ float4 chunk_resp(const float4 &u, int j, const ColOwner &k1,
                                             const ColOwner &dg, float m_self, float m_other,
                                             int c, int n, bool full, float4 &rn, float *rdiag) {
#pragma clang fp contract(off)
    float4 pos;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const bool self = k1.mine && k1.j == j && k1.e == e;
        const bool diag = dg.mine && dg.j == j && dg.e == e;
        const float v = f4get(u, e) - (self ? m_self : m_other);
        f4set(rn, e, v);
        f4set(pos, e, (diag || !(full || c + e < n)) ? 0.0f : fmaxf(0.0f, v));
        if (diag) *rdiag = v;
    }
    return pos;
}

__device__ __forceinline__ void add4(float4 &a, const float4 &b) {
    a.x += b.x;
    a.y += b.y;
    a.z += b.z;
    a.w += b.w;
}

// Store a chunk: one 16-byte buffer store, or element stores for the tail.
__device__ __forceinline__ void store_chunk(float *row, rsrc_t rs, int voff, int soff, int c, int n,
                                            bool full, const float4 &v) {
    if (full) {
        bst4(rs, voff, soff, v);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (c + e < n) row[c + e] = f4get(v, e);
    }
}

// Workgroup reduction of the decision and the top-2 (deterministic order):
// wavefront butterflies, one LDS slot per wavefront, then every wavefront
// reduces the NW slots lane-parallel and broadcasts lane 0's result.
template <int NW, bool DO_A, bool DO_R>
__device__ __forceinline__ void wg_reduce(Top2 &t2, ArgMax &dm, float (*sh_f)[3], int (*sh_i)[2],
                                          int lane, int wave) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        if constexpr (DO_R) {
            const float ov1 = __shfl_xor(t2.v1, off, 64);
            const int ok1 = __shfl_xor(t2.k1, off, 64);
            const float ov2 = __shfl_xor(t2.v2, off, 64);
            top2_merge(t2, ov1, ok1, ov2);
        }
        if constexpr (DO_A) {
            const float odv = __shfl_xor(dm.v, off, 64);
            const int odk = __shfl_xor(dm.k, off, 64);
            argmax_merge(dm, odv, odk);
        }
    }
    if (lane == 0) {
        sh_f[wave][0] = t2.v1;
        sh_f[wave][1] = t2.v2;
        sh_f[wave][2] = dm.v;
        sh_i[wave][0] = t2.k1;
        sh_i[wave][1] = dm.k;
    }
    lds_barrier();
    if constexpr (NW > 1) {
        const bool has = lane < NW;
        const int w = has ? lane : 0;
        if constexpr (DO_R) t2 = has ? Top2{sh_f[w][0], sh_i[w][0], sh_f[w][1]} : Top2{kNegInf, INT32_MAX, kNegInf};
        if constexpr (DO_A) dm = has ? ArgMax{sh_f[w][2], sh_i[w][1]} : ArgMax{kNegInf, INT32_MAX};
#pragma unroll
        for (int off = NW / 2; off >= 1; off >>= 1) {
            if constexpr (DO_R) {
                const float ov1 = __shfl_xor(t2.v1, off, 64);
                const int ok1 = __shfl_xor(t2.k1, off, 64);
                const float ov2 = __shfl_xor(t2.v2, off, 64);
                top2_merge(t2, ov1, ok1, ov2);
            }
            if constexpr (DO_A) {
                const float odv = __shfl_xor(dm.v, off, 64);
                const int odk = __shfl_xor(dm.k, off, 64);
                argmax_merge(dm, odv, odk);
            }
        }
        if constexpr (DO_R) t2 = Top2{__shfl(t2.v1, 0, 64), __shfl(t2.k1, 0, 64), __shfl(t2.v2, 0, 64)};
        if constexpr (DO_A) dm = ArgMax{__shfl(dm.v, 0, 64), __shfl(dm.k, 0, 64)};
    } else {
        t2 = Top2{sh_f[0][0], sh_i[0][0], sh_f[0][1]};
        dm = ArgMax{sh_f[0][2], sh_i[0][1]};
    }
}

// Decision bookkeeping of row ii (thread 0): raw decision, exemplar flag,
// change of the exemplar set, exemplar count.
__device__ __forceinline__ void note_decision(const PassArgs &p, int ii, int k, int &my_nex,
                                              int &my_changed) {
    if (p.dec) p.dec[ii] = k;
    if (p.eflag) {
        const uint8_t e = (uint8_t)(k == ii);
        if (p.eflag[ii] != e) my_changed = 1;
        p.eflag[ii] = e;
        my_nex += e;
    }
}

// Row pass, LDS-resident variant.  u = lambda*r + (1-lambda)*s and the
// column partials live in LDS (2 * 16 * ceil(n/4) bytes), which leaves the
// registers free to hold the next row's S, R, A chunks: they are loaded
// before the top-2 reduction of the current row, so HBM reads stay in flight
// across the reduction and the R_{t+1} stores.
template <int T, int J, int MODE>
__global__ __launch_bounds__(T) void k_row_pass(PassArgs p) {
    constexpr bool DO_A = (MODE == PASS_FULL || MODE == PASS_A_ONLY);
    constexpr bool DO_R = (MODE != PASS_A_ONLY);
    constexpr bool LD_S = DO_R;
    constexpr bool LD_RA = (MODE != PASS_R_COLD);
    constexpr int NW = T / 64;

    if (p.st != nullptr && p.st->frozen) return;
    __shared__ float sh_f[2][NW][3];
    __shared__ int sh_i[2][NW][2];
    extern __shared__ float4 dyn[];
    const int q = (p.n + 3) >> 2;                // float4 chunks per row
    float4 *lu = dyn;                            // u, q entries
    float4 *lpart = dyn + q;                     // column partials, q entries

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
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int voff = tid * 16;
    const int c0 = tid * 4;
    const int cl = ((J - 1) * T + tid) * 4;      // column of the last chunk
    const bool last_in = cl < n;                 // last chunk holds data
    const bool last_full = cl + 3 < n;

#pragma unroll
    for (int j = 0; j < J; ++j)
        if constexpr (DO_R)
            if (j < J - 1 || last_in) lpart[j * T + tid] = z4;
    int my_nex = 0, my_changed = 0;

    // The column vector t_k is read per chunk inside the availability step
    // (an L2 hit), never held in registers across the row reduction: with the
    // next row's loads in flight, t_k values held across the reduction came
    // out wrong in some lanes (lanes 12-15 of each 16) on gfx950 with this
    // compiler; reading them at use is exact and costs no HBM traffic.
    float4 s4[LD_S ? J : 1], r4[LD_RA ? J : 1], a4[LD_RA ? J : 1];
    auto load_row = [&](int64_t i) {
        const rsrc_t srs = row_rsrc(p.S + i * ld, ld);
        const rsrc_t rrs = row_rsrc(p.Rin + i * ld, ld);
        const rsrc_t ars = row_rsrc(p.A + i * ld, ld);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (j < J - 1 || last_in) {
                if constexpr (LD_S) s4[j] = bld4(srs, voff, j * T * 16);
                if constexpr (LD_RA) {
                    r4[j] = bld4(rrs, voff, j * T * 16);
                    a4[j] = bld4(ars, voff, j * T * 16);
                }
            }
        }
    };
    if (r0 < r1) load_row(r0);

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const ColOwner dg = owner_of<T>(ii, tid);
        float *Arow = p.A + i * ld;
        const rsrc_t a_rs = row_rsrc(Arow, ld);
        float ci = 0.0f;
        if constexpr (DO_A) ci = p.ccol[ii];
        float v1 = kNegInf, v2 = kNegInf, dv = kNegInf;
        int l1 = -1, dl = -1;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (!(j < J - 1 || last_in)) continue;
            const bool full = (j < J - 1) || last_full;
            const int c = c0 + j * T * 4;
            float4 a = z4, r = z4;
            if constexpr (LD_RA) {
                a = a4[j];
                r = r4[j];
            }
            if constexpr (DO_A) {
                chunk_avail(a, r, ld4(p.tcol + c), ci, j, dg, c, n, full, lam, oml, dv, dl);
                store_chunk(Arow, a_rs, voff, j * T * 16, c, n, full, a);
            }
            if constexpr (DO_R) lu[j * T + tid] = chunk_top2(a, r, s4[j], j, c, n, full, lam, oml, v1, l1, v2);
        }
        // Keep the scheduler from hoisting the next row's loads into the
        // computation above: both rows' registers would then be live at once.
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < r1) load_row(i + 1);
        __builtin_amdgcn_sched_barrier(0);

        Top2 t2{v1, l1 < 0 ? INT32_MAX : local_to_col<T>(l1, tid), v2};
        ArgMax dm{dv, dl < 0 ? INT32_MAX : local_to_col<T>(dl, tid)};
        const int slot = (int)(i & 1);
        wg_reduce<NW, DO_A, DO_R>(t2, dm, sh_f[slot], sh_i[slot], lane, wave);
        if constexpr (DO_A) {
            if (tid == 0) note_decision(p, ii, dm.k, my_nex, my_changed);
        }
        if constexpr (DO_R) {
            const float m_other = oml * t2.v1;   // (1-lambda) * max over k' != k, for k != k1
            const float m_self = oml * t2.v2;    // for k = k1
            const ColOwner ko = owner_of<T>(t2.k1, tid);
            float *Rout = p.Rout + i * ld;
            const rsrc_t r_rs = row_rsrc(Rout, ld);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!(j < J - 1 || last_in)) continue;
                const bool full = (j < J - 1) || last_full;
                const int c = c0 + j * T * 4;
                float4 rn;
                const float4 pos = chunk_resp(lu[j * T + tid], j, ko, dg, m_self, m_other, c, n,
                                              full, rn, p.rdiag + ii);
                store_chunk(Rout, r_rs, voff, j * T * 16, c, n, full, rn);
                float4 acc = lpart[j * T + tid];
                add4(acc, pos);
                lpart[j * T + tid] = acc;
            }
        }
    }

    if constexpr (DO_R) {
        float *P = p.partial + (int64_t)blockIdx.x * p.ldp;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < J - 1 || last_in) st4(P + c0 + j * T * 4, lpart[j * T + tid]);
    }
    if constexpr (DO_A) {
        if (tid == 0 && p.st != nullptr) {
            if (my_nex) atomicAdd(&p.st->nex, my_nex);
            if (my_changed) atomicOr(&p.st->changed, 1);
        }
    }
}

// Row pass, register variant for long rows (LDS too small for u and the
// partials): u and the partials live in registers, t_k is read per chunk
// from L2, and rows are not prefetched.
// PASS_FULL_DELTA also records the largest message changes of the pass,
// max |a_t - a_{t-1}| and max |r_{t+1} - r_t| over the valid elements.
template <int T, int J, int MODE>
__global__ __launch_bounds__(T) void k_row_pass_reg(PassArgs p) {
    constexpr bool DELTA = (MODE == PASS_FULL_DELTA);
    constexpr bool DO_A = (MODE == PASS_FULL || MODE == PASS_A_ONLY || DELTA);
    constexpr bool DO_R = (MODE != PASS_A_ONLY);
    constexpr bool LD_S = DO_R;
    constexpr bool LD_RA = (MODE != PASS_R_COLD);
    constexpr int NW = T / 64;

    if (p.st != nullptr && p.st->frozen) return;
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
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int voff = tid * 16;
    const int c0 = tid * 4;
    const int cl = ((J - 1) * T + tid) * 4;
    const bool last_in = cl < n;
    const bool last_full = cl + 3 < n;

    float4 part[DO_R ? J : 1];
#pragma unroll
    for (int j = 0; j < J; ++j)
        if constexpr (DO_R) part[j] = z4;
    int my_nex = 0, my_changed = 0;
    float mda = 0.0f, mdr = 0.0f;   // DELTA: largest |change| of A and R seen by this thread
    const rsrc_t t_rs = row_rsrc(p.tcol, p.ldp);

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const ColOwner dg = owner_of<T>(ii, tid);
        float *Arow = p.A + i * ld;
        const rsrc_t a_rs = row_rsrc(Arow, ld);
        const rsrc_t r_rs = row_rsrc(p.Rin + i * ld, ld);
        const rsrc_t s_rs = row_rsrc(p.S + i * ld, ld);
        float ci = 0.0f;
        if constexpr (DO_A) ci = p.ccol[ii];
        float v1 = kNegInf, v2 = kNegInf, dv = kNegInf;
        int l1 = -1, dl = -1;
        float4 u[DO_R ? J : 1];
        float4 rold[DELTA ? J : 1];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (!(j < J - 1 || last_in)) continue;
            const bool full = (j < J - 1) || last_full;
            const int c = c0 + j * T * 4;
            float4 a = z4, r = z4, sv = z4;
            if constexpr (LD_RA) {
                a = bld4(a_rs, voff, j * T * 16);
                r = bld4(r_rs, voff, j * T * 16);
            }
            if constexpr (LD_S) sv = bld4(s_rs, voff, j * T * 16);
            if constexpr (DO_A) {
                const float4 aold = a;
                chunk_avail(a, r, bld4(t_rs, voff, j * T * 16), ci, j, dg, c, n, full, lam, oml, dv, dl);
                store_chunk(Arow, a_rs, voff, j * T * 16, c, n, full, a);
                if constexpr (DELTA) {
                    rold[j] = r;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (full || c + e < n) mda = fmaxf(mda, fabsf(f4get(a, e) - f4get(aold, e)));
                }
            }
            if constexpr (DO_R) u[j] = chunk_top2(a, r, sv, j, c, n, full, lam, oml, v1, l1, v2);
        }
        Top2 t2{v1, l1 < 0 ? INT32_MAX : local_to_col<T>(l1, tid), v2};
        ArgMax dm{dv, dl < 0 ? INT32_MAX : local_to_col<T>(dl, tid)};
        const int slot = (int)(i & 1);
        wg_reduce<NW, DO_A, DO_R>(t2, dm, sh_f[slot], sh_i[slot], lane, wave);
        if constexpr (DO_A) {
            if (tid == 0) note_decision(p, ii, dm.k, my_nex, my_changed);
        }
        if constexpr (DO_R) {
            const float m_other = oml * t2.v1;
            const float m_self = oml * t2.v2;
            const ColOwner ko = owner_of<T>(t2.k1, tid);
            float *Rout = p.Rout + i * ld;
            const rsrc_t o_rs = row_rsrc(Rout, ld);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!(j < J - 1 || last_in)) continue;
                const bool full = (j < J - 1) || last_full;
                const int c = c0 + j * T * 4;
                float4 rn;
                add4(part[j], chunk_resp(u[j], j, ko, dg, m_self, m_other, c, n, full, rn,
                                         p.rdiag + ii));
                store_chunk(Rout, o_rs, voff, j * T * 16, c, n, full, rn);
                if constexpr (DELTA) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (full || c + e < n) mdr = fmaxf(mdr, fabsf(f4get(rn, e) - f4get(rold[j], e)));
                }
            }
        }
    }
    if constexpr (DO_R) {
        float *P = p.partial + (int64_t)blockIdx.x * p.ldp;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < J - 1 || last_in) st4(P + c0 + j * T * 4, part[j]);
    }
    if constexpr (DO_A) {
        if (tid == 0 && p.st != nullptr) {
            if (my_nex) atomicAdd(&p.st->nex, my_nex);
            if (my_changed) atomicOr(&p.st->changed, 1);
        }
    }
    if constexpr (DELTA) {
        // non-negative floats: their bit patterns order like the values
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mda = fmaxf(mda, __shfl_xor(mda, off, 64));
            mdr = fmaxf(mdr, __shfl_xor(mdr, off, 64));
        }
        if (lane == 0 && p.st != nullptr) {
            atomicMax(&p.st->d_a, __float_as_uint(mda));
            atomicMax(&p.st->d_r_next, __float_as_uint(mdr));
        }
    }
}

// Row pass for rows of any length: two sweeps over the row instead of
// holding it in registers.  Sweep 1 reads S, R_t, A_{t-1} chunk by chunk and
// forms A_t (written), the decision and the top-2 of A_t + S; after the
// workgroup reduction, sweep 2 reads S and R_t again and forms R_{t+1}
// (written) and the column partials, which accumulate in the workgroup's
// partial row in memory in row order (each thread owns its columns).  The
// per-chunk arithmetic is the register variant's, in the same order, so the
// results are bit-identical to it; 28 B per element and iteration instead
// of 20 (S and R_t are read twice), plus the partial row's update.  The
// first sweep's S and R_t loads are cached (the second sweep reads them
// again); everything else is streamed with the nontemporal hint.
template <int MODE>
__global__ __launch_bounds__(1024) void k_row_pass_2s(PassArgs p) {
#pragma clang fp contract(off)
    constexpr int T = 1024;
    constexpr bool DELTA = (MODE == PASS_FULL_DELTA);
    constexpr bool DO_A = (MODE == PASS_FULL || MODE == PASS_A_ONLY || DELTA);
    constexpr bool DO_R = (MODE != PASS_A_ONLY);
    constexpr bool LD_S = DO_R;
    constexpr bool LD_RA = (MODE != PASS_R_COLD);
    constexpr int NW = T / 64;

    if (p.st != nullptr && p.st->frozen) return;
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
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int c0 = tid * 4;
    // chunks of this thread that hold columns (j < Jn: c0 + 4 T j < n)
    const int Jn = c0 < n ? (n - c0 + 4 * T - 1) / (4 * T) : 0;

    float *P = p.partial + (int64_t)blockIdx.x * p.ldp;
    if constexpr (DO_R) {
        for (int j = 0; j < Jn; ++j) st4(P + c0 + j * T * 4, z4);
    }
    int my_nex = 0, my_changed = 0;
    float mda = 0.0f, mdr = 0.0f;

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const ColOwner dg = owner_of<T>(ii, tid);
        float *Arow = p.A + i * ld;
        const float *Rrow = p.Rin + i * ld;
        const float *Srow = p.S + i * ld;
        float ci = 0.0f;
        if constexpr (DO_A) ci = p.ccol[ii];
        float v1 = kNegInf, v2 = kNegInf, dv = kNegInf;
        int l1 = -1, dl = -1;
#pragma unroll 4
        for (int j = 0; j < Jn; ++j) {
            const int c = c0 + j * T * 4;
            const bool full = c + 3 < n;
            float4 a = z4, r = z4, sv = z4;
            if constexpr (LD_RA) {
                a = bld4(Arow, 0, c * 4);
                r = ld4(Rrow + c);
            }
            if constexpr (LD_S) sv = ld4(Srow + c);
            if constexpr (DO_A) {
                const float4 aold = a;
                chunk_avail(a, r, ld4(p.tcol + c), ci, j, dg, c, n, full, lam, oml, dv, dl);
                if (full) bst4(Arow, 0, c * 4, a);
                else
                    for (int e = 0; e < 4; ++e)
                        if (c + e < n) Arow[c + e] = f4get(a, e);
                if constexpr (DELTA) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (full || c + e < n) mda = fmaxf(mda, fabsf(f4get(a, e) - f4get(aold, e)));
                }
            }
            if constexpr (DO_R) (void)chunk_top2(a, r, sv, j, c, n, full, lam, oml, v1, l1, v2);
        }
        Top2 t2{v1, l1 < 0 ? INT32_MAX : local_to_col<T>(l1, tid), v2};
        ArgMax dm{dv, dl < 0 ? INT32_MAX : local_to_col<T>(dl, tid)};
        const int slot = (int)(i & 1);
        wg_reduce<NW, DO_A, DO_R>(t2, dm, sh_f[slot], sh_i[slot], lane, wave);
        if constexpr (DO_A) {
            if (tid == 0) note_decision(p, ii, dm.k, my_nex, my_changed);
        }
        if constexpr (DO_R) {
            const float m_other = oml * t2.v1;
            const float m_self = oml * t2.v2;
            const ColOwner ko = owner_of<T>(t2.k1, tid);
            float *Rout = p.Rout + i * ld;
#pragma unroll 4
            for (int j = 0; j < Jn; ++j) {
                const int c = c0 + j * T * 4;
                const bool full = c + 3 < n;
                float4 r = z4;
                if constexpr (LD_RA) r = bld4(Rrow, 0, c * 4);
                const float4 sv = bld4(Srow, 0, c * 4);
                // u = lambda r + (1 - lambda) s, as the first sweep's top-2 step forms it
                float4 u = z4;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (full || c + e < n) f4set(u, e, lam * f4get(r, e) + oml * f4get(sv, e));
                float4 rn;
                const float4 pos = chunk_resp(u, j, ko, dg, m_self, m_other, c, n, full, rn, p.rdiag + ii);
                if (full) bst4(Rout, 0, c * 4, rn);
                else
                    for (int e = 0; e < 4; ++e)
                        if (c + e < n) Rout[c + e] = f4get(rn, e);
                float4 acc = ld4(P + c);
                add4(acc, pos);
                st4(P + c, acc);
                if constexpr (DELTA) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (full || c + e < n) mdr = fmaxf(mdr, fabsf(f4get(rn, e) - f4get(r, e)));
                }
            }
        }
    }
    if constexpr (DO_A) {
        if (tid == 0 && p.st != nullptr) {
            if (my_nex) atomicAdd(&p.st->nex, my_nex);
            if (my_changed) atomicOr(&p.st->changed, 1);
        }
    }
    if constexpr (DELTA) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            mda = fmaxf(mda, __shfl_xor(mda, off, 64));
            mdr = fmaxf(mdr, __shfl_xor(mdr, off, 64));
        }
        if (lane == 0 && p.st != nullptr) {
            atomicMax(&p.st->d_a, __float_as_uint(mda));
            atomicMax(&p.st->d_r_next, __float_as_uint(mdr));
        }
    }
}

// alpha_t = 1 - lambda^t of the implicit responsibilities, from one function
// of t so every pass and the materialisation use the same rounding.
__device__ __forceinline__ float imp_alpha(float lam, int t) {
    return (float)(1.0 - pow((double)lam, (double)t));
}

// lambda^t of the block warm start, one function of t for every pass and
// the materialisation (the same rounding everywhere).
__device__ __forceinline__ float ia_lambda_pow(float lam, int t) {
    return t <= 0 ? 1.0f : (float)pow((double)lam, (double)t);
}

// Column sums: 64 columns per workgroup, 16 slices of the partial rows per
// column summed in FP64, slices combined in a fixed order.
__global__ __launch_bounds__(1024) void k_col_reduce(ColArgs a) {
#pragma clang fp contract(off)
    if (a.st != nullptr && a.st->frozen) return;
    __shared__ double part[16][64];
    const int cx = threadIdx.x & 63, gs = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + cx;
    // the column's own values, in flight with the partials
    float rd = 0.0f, ai = 0.0f, di = 0.0f;
    if (gs == 0 && k < a.n) {
        rd = a.rdiag[k];
        if (a.acol_out != nullptr) {
            ai = a.acol_in[k];
            di = a.adiag_in[k];
        }
    }
    double c = 0.0;
    if (k < a.n) {
        // eight partials in flight per step, summed in the same order
        int g = gs;
        for (; g + 7 * 16 < a.nparts; g += 8 * 16) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = a.partial[(int64_t)(g + u * 16) * a.ldp + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) c += (double)v[u];
        }
        for (; g < a.nparts; g += 16) c += (double)a.partial[(int64_t)g * a.ldp + k];
    }
    part[gs][cx] = c;
    __syncthreads();
    if (gs == 0 && k < a.n) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) tot += part[q][cx];
        const float tf = (float)((double)rd + tot), cf = (float)tot;
        a.tcol[k] = tf;
        a.ccol[k] = cf;
        if (a.acol_out != nullptr) {
            // the explicit update of Eqs. (3), (4) for elements with r <= 0, in its rounding
            const float oml = 1.0f - a.lam;
            a.acol_out[k] = a.lam * ai + oml * fminf(0.0f, tf);
            a.adiag_out[k] = a.lam * di + oml * cf;
        }
    }
    if (a.bookkeep && a.st != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
        ApState *st = a.st;
        const int t = st->iter + 1;
        const int same = (t > 1) && (st->changed == 0);
        // alphas of the implicit-R passes t+1 and t+2 (the pass just run was t)
        st->imp_al_prev = st->imp_al;
        st->imp_al = st->imp_al1;
        st->imp_al1 = st->imp_alpha_one ? 1.0f : imp_alpha(st->imp_lam, t + 2);
        const int run = same ? st->run + 1 : 1;
        st->iter = t;
        st->run = run;
        st->last_nex = st->nex;
        // message changes of iteration t: |A_t - A_{t-1}| from this pass,
        // |R_t - R_{t-1}| from the previous one
        const bool msg_stop = st->msg_on && t >= 2 &&
                              fmaxf(__uint_as_float(st->d_a), __uint_as_float(st->d_r)) <= st->msg_tol;
        st->d_r = st->d_r_next;
        st->d_r_next = 0u;
        st->d_a = 0u;
        if ((st->conv_iter > 0 && run >= st->conv_iter && st->nex > 0) || msg_stop) {
            st->converged = 1;
            st->frozen = 1;
        } else if (t >= st->max_iter) {
            st->frozen = 1;
        } else if (st->imp_abort) {
            st->frozen = 2;   // an implicit-R list overflowed: the host continues with explicit R
        }
        st->nex = 0;
        st->changed = 0;
    }
}

__global__ void k_state_init(ApState *st, int32_t max_iter, int32_t conv_iter, float lam, int msg_on,
                             float msg_tol, int alpha_one) {
    if (threadIdx.x == 0) {
        ApState s{};
        s.max_iter = max_iter;
        s.conv_iter = conv_iter;
        s.msg_on = msg_on;
        s.msg_tol = msg_tol;
        s.imp_lam = lam;
        s.imp_alpha_one = alpha_one;
        s.imp_al = alpha_one ? 1.0f : imp_alpha(lam, 1);
        s.imp_al1 = alpha_one ? 1.0f : imp_alpha(lam, 2);
        s.imp_al_prev = 0.0f;
        *st = s;
    }
}

// Column vectors of a column-structured A_0 (n >= 2): acol[k] = a_0(r,k)
// with r = 0 (r = 1 for k = 0), adiag[k] = a_0(k,k).
__global__ void k_extract_cols(const float *A, int64_t ld, int32_t n, float *acol, float *adiag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    acol[k] = A[(k == 0 ? ld : 0) + k];
    adiag[k] = A[(int64_t)k * ld + k];
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

// flag |= 1 when an entry of the rows x cols block (leading dimension ld) is
// NaN or infinite (exponent field all ones).
__global__ __launch_bounds__(256) void k_check_finite(const float *M, int64_t rows, int64_t cols, int64_t ld,
                                                      int32_t *flag) {
    uint32_t bad = 0u;
    for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
        const float *row = M + r * ld;
        for (int64_t c = threadIdx.x; c < cols; c += blockDim.x)
            bad |= (uint32_t)((__float_as_uint(row[c]) & 0x7f800000u) == 0x7f800000u);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// One wavefront per row: d_i = argmax_k a(i,k) + r(i,k) in FP32, lowest k
// on ties (the decision the row passes take).
__global__ __launch_bounds__(256) void k_decide(const float *A, const float *R, int64_t n, int64_t ld,
                                                int32_t *dec) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const float *ar = A + i * ld, *rr = R + i * ld;
    float bv = kNegInf;
    int bk = INT32_MAX;
    for (int64_t k = lane; k < n; k += 64) {
        const float v = ar[k] + rr[k];
        if (v > bv) {   // ascending k within a lane: a tie keeps the lower k
            bv = v;
            bk = (int)k;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const float ov = __shfl_xor(bv, off, 64);
        const int ok = __shfl_xor(bk, off, 64);
        if (ov > bv || (ov == bv && ok < bk)) {
            bv = ov;
            bk = ok;
        }
    }
    if (lane == 0) dec[i] = bk;
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
    const int64_t i = a.row0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= (a.row1 > 0 ? a.row1 : a.n)) return;
    const int m = *a.nex;
    const float *Srow = a.S + i * a.ld;
    double dp = 0.0, ep = 0.0;
    int lab;
    if (a.raw != nullptr) {
        // raw decisions as labels: exemplars (d_i = i) add s(i,i) to expref
        lab = a.raw[i];
        if (lab == (int)i) ep = (double)Srow[i];
        else dp = (double)Srow[lab];
    } else if (m == 0) {
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

template <int T, int J, int MODE>
hipError_t launch_lds(const PassArgs &a, int grid, size_t lds, hipStream_t s) {
    static bool attr_set = false;   // per process; the attribute is per function
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_row_pass<T, J, MODE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    k_row_pass<T, J, MODE><<<grid, T, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_2s(int mode, const PassArgs &a, int grid, hipStream_t s) {
    switch (mode) {
    case PASS_FULL_DELTA: k_row_pass_2s<PASS_FULL_DELTA><<<grid, 1024, 0, s>>>(a); break;
    case PASS_FULL: k_row_pass_2s<PASS_FULL><<<grid, 1024, 0, s>>>(a); break;
    case PASS_R_ONLY: k_row_pass_2s<PASS_R_ONLY><<<grid, 1024, 0, s>>>(a); break;
    case PASS_R_COLD: k_row_pass_2s<PASS_R_COLD><<<grid, 1024, 0, s>>>(a); break;
    default: k_row_pass_2s<PASS_A_ONLY><<<grid, 1024, 0, s>>>(a); break;
    }
    return hipGetLastError();
}

template <int T, int J>
hipError_t launch_t(int mode, const PassArgs &a, const PassPlan &pl, hipStream_t s) {
    if (mode == PASS_FULL_DELTA) {
        // register variant only (keeps R_t of the row for the change)
        k_row_pass_reg<T, J, PASS_FULL_DELTA><<<pl.grid, T, 0, s>>>(a);
        return hipGetLastError();
    }
    if (pl.lds_bytes > 0) {
        switch (mode) {
        case PASS_FULL: return launch_lds<T, J, PASS_FULL>(a, pl.grid, pl.lds_bytes, s);
        case PASS_R_ONLY: return launch_lds<T, J, PASS_R_ONLY>(a, pl.grid, pl.lds_bytes, s);
        case PASS_R_COLD: return launch_lds<T, J, PASS_R_COLD>(a, pl.grid, pl.lds_bytes, s);
        default: return launch_lds<T, J, PASS_A_ONLY>(a, pl.grid, pl.lds_bytes, s);
        }
    }
    switch (mode) {
    case PASS_FULL: k_row_pass_reg<T, J, PASS_FULL><<<pl.grid, T, 0, s>>>(a); break;
    case PASS_R_ONLY: k_row_pass_reg<T, J, PASS_R_ONLY><<<pl.grid, T, 0, s>>>(a); break;
    case PASS_R_COLD: k_row_pass_reg<T, J, PASS_R_COLD><<<pl.grid, T, 0, s>>>(a); break;
    default: k_row_pass_reg<T, J, PASS_A_ONLY><<<pl.grid, T, 0, s>>>(a); break;
    }
    return hipGetLastError();
}


// ---- implicit responsibilities ---------------------------------------------
// R_t(i,k) = alpha_t s(i,k) - beta_t(i) off the row's list, and the stored
// value r_t(i,k) (updated by the explicit damped Eq. (2)) on it; see
// ImpArgs.  A pass reads S and A and writes A (12 bytes per element instead
// of 20); R is rebuilt in registers from the row's state.  alpha_t,
// alpha_{t+1} are read from the run state, so the partials formed for
// R_{t+1} in pass t and the values pass t+1 rebuilds use the same numbers.

template <int T, int J, int KIND, bool PREF>
__global__ __launch_bounds__(T) void k_row_imp(ImpArgs p) {
#pragma clang fp contract(off)
    constexpr bool DO_A = (KIND == IMP_FULL);
    constexpr bool LD_A = (KIND != IMP_PRO_COLD);
    constexpr int NW = T / 64;
    constexpr int NOWN = 2;                      // listed columns a thread keeps in registers

    if (p.st != nullptr && p.st->frozen) return;
    __shared__ float sh_f[2][NW][3];
    __shared__ int sh_i[2][NW][2];
    // Row state, three slots: the state of row i+1 is staged during row i
    // before the reduction barrier, which orders it before its use; the slot
    // it overwrites was last read in row i-2, before row i-1's barrier.
    __shared__ int st_col[3][IMP_K];
    __shared__ float st_gam[3][IMP_K];
    __shared__ float st_beta[3];
    __shared__ int st_cnt[3];
    __shared__ float st_ci[3];
    extern __shared__ float4 dyn[];
    const int q = (p.n + 3) >> 2;
    float4 *lpart = dyn;                         // column partials, q entries
    float4 *ls = dyn + q;                        // S of the current row (PREF), q entries
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
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int voff = tid * 16;
    const int c0 = tid * 4;
    const int cl = ((J - 1) * T + tid) * 4;
    const bool last_in = cl < n;
    const bool last_full = cl + 3 < n;
    // alpha_t, alpha_{t+1} and the iteration come from the run state (kept
    // there by the column reduce), so replays of a captured pass stay valid.
    const int tpass = p.prologue ? 0 : p.st->iter + 1;
    const float al = p.prologue ? 0.0f : p.st->imp_al;       // alpha_t
    const float al1 = p.prologue ? p.st->imp_al : p.st->imp_al1;  // alpha_{t+1}
    const ImpLayout L = imp_layout(n);
    const char *sin = p.state + (int64_t)(tpass & 1) * p.stride;
    char *sout = p.state + (int64_t)((tpass + 1) & 1) * p.stride;
    const float *beta_in = reinterpret_cast<const float *>(sin + L.beta);
    const int32_t *cnt_in = reinterpret_cast<const int32_t *>(sin + L.cnt);
    const int32_t *col_in = reinterpret_cast<const int32_t *>(sin + L.col);
    const float *gam_in = reinterpret_cast<const float *>(sin + L.gam);
    float *beta_out = reinterpret_cast<float *>(sout + L.beta);
    int32_t *cnt_out = reinterpret_cast<int32_t *>(sout + L.cnt);
    int32_t *col_out = reinterpret_cast<int32_t *>(sout + L.col);
    float *gam_out = reinterpret_cast<float *>(sout + L.gam);
    float *const Rx_base = p.Rx[(tpass + 1) & 1];

#pragma unroll
    for (int j = 0; j < J; ++j)
        if (j < J - 1 || last_in) lpart[j * T + tid] = z4;
    int my_nex = 0, my_changed = 0;

    // Row state is fetched into a register one row ahead (by threads
    // 0..2K+2) and written to its LDS slot later, so the loads overlap a row.
    auto fetch_state = [&](int64_t i) -> uint32_t {
        if (tid < IMP_K) return (uint32_t)col_in[i * IMP_K + tid];
        if (tid < 2 * IMP_K) return __float_as_uint(gam_in[i * IMP_K + tid - IMP_K]);
        if (tid == 2 * IMP_K) return __float_as_uint(beta_in[i]);
        if (tid == 2 * IMP_K + 1) return (uint32_t)cnt_in[i];
        if (tid == 2 * IMP_K + 2 && DO_A) return __float_as_uint(p.ccol[i]);
        return 0u;
    };
    auto put_state = [&](int64_t i, uint32_t v) {
        const int sl = (int)(i % 3);
        if (tid < IMP_K) st_col[sl][tid] = (int)v;
        else if (tid < 2 * IMP_K) st_gam[sl][tid - IMP_K] = __uint_as_float(v);
        else if (tid == 2 * IMP_K) st_beta[sl] = __uint_as_float(v);
        else if (tid == 2 * IMP_K + 1) st_cnt[sl] = (int)v;
        else if (tid == 2 * IMP_K + 2) st_ci[sl] = __uint_as_float(v);
    };
    // The prefetching variant holds the next row's S and A in registers; the
    // other (long rows) holds only S and reads A chunk by chunk.
    float4 s4[J], a4[(LD_A && PREF) ? J : 1];
    auto load_row = [&](int64_t i) {
        const rsrc_t srs = row_rsrc(p.S + i * ld, ld);
        const rsrc_t ars = row_rsrc(p.A + i * ld, ld);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (j < J - 1 || last_in) {
                s4[j] = bld4(srs, voff, j * T * 16);
                if constexpr (LD_A && PREF) a4[j] = bld4(ars, voff, j * T * 16);
            }
        }
    };
    if (r0 < r1) {
        put_state(r0, fetch_state(r0));
        load_row(r0);
    }
    __syncthreads();

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const int sl = (int)(i % 3);
        const ColOwner dg = owner_of<T>(ii, tid);
        const int dle = dg.mine ? 4 * dg.j + dg.e : -1;     // local index of the diagonal
        const bool wave_diag = __any(dg.mine);
        float *Arow = p.A + i * ld;
        const rsrc_t a_rs = row_rsrc(Arow, ld);
        // state of R_t for this row; the listed columns this thread owns go
        // to registers (local index 4*chunk + element, stored r_t, list slot)
        const float beta = st_beta[sl];
        const int cnt = st_cnt[sl];
        uint32_t next_state = 0u;
        if constexpr (PREF) next_state = (i + 1 < r1) ? fetch_state(i + 1) : 0u;
        int own_le[NOWN], own_q[NOWN];
        float own_g[NOWN];
#pragma unroll
        for (int o = 0; o < NOWN; ++o) {
            own_le[o] = -1;
            own_q[o] = -1;
            own_g[o] = 0.0f;
        }
        int nown = 0;
        for (int qq = 0; qq < cnt; ++qq) {
            const int c = st_col[sl][qq];
            if (((c >> 2) % T) == tid) {
                const int le = ((c >> 2) / T) * 4 + (c & 3);
#pragma unroll
                for (int o = 0; o < NOWN; ++o) {
                    const bool put = nown == o;
                    own_le[o] = put ? le : own_le[o];
                    own_q[o] = put ? qq : own_q[o];
                    own_g[o] = put ? st_gam[sl][qq] : own_g[o];
                }
                ++nown;
            }
        }
        const bool wave_own = __any(nown > 0);
        float ci = 0.0f;
        if constexpr (DO_A) ci = st_ci[sl];
        float v1 = kNegInf, v2 = kNegInf, dv = kNegInf;
        int l1 = -1, dl = -1;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (!(j < J - 1 || last_in)) continue;
            const bool full = (j < J - 1) || last_full;
            const int c = c0 + j * T * 4;
            const float4 sv = s4[j];
            float4 a = z4;
            if constexpr (LD_A) {
                if constexpr (PREF) a = a4[j];
                else a = bld4(a_rs, voff, j * T * 16);
            }
            float4 r;
#pragma unroll
            for (int e = 0; e < 4; ++e) f4set(r, e, al * f4get(sv, e) - beta);
            if (wave_own) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int o = 0; o < NOWN; ++o)
                        if (own_le[o] == 4 * j + e) f4set(r, e, own_g[o]);
            }
            if constexpr (DO_A) {
                const float4 tv = ld4(p.tcol + c);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (full || c + e < n) {
                        float upd = fminf(0.0f, f4get(tv, e) - fmaxf(0.0f, f4get(r, e)));
                        if (wave_diag && dle == 4 * j + e) upd = ci;
                        const float an = lam * f4get(a, e) + oml * upd;
                        f4set(a, e, an);
                        const float v = an + f4get(r, e);
                        const bool gt = v > dv;
                        dl = gt ? 4 * j + e : dl;
                        dv = gt ? v : dv;
                    }
                }
                store_chunk(Arow, a_rs, voff, j * T * 16, c, n, full, a);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (full || c + e < n) {
                    const float v = f4get(a, e) + f4get(sv, e);
                    const bool gt = v > v1;
                    v2 = gt ? v1 : fmaxf(v2, v);
                    l1 = gt ? 4 * j + e : l1;
                    v1 = gt ? v : v1;
                }
            }
            if constexpr (PREF) ls[j * T + tid] = sv;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < r1) {
            if constexpr (PREF) {
                put_state(i + 1, next_state);
                load_row(i + 1);
            } else {
                put_state(i + 1, fetch_state(i + 1));
            }
        }
        __builtin_amdgcn_sched_barrier(0);

        Top2 t2{v1, l1 < 0 ? INT32_MAX : local_to_col<T>(l1, tid), v2};
        ArgMax dm{dv, dl < 0 ? INT32_MAX : local_to_col<T>(dl, tid)};
        wg_reduce<NW, DO_A, true>(t2, dm, sh_f[i & 1], sh_i[i & 1], lane, wave);
        if constexpr (DO_A) {
            if (tid == 0) {
                const int k = dm.k;
                if (p.dec) p.dec[ii] = k;
                if (p.eflag) {
                    const uint8_t ef = (uint8_t)(k == ii);
                    if (p.eflag[ii] != ef) my_changed = 1;
                    p.eflag[ii] = ef;
                    my_nex += ef;
                }
            }
        }

        // State of R_{t+1}: beta' = lam beta + (1-lam) v1 for the columns off
        // the list; on it (and for k1, which joins it) the damped Eq. (2),
        // r' = (lam r + (1-lam) s) - (1-lam) (k = k1 ? v2 : v1), in the
        // explicit pass's rounding.  Keeping r itself on the list, not an
        // offset from alpha s - beta, avoids the cancellation of two large
        // terms in rows whose argmax column has a large availability.
        const int k1 = t2.k1;
        const float m_other = oml * t2.v1, m_self = oml * t2.v2;
        const float beta1 = lam * beta + oml * t2.v1;
        // A new column k1 overflows the row when the list is full or when the
        // thread owning k1 already keeps NOWN listed columns (every thread
        // evaluates the same test, so the decision is uniform).
        int pos1 = -1, k1_owner_has = 0;
        const int k1_owner = (k1 >> 2) % T;
        for (int qq = 0; qq < cnt; ++qq) {
            const int c = st_col[sl][qq];
            pos1 = (c == k1) ? qq : pos1;
            k1_owner_has += (((c >> 2) % T) == k1_owner) ? 1 : 0;
        }
        const bool ovf = pos1 < 0 && (cnt >= p.kmax || k1_owner_has >= NOWN);
        if (tid == 0) {
            beta_out[ii] = beta1;
            if (ovf) {
                cnt_out[ii] = -1;
                atomicOr(&p.st->imp_abort, cnt >= p.kmax ? 1 : 4);
            } else {
                for (int qq = 0; qq < cnt; ++qq) col_out[(int64_t)ii * IMP_K + qq] = st_col[sl][qq];
                if (pos1 < 0) col_out[(int64_t)ii * IMP_K + cnt] = k1;
                cnt_out[ii] = cnt + (pos1 < 0 ? 1 : 0);
            }
        }
        // r_{t+1} of the listed columns (and of k1 when it joins), formed by
        // their owners in the loop below and stored in the new list
        float own_r1[NOWN];
#pragma unroll
        for (int o = 0; o < NOWN; ++o) own_r1[o] = 0.0f;
        float k1_r1 = 0.0f;
        const bool k1_mine = pos1 < 0 && k1_owner == tid;
        const int k1_le = ((k1 >> 2) / T) * 4 + (k1 & 3);
        const bool wave_k1 = __any(k1_mine);

        // Column partials of max(0, R_{t+1}); on overflow the row of R_{t+1}
        // is also written explicitly.
        float *Rx = Rx_base + i * ld;
        const rsrc_t x_rs = row_rsrc(Rx, ld);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (!(j < J - 1 || last_in)) continue;
            const bool full = (j < J - 1) || last_full;
            const int c = c0 + j * T * 4;
            float4 sv;
            if constexpr (PREF) sv = ls[j * T + tid];
            else sv = s4[j];
            float4 rv4;
#pragma unroll
            for (int e = 0; e < 4; ++e) f4set(rv4, e, al1 * f4get(sv, e) - beta1);
            if (wave_k1) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (k1_mine && k1_le == 4 * j + e) {
                        // r_t = alpha_t s - beta (k1 was off the list)
                        const float s = f4get(sv, e);
                        k1_r1 = (lam * (al * s - beta) + oml * s) - m_self;
                        f4set(rv4, e, k1_r1);
                    }
            }
            if (wave_own) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int o = 0; o < NOWN; ++o)
                        if (own_le[o] == 4 * j + e) {
                            own_r1[o] = (lam * own_g[o] + oml * f4get(sv, e)) - (own_q[o] == pos1 ? m_self : m_other);
                            f4set(rv4, e, own_r1[o]);
                        }
            }
            float4 pos;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                f4set(pos, e, (full || c + e < n) ? fmaxf(0.0f, f4get(rv4, e)) : 0.0f);
            if (wave_diag) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (dle == 4 * j + e) {
                        f4set(pos, e, 0.0f);
                        p.rdiag[ii] = f4get(rv4, e);
                    }
            }
            float4 acc = lpart[j * T + tid];
            add4(acc, pos);
            lpart[j * T + tid] = acc;
        }
        if (!ovf) {
#pragma unroll
            for (int o = 0; o < NOWN; ++o)
                if (own_q[o] >= 0) gam_out[(int64_t)ii * IMP_K + own_q[o]] = own_r1[o];
            if (k1_mine) gam_out[(int64_t)ii * IMP_K + cnt] = k1_r1;
        }
        if (ovf) {
            // the overflowing row of R_{t+1}, written explicitly (same values)
#pragma unroll
            for (int j = 0; j < J; ++j) {
                if (!(j < J - 1 || last_in)) continue;
                const bool full = (j < J - 1) || last_full;
                const int c = c0 + j * T * 4;
                float4 sv;
                if constexpr (PREF) sv = ls[j * T + tid];
                else sv = s4[j];
                float4 rn;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float rv = al1 * f4get(sv, e) - beta1;
                    if (k1_mine && k1_le == 4 * j + e) rv = k1_r1;
#pragma unroll
                    for (int o = 0; o < NOWN; ++o)
                        if (own_le[o] == 4 * j + e) rv = own_r1[o];
                    f4set(rn, e, rv);
                }
                store_chunk(Rx, x_rs, voff, j * T * 16, c, n, full, rn);
            }
        }
        if constexpr (!PREF) {
            if (i + 1 < r1) load_row(i + 1);
        }
    }

    {
        float *P = p.partial + (p.part0 + (int64_t)blockIdx.x) * p.ldp;
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < J - 1 || last_in) st4(P + c0 + j * T * 4, lpart[j * T + tid]);
    }
    if constexpr (DO_A) {
        if (tid == 0 && p.st != nullptr) {
            if (my_nex) atomicAdd(&p.st->nex, my_nex);
            if (my_changed) atomicOr(&p.st->changed, 1);
        }
    }
}

// ---- implicit availabilities -----------------------------------------------
// Pass t with R_t implicit (as in k_row_imp) and A_{t-1} implicit (see
// XLayout): it reads S and short per-row lists and writes no matrix.
// The row scan covers the ordinary elements: off-diagonal, not in the row's
// exception list, not in its R list, responsibility not positive.  Their
// availability is acol_t(k) and R_t has no gamma term there, so the scan is
// a few instructions per element.  Every other element is merged after the
// scan, with its column index, by the thread holding it:
//   - exception-list entries by their list holder (update from the stored
//     value, Eq. (3) with damping),
//   - R-list entries by their holder, lane q of wavefront 0 for entry q,
//   - the diagonal (adiag_t(i)) by thread 0,
//   - first positive responsibilities by the column owner (update from
//     acol_{t-1}(k), exactly what the explicit update gives a never-positive
//     element; appended to the list).
// Holders gather their S values at the start of the row, so the row
// registers are free after the scan and the next row's S is loaded before
// the reduction.  The column partials of max(0, R_{t+1}) take one addition
// per row and column, in row order, by the same holders; ordinary elements
// are reread (from L2) only by threads whose largest ordinary s can give a
// positive value (al1 s - beta1 is monotone in s).
// Each row has an LDS byte mask (one byte per float4 chunk): bit e marks an
// exception-list column, bit 4+e an R-listed column or the diagonal.  NXS
// slots: row i+1's bits are set during row i before the reduction barrier,
// and each thread zeroes its own bytes of row i-1's slot after it, two
// barriers before the slot is set again.
// GP: the partials accumulate in the workgroup's global partial row (rows too
// long for LDS), added by the same threads; the reduction barrier orders LDS
// only, so a wavefront that added to them releases its stores before the
// next row's barrier (a wait for its outstanding memory operations, which
// by then are the next row's S, needed by the scan anyway) and every
// wavefront acquires after it.
constexpr int NXS = 4;
constexpr int kMaxDynLdsIa = 160 * 1024 - 4 * 1024;


__device__ __forceinline__ uint32_t xbit(int k) { return 1u << ((((k >> 2) & 3) << 3) + (k & 3)); }

// max(a, b) as one med3 (no canonicalisation of the operands; no NaNs here).
// max(a, b) for a, b below +inf (finite values and the -inf sentinel): one
// v_med3 against the largest finite float, which needs no NaN quieting of
// its inputs (a max against +inf is folded into a canonicalising max)
__device__ __forceinline__ float max3f(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 3.40282347e+38f); }

// Neighbouring floats of x (x not NaN; -inf steps up to -FLT_MAX).
__device__ __forceinline__ float f_up(float x) {
    if (x == 0.0f) return __int_as_float(1);
    const int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b + 1 : b - 1);
}
__device__ __forceinline__ float f_down(float x) {
    if (x == 0.0f) return -__int_as_float(1);
    const int b = __float_as_int(x);
    return __int_as_float(x > 0.0f ? b - 1 : b + 1);
}
// The largest float sth with fl(al sth) <= beta.  The off-list value
// fl(fl(al s) - beta) is positive exactly when fl(al s) > beta (with gradual
// underflow a difference of two floats is zero only when they are equal),
// and fl(al s) is monotone in s, so r > 0 iff s > sth.  beta / al is within
// an ulp or two of the boundary; the walk ends on it and the result is
// certified, else NaN (al <= 0, overflow), and the row forms r itself.
__device__ float pos_threshold(float al, float beta) {
#pragma clang fp contract(off)
    float x = beta / al;
    for (int k = 0; k < 4 && al * x > beta; ++k) x = f_down(x);
    for (int k = 0; k < 4 && !(al * f_up(x) > beta); ++k) x = f_up(x);
    return (al * x <= beta && al * f_up(x) > beta) ? x : __int_as_float(0x7FC00000);
}

// DPP lane moves; lanes a row mask leaves out keep the identity of the
// reduction (-inf for max, INT32_MAX for min), so an integer min fuses the
// move into one v_min_i32_dpp
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ float dpp_f(float x) {
    if constexpr (RM == 0xF)   // every lane written: no identity to load
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
    else
        return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(-INFINITY), __float_as_int(x), CTRL, RM, 0xF, false));
}
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dpp_i(int x) {
    return __builtin_amdgcn_update_dpp(INT32_MAX, x, CTRL, RM, 0xF, false);
}

template <int CTRL, int RM = 0xF>
__device__ __forceinline__ float dmax(float x) { return max3f(x, dpp_f<CTRL, RM>(x)); }
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dmin(int x) { return min(x, dpp_i<CTRL, RM>(x)); }
// max / min over each 16-lane row (every lane of the row gets it): quad
// swaps, then half-row and row mirrors
__device__ __forceinline__ float row_max(float x) {
    return dmax<0x140>(dmax<0x141>(dmax<0x4E>(dmax<0xB1>(x))));
}
__device__ __forceinline__ int row_min(int x) {
    return dmin<0x140>(dmin<0x141>(dmin<0x4E>(dmin<0xB1>(x))));
}
// over the wavefront: rows, then row broadcasts of lane 15 (into rows 1, 3)
// and lane 31 (into rows 2, 3); lane 63 holds the result
__device__ __forceinline__ float wave_max(float x) {
    x = dmax<0x143, 0xC>(dmax<0x142, 0xA>(row_max(x)));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
__device__ __forceinline__ int wave_min(int x) {
    x = dmin<0x143, 0xC>(dmin<0x142, 0xA>(row_min(x)));
    return __builtin_amdgcn_readlane(x, 63);
}
// bucket of an R-listed column in a row's 64-entry hash table
__device__ __forceinline__ int rl_hash(int c) { return (int)(((uint32_t)c * 2654435761u) >> 26); }

// Order-preserving integer key of a float that is finite or -inf (-0 is
// taken as +0 first, so keys are equal exactly when the floats are equal):
// integer max and min fuse their DPP lane moves, float max does not.
__device__ __forceinline__ int okey(float x) {
    const int b = __float_as_int(x + 0.0f);
    return b ^ ((b >> 31) & 0x7FFFFFFF);
}
__device__ __forceinline__ float okey_f(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7FFFFFFF)); }
template <int CTRL, int RM = 0xF>
__device__ __forceinline__ int dmaxi(int x) {
    return max(x, __builtin_amdgcn_update_dpp(INT32_MIN, x, CTRL, RM, 0xF, false));
}
__device__ __forceinline__ int row_maxi(int x) {
    return dmaxi<0x140>(dmaxi<0x141>(dmaxi<0x4E>(dmaxi<0xB1>(x))));
}
__device__ __forceinline__ int wave_maxi(int x) {
    x = dmaxi<0x143, 0xC>(dmaxi<0x142, 0xA>(row_maxi(x)));
    return __builtin_amdgcn_readlane(x, 63);
}

// Workgroup top-2 of a+s from each lane's (v1, k1, v2), in three passes
// that need no merge order: the largest v1, the lowest column reaching it,
// and the largest of the winner's v2 and every other lane's v1 (a candidate
// column is held by one lane only).  Each 16-lane row reduces with DPP and
// writes one LDS slot (4 per wavefront); after the barrier every wavefront
// reduces the 4*NW slots, one per lane.  The values travel as okey keys.
template <int NW>
__device__ __forceinline__ void wg_top2(Top2 &t, int (*sh_v)[2], int *sh_i, int lane, int wave) {
    static_assert(4 * NW <= 64, "one slot per lane");
    {
        const int a1 = okey(t.v1), a2 = okey(t.v2);
        const int V = row_maxi(a1);
        const int K = row_min(a1 == V ? t.k1 : INT32_MAX);
        const int V2 = row_maxi(a1 == V && t.k1 == K ? a2 : a1);
        if ((lane & 15) == 0) {
            const int slot = wave * 4 + (lane >> 4);
            sh_v[slot][0] = V;
            sh_v[slot][1] = V2;
            sh_i[slot] = K;
        }
    }
    lds_barrier();
    const bool has = lane < 4 * NW;
    const int v1 = has ? sh_v[lane][0] : INT32_MIN;
    const int k1 = has ? sh_i[lane] : INT32_MAX;
    const int v2 = has ? sh_v[lane][1] : INT32_MIN;
    const int V = wave_maxi(v1);
    const int K = wave_min(v1 == V ? k1 : INT32_MAX);
    const int V2 = wave_maxi(v1 == V && k1 == K ? v2 : v1);
    t = Top2{okey_f(V), K, okey_f(V2)};
}

template <int T, int J, bool GP, bool WB>
__global__ __launch_bounds__(T) void k_row_ia(ImpArgs p) {
#pragma clang fp contract(off)
    constexpr int NW = T / 64;
    constexpr int NOWN = 2;                      // listed columns per owner in k_row_imp
    constexpr int EPT = (IMP_KA + T - 1) / T;    // exception-list entries per thread
    static_assert(IMP_K <= 64, "R-list holders are lanes of wavefront 0");
    // Lean scan (no block term): the ordinary columns' part of the exemplar
    // decision is left out of the scan.  It can change the decision only when
    // no listed, new or special column beats the diagonal and D = a(i,i) +
    // r(i,i) <= 0 (an ordinary a + r is a sum of two values <= 0 when every
    // column value is), and such rows are scanned again after the reduction.
    constexpr bool LEAN = !WB;

    if (p.st->frozen) return;
    __shared__ int sh_v[2][4 * NW][2];
    __shared__ int sh_i[2][4 * NW];
    __shared__ __align__(16) int st_col[3][IMP_K];
    __shared__ int st_hash[3][64];               // R-listed column -> list position
    __shared__ float st_gam[3][IMP_K];
    __shared__ float st_beta[3];
    __shared__ float st_sth[3];                  // r = al s - beta > 0 iff s > st_sth (NaN: not certified)
    __shared__ int st_cnt[3];
    __shared__ float st_ad[3];
    __shared__ float st_sd[3];                   // s(i,i)
    __shared__ float st_gd[3];                   // gamma(i,i) when R-listed ...
    __shared__ int st_gdr[3];                    // ... for the row stored here
    __shared__ int xa_new[NXS];
    __shared__ int dec_fail[NXS];                // a column beats the diagonal
    extern __shared__ float4 dyn[];
    const int q = (p.n + 3) >> 2;
    const int mw = (q + 3) >> 2;                 // mask words per slot
    float4 *lpart = dyn;                         // column partials (LDS variant), q entries
    float *lp = reinterpret_cast<float *>(dyn);  // the same, indexed by column
    uint32_t *mask = reinterpret_cast<uint32_t *>(dyn + (GP ? 0 : q));
    uint8_t *mask8 = reinterpret_cast<uint8_t *>(mask);
    int *rcnt = reinterpret_cast<int *>(mask + NXS * mw);   // list lengths of this workgroup's rows
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
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int c0 = tid * 4;
    const int cl = ((J - 1) * T + tid) * 4;
    const bool last_in = cl < n;
    const bool last_full = cl + 3 < n;
    // mask bits of the last chunk's columns at or beyond n (both nibbles)
    const uint32_t oob_bits = last_full ? 0u : (0x11u * ((0xFu << (n - cl > 0 ? n - cl : 0)) & 0xFu)) & 0xFFu;
    const int tpass = p.st->iter + 1;
    const float al = p.st->imp_al;               // alpha_t
    const float al1 = p.st->imp_al1;             // alpha_{t+1}
    // block warm start: lambda^t and lambda^(t-1) (A_t and A_{t-1} of
    // never-positive elements: acol + lambda^t a_0)
    const float lt = WB ? ia_lambda_pow(lam, tpass) : 0.0f;
    const float ltp = WB ? ia_lambda_pow(lam, tpass - 1) : 0.0f;
    const ImpLayout L = imp_layout(n);
    const char *sin = p.state + (int64_t)(tpass & 1) * p.stride;
    char *sout = p.state + (int64_t)((tpass + 1) & 1) * p.stride;
    const float *beta_in = reinterpret_cast<const float *>(sin + L.beta);
    const int32_t *cnt_in = reinterpret_cast<const int32_t *>(sin + L.cnt);
    const int32_t *col_in = reinterpret_cast<const int32_t *>(sin + L.col);
    const float *gam_in = reinterpret_cast<const float *>(sin + L.gam);
    float *beta_out = reinterpret_cast<float *>(sout + L.beta);
    int32_t *cnt_out = reinterpret_cast<int32_t *>(sout + L.cnt);
    int32_t *col_out = reinterpret_cast<int32_t *>(sout + L.col);
    float *gam_out = reinterpret_cast<float *>(sout + L.gam);
    float *const Rx_base = p.Rx[(tpass + 1) & 1];
    const XLayout X = x_layout(n);
    const char *xin = p.xstate + (int64_t)((tpass + 1) & 1) * p.xstride;   // lists of A_{t-1}
    char *xout = p.xstate + (int64_t)(tpass & 1) * p.xstride;             // lists of A_t
    const int32_t *xcnt_in = reinterpret_cast<const int32_t *>(xin + X.cnt);
    const int32_t *xcol_in = reinterpret_cast<const int32_t *>(xin + X.col);
    const float *xval_in = reinterpret_cast<const float *>(xin + X.val);
    int32_t *xcnt_out = reinterpret_cast<int32_t *>(xout + X.cnt);
    int32_t *xcol_out = reinterpret_cast<int32_t *>(xout + X.col);
    float *xval_out = reinterpret_cast<float *>(xout + X.val);
    const float *acol_t = p.acol[tpass & 1];
    const float *acol_p = p.acol[(tpass + 1) & 1];
    const float *adiag_t = p.adiag[tpass & 1];
    const int xcap = p.xcap;
    float *P = p.partial + (p.part0 + (int64_t)blockIdx.x) * p.ldp;

#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (j < J - 1 || last_in) {
            if constexpr (GP) st4(P + c0 + j * T * 4, z4);
            else lpart[j * T + tid] = z4;
        }
    }
    for (int w = tid; w < NXS * mw; w += T) mask[w] = 0u;
    for (int64_t r = r0 + tid; r < r1; r += T) {
        const int c = xcnt_in[r];
        rcnt[r - r0] = c < 0 ? 0 : (c > IMP_KA ? IMP_KA : c);
    }
    if (tid < 3) st_gdr[tid] = -1;
    int my_nex = 0, my_changed = 0;
    __syncthreads();

    // The next row's R state is fetched and staged by wavefront SW (on
    // another SIMD than wavefront 0, which holds the R list, and the
    // wavefronts that hold the exception lists' first entries): one word per
    // lane: list columns, gammas, beta, count, a(i,i), s(i,i)
    constexpr int SW = 3;
    static_assert(NW > SW, "state wavefront");
    const bool sw = wave == SW;
    // (list words by byte offsets from the state buffer, whose size is far
    // below 4 GB; a(i,i) and s(i,i) are uniform loads, used at the put)
    struct RowState { uint32_t v; float ad, sd; };
    auto fetch_state = [&](int64_t i) -> RowState {
        RowState r{0u, 0.0f, 0.0f};
        if (!sw) return r;
        if (lane < 2 * IMP_K + 2) {
            const uint32_t ri = (uint32_t)i;
            const uint32_t off = lane < 2 * IMP_K
                ? (uint32_t)(lane < IMP_K ? L.col : L.gam) + (ri * IMP_K + (lane & (IMP_K - 1))) * 4u
                : (uint32_t)(lane == 2 * IMP_K ? L.beta : L.cnt) + ri * 4u;
            r.v = *reinterpret_cast<const uint32_t *>(sin + off);
        }
        r.ad = adiag_t[i];
        r.sd = p.S[i * ld + i];
        return r;
    };
    // R state of row i into its LDS slot; the R-listed columns and the
    // diagonal are marked in the high nibble of the row's mask bytes
    auto put_state = [&](int64_t i, const RowState &rs, int rc, float rgam) {
        if (!sw) return;
        const uint32_t v = rs.v;
        const int sl = (int)(i % 3);
        uint32_t *m = mask + (i % NXS) * mw;
        // the slot's hash table is empty before the inserts (one wavefront:
        // its LDS operations are ordered)
        st_hash[sl][lane] = -1;
        if (lane < IMP_K) {
            st_col[sl][lane] = (int)v;
            const int c = (int)v;
            if (lane < rc && (unsigned)c < (unsigned)n) {
                atomicOr(&m[c >> 4], xbit(c) << 4);
                // open addressing, at most IMP_K entries in 64 buckets
                int h = rl_hash(c);
                while (atomicCAS(&st_hash[sl][h], -1, c * IMP_K + lane) != -1) h = (h + 1) & 63;
            }
            if (lane < rc && c == (int)i) {
                st_gd[sl] = rgam;
                st_gdr[sl] = (int)i;
            }
        } else if (lane < 2 * IMP_K) {
            st_gam[sl][lane - IMP_K] = __uint_as_float(v);
        } else if (lane == 2 * IMP_K) {
            st_beta[sl] = __uint_as_float(v);
            st_sth[sl] = (LEAN && p.lean) ? pos_threshold(al, __uint_as_float(v)) : __int_as_float(0x7FC00000);
        } else if (lane == 2 * IMP_K + 1) {
            st_cnt[sl] = (int)v;
        } else if (lane == 2 * IMP_K + 2) {
            st_ad[sl] = rs.ad;
        } else if (lane == 2 * IMP_K + 3) {
            st_sd[sl] = rs.sd;
        }
        if (lane == 0) atomicOr(&m[i >> 4], xbit((int)i) << 4);
    };
    // Exception list of a row: thread tid holds entries xq0 + u*T in
    // registers (column -1 when absent); the first entries go to wavefronts
    // 1.. so that wavefront 0, which holds the R list, does not hold them too
    const int xq0 = (tid + T - 64) % T;
    auto fetch_x = [&](int64_t i, int *xc, float *xv) {
        const int len = rcnt[i - r0];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int qx = xq0 + u * T;
            xc[u] = -1;
            xv[u] = 0.0f;
            if (qx < len) {
                xc[u] = xcol_in[i * IMP_KA + qx];
                xv[u] = xval_in[i * IMP_KA + qx];
            }
        }
    };
    auto mark_x = [&](int64_t i, const int *xc) {
        const int xs = (int)(i % NXS);
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            if ((unsigned)xc[u] < (unsigned)n) atomicOr(&mask[xs * mw + (xc[u] >> 4)], xbit(xc[u]));
        if (tid == 0) {
            xa_new[xs] = 0;
            dec_fail[xs] = 0;
        }
    };
    // position of column k in the R list of slot sl (-1 if absent), from
    // the slot's hash table (the listed columns are distinct; the table has
    // at least 64 - IMP_K empty buckets, so a probe ends)
    auto rl_find = [&](int sl, int k) -> int {
        int h = rl_hash(k);
#pragma unroll 1
        for (int probe = 0; probe < 64; ++probe) {
            const int e = st_hash[sl][h];
            if (e < 0) break;
            if (e / IMP_K == k) return e % IMP_K;
            h = (h + 1) & 63;
        }
        return -1;
    };
    // acol_t of this thread's columns is the same for every row of the pass:
    // short rows keep it in registers, long rows read it per chunk
    constexpr bool ACV = J <= 5;
    float4 acv[ACV ? J : 1];
    if constexpr (ACV) {
#pragma unroll
        for (int j = 0; j < J; ++j) acv[j] = (j < J - 1 || last_in) ? ld4(acol_t + c0 + j * T * 4) : z4;
    }
    float4 s4[J];
    // block warm start: the thread's chunks that meet the row's block
    // [b0, b1) are consecutive, at most NB of them (checked by the host):
    // a_0 of chunk a0f + q in a0q[q] (zero outside the block)
    constexpr int NB = WB ? (J < 3 ? J : 3) : 1;
    float4 a0q[NB];
    int a0f = J;
    auto load_row = [&](int64_t i, float4 *dst) {
        const rsrc_t srs = row_rsrc(p.S + i * ld, ld);
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < J - 1 || last_in) dst[j] = bld4(srs, tid * 16, j * T * 16);
        if constexpr (WB) {
            const int b0 = p.blk[2 * i], b1 = p.blk[2 * i + 1];
            // first chunk with c + 3 >= b0 (chunk j starts at c0 + 4 T j)
            const int lo = b0 - 3 - c0;
            a0f = lo <= 0 ? 0 : (lo + 4 * T - 1) / (4 * T);
            const rsrc_t ars = row_rsrc(p.A + i * ld, ld);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const int j = a0f + q;
                const int c = c0 + j * T * 4;
                a0q[q] = (j < J && c < b1 && (j < J - 1 || last_in)) ? bld4(ars, tid * 16, j * T * 16) : z4;
            }
        }
    };
    // acol + lambda^t a_0 for chunk j (WB): the block chunk, if it is one
    auto warm_av = [&](int j, float4 &av) {
        if constexpr (WB) {
            const int q = j - a0f;
            if (__any(q >= 0 && q < NB)) {
                float4 a0 = z4;
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if (q == u) a0 = a0q[u];
                av.x = av.x + lt * a0.x;
                av.y = av.y + lt * a0.y;
                av.z = av.z + lt * a0.z;
                av.w = av.w + lt * a0.w;
            }
        }
    };
    int cur_c[EPT], nxt_c[EPT];
    float cur_v[EPT], nxt_v[EPT];
    // exception-list entries' s(i,k) and t_k, gathered right after the row's
    // S loads are issued (a row ahead), so that their latency overlaps the
    // previous row's reduction instead of following the scan
    float xsv[EPT], xtv[EPT], nxs[EPT], nxt[EPT];
    auto gather_x = [&](int64_t i, const int *xc, float *sv, float *tv) {
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            sv[u] = 0.0f;
            tv[u] = 0.0f;
            if ((unsigned)xc[u] < (unsigned)n) {
                sv[u] = p.S[i * ld + xc[u]];
                tv[u] = p.tcol[xc[u]];
            }
        }
    };
    if (r0 < r1) {
        const int rc = sw && lane < IMP_K ? cnt_in[r0] : 0;
        const float rgam = sw && lane < IMP_K ? gam_in[r0 * IMP_K + lane] : 0.0f;
        put_state(r0, fetch_state(r0), rc, rgam);
        fetch_x(r0, cur_c, cur_v);
        mark_x(r0, cur_c);
        load_row(r0, s4);
        gather_x(r0, cur_c, xsv, xtv);
    }
    // a column value above zero (a warm start) voids the D > 0 argument
    float amx = kNegInf;
    if constexpr (LEAN) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = c0 + j * T * 4;
            if (c < n) {
                float4 av;
                if constexpr (ACV) av = acv[j];
                else av = ld4(acol_t + c);
                amx = max3f(amx, av.x);
                if (c + 1 < n) amx = max3f(amx, av.y);
                if (c + 2 < n) amx = max3f(amx, av.z);
                if (c + 3 < n) amx = max3f(amx, av.w);
            }
        }
    }
    const bool acol_pos = __syncthreads_or(amx > 0.0f) != 0;

    for (int64_t i = r0; i < r1; ++i) {
        const int ii = (int)i;
        const int sl = (int)(i % 3);
        const int xs = (int)(i % NXS);
        // Positivity of the off-list r = al s - beta in the lean scan:
        // fl(mc s) > sc with (mc, sc) = (1, the row's threshold) when it is
        // certified and (al, beta) otherwise, exact either way; a row without
        // a certified threshold is decided over its ordinary columns after
        // the reduction.
        const float beta = st_beta[sl];
        const float sth = st_sth[sl];
        const bool cert = LEAN && sth == sth;
        const float mc = cert ? 1.0f : al;
        const float sc = cert ? sth : beta;
        const int cnt = st_cnt[sl];
        const float adg = st_ad[sl];
        const float sdg = st_sd[sl];
        const ColOwner dg = owner_of<T>(ii, tid);
        const int dle = dg.mine ? 4 * dg.j + dg.e : -1;   // local index of the diagonal
        const int xcnt = rcnt[i - r0];
        const int wb0 = WB ? p.blk[2 * i] : 0, wb1 = WB ? p.blk[2 * i + 1] : 0;
        // a_0(i,k) of a column of the row's block (WB; a global load, rare paths)
        auto a0_at = [&](int k) -> float {
            if constexpr (WB) return (k >= wb0 && k < wb1 && k != ii) ? p.A[i * ld + k] : 0.0f;
            return 0.0f;
        };
        // The exemplar decision: column ii wins iff no column k < ii has
        // a+r >= D and no column k > ii has a+r > D, D = a(i,i) + r(i,i)
        // (lowest index on ties).  v > D is tested as v >= next float above D.
        const float rdg = st_gdr[sl] == ii ? st_gd[sl] : al * sdg - beta;
        const float D = adg + rdg;
        const float Dn = __int_as_float(D >= 0.0f ? (D == 0.0f ? 1 : __float_as_int(D) + 1) : __float_as_int(D) - 1);
        bool fl = false;   // this thread saw a column that beats the diagonal
        const uint8_t *mb8 = mask8 + (size_t)xs * mw * 4;
        // previous exemplar flag of the row, read before the next row's S is
        // in flight (a later global load would wait for it)
        const uint8_t ef_prev = tid == 0 ? p.eflag[ii] : 0;
        // next row's R state and list, in flight during this row
        RowState nstate{0u, 0.0f, 0.0f};
        if (i + 1 < r1) {
            nstate = fetch_state(i + 1);
            fetch_x(i + 1, nxt_c, nxt_v);
        }
        // R-list entry tid (lanes of wavefront 0): column, stored r_t, s, acol_t
        int rk = -1;
        float rg = 0.0f, rs = 0.0f, rav = 0.0f;
        if (tid < cnt) {
            rk = st_col[sl][tid];
            rg = st_gam[sl][tid];
            if ((unsigned)rk < (unsigned)n) {
                rs = p.S[i * ld + rk];
                rav = acol_t[rk];
                if constexpr (WB) rav = rav + lt * a0_at(rk);
            } else {
                rk = -1;
            }
        }

        // ---- scan of the ordinary elements
        float v1 = kNegInf, v2 = kNegInf;
        float smax = kNegInf;   // largest s of the thread's columns that phase 2 leaves to it
        // the same per chunk (rows of up to six chunks per thread; longer
        // ones have no registers to spare and reread every chunk)
        constexpr bool CHM = J <= 6;
        float cmx[CHM ? J : 1];
#pragma unroll
        for (int j = 0; j < (CHM ? J : 1); ++j) cmx[j] = kNegInf;
        int l1 = -1;
        uint32_t fch = 0;       // chunks holding a first positive responsibility
        // longer rows: acol_t chunks stream from L2, one chunk ahead of use
        // (a load waited on at once per chunk serialises J latencies); at
        // J > 7 the extra registers spill and loading at use is faster
        constexpr int APF = (ACV || J > 7) ? 0 : 1;
        float4 avq[APF + 1];
        if constexpr (!ACV) {
#pragma unroll
            for (int j = 0; j < APF && j < J; ++j)
                if (j < J - 1 || last_in) avq[j] = ld4(acol_t + c0 + j * T * 4);
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (!(j < J - 1 || last_in)) continue;
            const bool full = (j < J - 1) || last_full;
            const int c = c0 + j * T * 4;
            const float4 sv = s4[j];
            float4 av;
            if constexpr (ACV) {
                av = acv[j];
            } else {
                if (j + APF < J && (j + APF < J - 1 || last_in))
                    avq[(j + APF) % (APF + 1)] = ld4(acol_t + c0 + (j + APF) * T * 4);
                av = avq[j % (APF + 1)];
            }
            warm_av(j, av);
            // out-of-range columns of the last chunk count as listed
            const uint32_t mb = mb8[j * T + tid] | (full ? 0u : oob_bits);
            // columns of this chunk below the diagonal beat it with a tie
            // (the diagonal's own chunk is finished after the scan)
            const float dth = c + 3 < ii ? D : Dn;
            bool fj = false;   // the chunk holds a first positive
            float cm = kNegInf;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float s = f4get(sv, e);
                // listed in either list (or out of range): one mask test
                const bool lst = (mb & (0x11u << e)) != 0u;
                float a;
                if constexpr (LEAN) {
                    // ordinary with r <= 0: A is the column value
                    const bool pos = mc * s > sc;
                    fj = fj || (pos && !lst);
                    a = !(lst || pos) ? f4get(av, e) : kNegInf;
                } else {
                    const float r = al * s - beta;
                    const bool ord = !(lst || r > 0.0f);
                    a = ord ? f4get(av, e) : kNegInf;
                    fl = fl || (a + r >= dth);
                }
                const float w = a + s;
                const bool g1 = w > v1;
                l1 = g1 ? 4 * j + e : l1;
                v2 = __builtin_amdgcn_fmed3f(v1, v2, w);
                v1 = g1 ? w : v1;
                // largest s of the ordinary columns (positive r included):
                // r = al s - beta is monotone in s, so it tells whether the
                // thread holds a first positive, and bounds phase 2's values
                cm = max3f(cm, lst ? kNegInf : s);
            }
            if constexpr (CHM) cmx[j] = cm;
            smax = max3f(smax, cm);
            if constexpr (LEAN) fch = fj ? (fch | (1u << j)) : fch;
        }
        // Chunks that can hold a positive R_{t+1} in phase 2: beta1 =
        // lam beta + (1-lam) V1 with V1 (the row's largest a + s) >= this
        // thread's v1, and fl(al1 s - b) rises with s and falls with b, so a
        // chunk whose largest ordinary s gives fl(al1 s - b_lo) <= 0, b_lo =
        // lam beta + (1-lam) v1, adds nothing there.
        uint32_t hch = ~0u;
        if constexpr (CHM) {
            const float blo = lam * beta + oml * v1;
            hch = 0u;
#pragma unroll
            for (int j = 0; j < J; ++j) hch |= (al1 * cmx[j] - blo > 0.0f) ? (1u << j) : 0u;
        }
        // a first positive somewhere in the thread's ordinary columns: every
        // chunk is searched (rare once the lists settle)
        if constexpr (!LEAN)
            fch = (al * smax - beta > 0.0f) ? ((1u << J) - 1u) & (last_in ? ~0u : ~(1u << (J - 1))) : 0u;
        Top2 t2{v1, l1 < 0 ? INT32_MAX : local_to_col<T>(l1, tid), v2};
        auto merge = [&](float v, float w, int k) {
            fl = fl || (k < ii ? v >= D : v > D);
            top2_merge(t2, w, k, kNegInf);
        };
        // the diagonal's chunk: its columns below the diagonal were tested
        // against Dn; a tie with D there also beats the diagonal
        if (!LEAN && __any(dle >= 0)) {
            if (dle >= 0) {
                float4 sv = s4[0];
                float4 av;
#pragma unroll
                for (int jj = 1; jj < J; ++jj)
                    if (jj == dle >> 2) sv = s4[jj];
                if constexpr (ACV) {
                    av = acv[0];
#pragma unroll
                    for (int jj = 1; jj < J; ++jj)
                        if (jj == dle >> 2) av = acv[jj];
                } else {
                    av = ld4(acol_t + c0 + (dle >> 2) * T * 4);
                }
                if constexpr (WB) {
                    // the diagonal's chunk is in the block
                    const int q = (dle >> 2) - a0f;
                    float4 a0 = z4;
#pragma unroll
                    for (int u = 0; u < NB; ++u)
                        if (q == u) a0 = a0q[u];
                    av.x = av.x + lt * a0.x;
                    av.y = av.y + lt * a0.y;
                    av.z = av.z + lt * a0.z;
                    av.w = av.w + lt * a0.w;
                }
                const uint32_t mb = mb8[(dle >> 2) * T + tid];
                const uint32_t ex = (mb | (mb >> 4)) & 0xFu;
                for (int e = 0; e < (dle & 3); ++e) {
                    const float r = al * f4get(sv, e) - beta;
                    if (!((ex >> e) & 1u) && !(r > 0.0f) && f4get(av, e) + r == D) fl = true;
                }
            }
        }
        // first positive responsibility: A from acol_{t-1}, a new list entry
        auto fresh = [&](int k, float s, float r) {
            float ap = acol_p[k];
            if constexpr (WB) ap = ap + ltp * a0_at(k);
            const float an = lam * ap + oml * fminf(0.0f, p.tcol[k] - r);
            merge(an + r, an + s, k);
            const int pos = xcnt + atomicAdd(&xa_new[xs], 1);
            if (pos < xcap) {
                xcol_out[i * IMP_KA + pos] = k;
                xval_out[i * IMP_KA + pos] = an;
            }
        };
        if (__any(fch != 0)) {
            uint32_t m = fch;
            while (m) {
                const int j = __builtin_ctz(m);
                m &= m - 1;
                float4 sv = s4[0];
#pragma unroll
                for (int jj = 1; jj < J; ++jj)
                    if (jj == j) sv = s4[jj];
                const uint32_t mb = mb8[j * T + tid];
                const uint32_t ex = (mb | (mb >> 4)) & 0xFu;
                const int cj = c0 + j * T * 4;
                if constexpr (CHM) {
                    // the chunk's first positives as a bit mask, then one
                    // append per entry (a wavefront runs the append as often
                    // as its busiest lane needs it, not once per element
                    // position)
                    uint32_t fm = 0u;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float r = al * f4get(sv, e) - beta;
                        fm |= (cj + e < n && !((ex >> e) & 1u) && r > 0.0f) ? (1u << e) : 0u;
                    }
                    while (fm) {
                        const int e = __builtin_ctz(fm);
                        fm &= fm - 1;
                        const float s = f4get(sv, e);
                        fresh(cj + e, s, al * s - beta);
                    }
                } else {
                    for (int e = 0; e < 4; ++e) {
                        const int k = cj + e;
                        if (k >= n) break;
                        const float s = f4get(sv, e);
                        const float r = al * s - beta;
                        if (!((ex >> e) & 1u) && r > 0.0f) fresh(k, s, r);
                    }
                }
            }
        }
        // R-listed columns, by the holder of the entry (those also in the
        // exception list are merged by the list holder)
        const bool rl_diag = __ballot(rk == ii) != 0;     // meaningful in wavefront 0
        if (rk >= 0) {
            const float r = rg;
            if (rk == ii) {
                top2_merge(t2, adg + rs, ii, kNegInf);
            } else if (!((mask8[(size_t)xs * mw * 4 + (rk >> 2)] >> (rk & 3)) & 1u)) {
                if (r > 0.0f) fresh(rk, rs, r);
                else merge(rav + r, rav + rs, rk);
            }
        }
        // the diagonal (thread 0) unless it is R-listed: top-2 only
        if (tid == 0 && !rl_diag) top2_merge(t2, adg + sdg, ii, kNegInf);
        // exception-list entries: A from the stored value
        bool xrl[EPT];   // the column is R-listed (its R-list holder forms the partial)
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            xrl[u] = false;
            const int k = cur_c[u];
            if ((unsigned)k < (unsigned)n) {
                float r = al * xsv[u] - beta;
                if ((mb8[k >> 2] >> (4 + (k & 3))) & 1u) {
                    xrl[u] = true;
                    const int at = rl_find(sl, k);
                    if (at >= 0) r = st_gam[sl][at];
                }
                const float an = lam * cur_v[u] + oml * fminf(0.0f, xtv[u] - fmaxf(0.0f, r));
                merge(an + r, an + xsv[u], k);
                xcol_out[i * IMP_KA + xq0 + u * T] = k;
                xval_out[i * IMP_KA + xq0 + u * T] = an;
            }
        }
        if (__any(fl) && lane == 0) atomicOr(&dec_fail[xs], 1);
        __builtin_amdgcn_sched_barrier(0);
        if (i + 1 < r1) {
            int ncnt = 0;
            float ngam = 0.0f;
            if (sw) {
                // the count (lane 2K+1) and stored r (lane + K) of the state words
                ncnt = __builtin_amdgcn_readlane((int)nstate.v, 2 * IMP_K + 1);
                ngam = __uint_as_float((uint32_t)__shfl((int)nstate.v, lane + IMP_K));
            }
            put_state(i + 1, nstate, ncnt, ngam);
            mark_x(i + 1, nxt_c);
            load_row(i + 1, s4);
            gather_x(i + 1, nxt_c, nxs, nxt);
        }
        __builtin_amdgcn_sched_barrier(0);

        wg_top2<NW>(t2, sh_v[i & 1], sh_i[i & 1], lane, wave);
        // the previous row's additions to global partials are visible
        if constexpr (GP) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "global");
        // A lean row whose listed and special columns do not beat the
        // diagonal, with D <= 0 (or a positive column value), or without a
        // certified threshold: the ordinary columns decide, tested as the
        // full scan tests them (S and acol reloaded; the row's mask slot is
        // intact until the next row)
        if (LEAN && __builtin_amdgcn_readfirstlane((int)(!cert || (dec_fail[xs] == 0 && (!(D > 0.0f) || acol_pos))))) {
            bool f2 = false;
            const float *srow = p.S + i * ld;
#pragma unroll 1
            for (int j = 0; j < J; ++j) {
                const int c = c0 + j * T * 4;
                if (c >= n) continue;
                const float4 sv = ld4(srow + c);
                const float4 av = ld4(acol_t + c);
                const uint32_t mb = mb8[j * T + tid];
                const uint32_t ex = (mb | (mb >> 4)) & 0xFu;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = c + e;
                    const float r = al * f4get(sv, e) - beta;
                    if (k < n && !((ex >> e) & 1u) && !(r > 0.0f)) {
                        const float q = f4get(av, e) + r;
                        f2 = f2 || (k < ii ? q >= D : q > D);
                    }
                }
            }
            if (__any(f2) && lane == 0) atomicOr(&dec_fail[xs], 1);
            if (tid == 0) atomicAdd(&p.st->lean_rescans, 1);
            __syncthreads();
        }
        if (tid == 0) {
            const uint8_t ef = (uint8_t)(dec_fail[xs] == 0);
            if (ef_prev != ef) my_changed = 1;
            p.eflag[ii] = ef;
            my_nex += ef;
        }
        const int xnew = xa_new[xs];
        const bool xovf = xcnt + xnew > xcap;
        if (tid == 0) {
            xcnt_out[ii] = xovf ? -1 : xcnt + xnew;
            if (xovf) atomicOr(&p.st->imp_abort, 2);
        }

        // State of R_{t+1}: beta' = lam beta + (1-lam) v1 off the list; on
        // it (and for k1 when it joins) the damped Eq. (2) in the explicit
        // pass's rounding, r' = (lam r + (1-lam) s) - (1-lam) (k = k1 ? v2 :
        // v1), stored as r itself (no cancellation of alpha s - beta against
        // a large offset).  The list is held by wavefront 0, so its searches
        // are ballots there.
        const int k1 = t2.k1;
        const float m_other = oml * t2.v1, m_self = oml * t2.v2;
        const float beta1 = lam * beta + oml * t2.v1;
        const uint64_t bk1 = __ballot(rk >= 0 && rk == k1);
        const int pos1 = bk1 ? __builtin_ctzll(bk1) : -1;                  // wavefront 0
        const int k1_owner = (k1 >> 2) % T;
        const int k1_owner_has = __popcll(__ballot(rk >= 0 && ((rk >> 2) % T) == k1_owner));
        // Only a full list overflows here: listed columns are handled by
        // their holders, not their owners.  A list that the implicit-R pass
        // could not take over (an owner with more than NOWN listed columns)
        // is noted in the run state, so that a fallback from implicit A
        // makes R explicit too.
        const bool ovf = pos1 < 0 && cnt >= p.kmax;                        // wavefront 0
        if (tid == 0 && pos1 < 0 && !ovf && k1_owner_has >= NOWN) atomicOr(&p.st->imp_owner, 1);
        // r_{t+1} of this lane's list entry, and of k1 when it joins the list
        // (its s: one load, rare once the lists settle)
        const float rl1 = (lam * rg + oml * rs) - (tid == pos1 ? m_self : m_other);
        float k1_r1 = 0.0f;
        if (tid == 0 && pos1 < 0) {
            const float s1 = p.S[i * ld + k1];
            k1_r1 = (lam * (al * s1 - beta) + oml * s1) - m_self;
        }
        if (wave == 0) {
            if (rk >= 0 && !ovf) {
                col_out[(int64_t)ii * IMP_K + tid] = rk;
                gam_out[(int64_t)ii * IMP_K + tid] = rl1;
            }
            if (tid == 0) {
                beta_out[ii] = beta1;
                if (ovf) {
                    cnt_out[ii] = -1;
                    atomicOr(&p.st->imp_abort, 1);
                } else {
                    if (pos1 < 0) {
                        col_out[(int64_t)ii * IMP_K + cnt] = k1;
                        gam_out[(int64_t)ii * IMP_K + cnt] = k1_r1;
                    }
                    cnt_out[ii] = cnt + (pos1 < 0 ? 1 : 0);
                }
            }
        }

        // this thread's bytes of the previous row's mask slot
        if (i > r0) {
            uint8_t *pm = mask8 + (size_t)((i - 1) % NXS) * mw * 4;
#pragma unroll
            for (int j = 0; j < J; ++j)
                if (j < J - 1 || last_in) pm[j * T + tid] = 0;
        }

        // ---- column partials of max(0, R_{t+1}), one addition per row and
        // column, in row order: special columns and listed ones by their
        // holders, the rest by their owners.  The reduction barrier orders
        // the additions of consecutive rows (LDS partials); with global
        // partials a wavefront that added makes its stores visible before
        // the next row's barrier (release below, acquire after the reduction).
        bool added = false;
        auto padd = [&](int k, float r) {
            if constexpr (GP) P[k] = P[k] + r;
            else lp[k] = lp[k] + r;
            added = true;
        };
        if (rk >= 0) {
            const float r = rl1;
            if (rk == ii) p.rdiag[ii] = r;
            else if (r > 0.0f) padd(rk, r);
        }
        if (tid == 0) {
            if (pos1 < 0) {
                // a new list column
                const float r = k1_r1;
                if (k1 == ii) p.rdiag[ii] = r;
                else if (r > 0.0f) padd(k1, r);
            }
            if (!rl_diag && !(pos1 < 0 && k1 == ii)) p.rdiag[ii] = al1 * sdg - beta1;
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int k = cur_c[u];
            if ((unsigned)k < (unsigned)n && !xrl[u] && k != k1) {
                const float r = al1 * xsv[u] - beta1;
                if (r > 0.0f) padd(k, r);
            }
        }
        // ordinary elements: a positive value needs al1 s - beta1 > 0,
        // which is monotone in s, so only threads whose largest ordinary
        // s passes reread their chunks (from L2), and only the chunks that
        // the scan's bound leaves open
        const bool hot = al1 * smax - beta1 > 0.0f;
        if (__any(hot)) {
            if (hot) {
                const float *srow = p.S + i * ld;
#pragma unroll 1
                for (int j = 0; j < J; ++j) {
                    if (!(j < J - 1 || last_in) || !((hch >> j) & 1u)) continue;
                    const int c = c0 + j * T * 4;
                    const float4 sv = ld4(srow + c);
                    const uint32_t mb = mb8[j * T + tid];
                    if (mb == 0u && (k1 >> 2) != (c >> 2) && c + 3 < n) {
                        // no listed column and not k1's chunk: no other
                        // thread adds to these columns in this row
                        float4 a4;
                        if constexpr (GP) a4 = ld4(P + c);
                        else a4 = lpart[c >> 2];
                        a4.x = (al1 * sv.x - beta1 > 0.0f) ? a4.x + (al1 * sv.x - beta1) : a4.x;
                        a4.y = (al1 * sv.y - beta1 > 0.0f) ? a4.y + (al1 * sv.y - beta1) : a4.y;
                        a4.z = (al1 * sv.z - beta1 > 0.0f) ? a4.z + (al1 * sv.z - beta1) : a4.z;
                        a4.w = (al1 * sv.w - beta1 > 0.0f) ? a4.w + (al1 * sv.w - beta1) : a4.w;
                        if constexpr (GP) st4(P + c, a4);
                        else lpart[c >> 2] = a4;
                        added = true;
                        continue;
                    }
                    const uint32_t ex = (mb | (mb >> 4)) & 0xFu;
                    for (int e = 0; e < 4; ++e) {
                        const int k = c + e;
                        const float r = al1 * f4get(sv, e) - beta1;
                        if (k < n && !((ex >> e) & 1u) && k != k1 && r > 0.0f) padd(k, r);
                    }
                }
            }
        }
        if constexpr (GP) {
            if (__any(added)) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "global");
        }

        // Overflowing rows (at most once per run), written explicitly with
        // the same values.  R_{t+1}: by wavefront 0, which holds the list.
        if (wave == 0 && ovf) {
            float *Rx = Rx_base + i * ld;
            for (int k = lane; k < n; k += 64) {
                const float s = p.S[i * ld + k];
                float r = al1 * s - beta1;
                bool listed = false;
                for (int qq = 0; qq < cnt; ++qq) {
                    if (st_col[sl][qq] == k) {
                        r = (lam * st_gam[sl][qq] + oml * s) - (k == k1 ? m_self : m_other);
                        listed = true;
                    }
                }
                if (!listed && k == k1) r = (lam * (al * s - beta) + oml * s) - m_self;
                Rx[k] = r;
            }
        }
        if (xovf) {
            // A_t: listed values from this row's output list (written before
            // the reduction barrier by their holders)
            __syncthreads();
            float *Arow = p.A + i * ld;
#pragma unroll 1
            for (int j = 0; j < J; ++j) {
                const int c = c0 + j * T * 4;
                const uint32_t mb = (j < J - 1 || last_in) ? mb8[j * T + tid] : 0u;
                for (int e = 0; e < 4; ++e) {
                    const int k = c + e;
                    if (k >= n) break;
                    const float s = p.S[i * ld + k];
                    float r = al * s - beta;
                    if ((mb >> (4 + e)) & 1u) {
                        for (int qq = 0; qq < cnt; ++qq)
                            if (st_col[sl][qq] == k) r = st_gam[sl][qq];
                    }
                    const float a0 = a0_at(k);   // read before this element is overwritten
                    float a = acol_t[k];
                    if constexpr (WB) a = a + lt * a0;
                    if (k == ii) {
                        a = adg;
                    } else if ((mb >> e) & 1u) {
                        for (int qq = 0; qq < xcnt; ++qq)
                            if (xcol_out[i * IMP_KA + qq] == k) a = xval_out[i * IMP_KA + qq];
                    } else if (r > 0.0f) {
                        float ap = acol_p[k];
                        if constexpr (WB) ap = ap + ltp * a0;
                        a = lam * ap + oml * fminf(0.0f, p.tcol[k] - r);
                    }
                    Arow[k] = a;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            cur_c[u] = nxt_c[u];
            cur_v[u] = nxt_v[u];
            xsv[u] = nxs[u];
            xtv[u] = nxt[u];
        }
    }

    if constexpr (!GP) {
        __syncthreads();   // holders add to other threads' columns
#pragma unroll
        for (int j = 0; j < J; ++j)
            if (j < J - 1 || last_in) st4(P + c0 + j * T * 4, lpart[j * T + tid]);
    }
    if (tid == 0) {
        if (my_nex) atomicAdd(&p.st->nex, my_nex);
        if (my_changed) atomicOr(&p.st->changed, 1);
    }
}

// A = acol off the diagonal, adiag on it, then the listed exceptions.
__global__ void k_ia_materialize(float *A, int64_t ld, int32_t n, const float *acol, const float *adiag,
                                 const char *xs, const int32_t *blk, float lam, int32_t t) {
    const XLayout X = x_layout(n);
    const int32_t *cnt = reinterpret_cast<const int32_t *>(xs + X.cnt);
    const int32_t *col = reinterpret_cast<const int32_t *>(xs + X.col);
    const float *val = reinterpret_cast<const float *>(xs + X.val);
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int c = cnt[i];
        if (c < 0) continue;
        float *row = A + i * ld;
        const float ad = adiag[i];
        if (blk != nullptr) {
            // block warm start: acol + lambda^t a_0 inside the row's block
            // (a_0 read from A itself, each element by the thread writing it)
            const float lt = ia_lambda_pow(lam, t);
            const int64_t b0 = blk[2 * i], b1 = blk[2 * i + 1];
            for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
                float v = acol[k];
                if (k >= b0 && k < b1 && k != i) v = v + lt * row[k];
                row[k] = k == i ? ad : v;
            }
        } else {
            // 16-byte stores (rows are 16-byte aligned, the column vector is
            // padded to a multiple of four); the tail past n is left alone
            for (int64_t k = 4 * (int64_t)threadIdx.x; k < n; k += 4 * (int64_t)blockDim.x) {
                if (k + 3 < n) {
                    float4 v = *reinterpret_cast<const float4 *>(acol + k);
                    v.x = k == i ? ad : v.x;
                    v.y = k + 1 == i ? ad : v.y;
                    v.z = k + 2 == i ? ad : v.z;
                    v.w = k + 3 == i ? ad : v.w;
                    *reinterpret_cast<float4 *>(row + k) = v;
                } else {
                    for (int64_t q = k; q < n; ++q) row[q] = (q == i) ? ad : acol[q];
                }
            }
        }
        __syncthreads();
        for (int qq = threadIdx.x; qq < c && qq < IMP_KA; qq += blockDim.x) {
            const int k = col[i * IMP_KA + qq];
            if ((unsigned)k < (unsigned)n) row[k] = val[i * IMP_KA + qq];
        }
        __syncthreads();
    }
}

// R(i,k) = alpha s(i,k) - beta(i) off the row's list and the stored value
// on it, for every row with a list; the same values the passes use.
__global__ void k_imp_materialize(const float *S, float *R, int64_t ld, int32_t n, const float *alpha,
                                  const char *state) {
#pragma clang fp contract(off)
    const ImpLayout L = imp_layout(n);
    const float *beta = reinterpret_cast<const float *>(state + L.beta);
    const int32_t *cnt = reinterpret_cast<const int32_t *>(state + L.cnt);
    const int32_t *col = reinterpret_cast<const int32_t *>(state + L.col);
    const float *gam = reinterpret_cast<const float *>(state + L.gam);
    const float al = *alpha;
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int c = cnt[i];
        if (c < 0) continue;
        const float b = beta[i];
        const float *srow = S + i * ld;
        float *rrow = R + i * ld;
        for (int64_t k = 4 * (int64_t)threadIdx.x; k < n; k += 4 * (int64_t)blockDim.x) {
            if (k + 3 < n) {
                const float4 sv = *reinterpret_cast<const float4 *>(srow + k);
                float4 rv;
                rv.x = al * sv.x - b;
                rv.y = al * sv.y - b;
                rv.z = al * sv.z - b;
                rv.w = al * sv.w - b;
                *reinterpret_cast<float4 *>(rrow + k) = rv;
            } else {
                for (int64_t q = k; q < n; ++q) rrow[q] = al * srow[q] - b;
            }
        }
        __syncthreads();
        if (threadIdx.x < c) {
            const int64_t k = col[i * IMP_K + threadIdx.x];
            rrow[k] = gam[i * IMP_K + threadIdx.x];
        }
        __syncthreads();
    }
}

__global__ void k_state_resume(ApState *st) {
    if (threadIdx.x == 0) {
        st->frozen = 0;
        st->imp_abort = 0;
    }
}

template <int T, int J, int KIND, bool PREF>
hipError_t launch_imp_k(const ImpArgs &a, int grid, size_t lds, hipStream_t s) {
    static bool attr_set = false;   // per process; the attribute is per function
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_row_imp<T, J, KIND, PREF>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLdsImp);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    k_row_imp<T, J, KIND, PREF><<<grid, T, lds, s>>>(a);
    return hipGetLastError();
}

template <int T, int J, bool PREF>
hipError_t launch_imp_tj(int kind, const ImpArgs &a, const PassPlan &pl, hipStream_t s) {
    switch (kind) {
    case IMP_FULL: return launch_imp_k<T, J, IMP_FULL, PREF>(a, pl.grid, pl.lds_bytes, s);
    case IMP_PRO_COLD: return launch_imp_k<T, J, IMP_PRO_COLD, PREF>(a, pl.grid, pl.lds_bytes, s);
    default: return launch_imp_k<T, J, IMP_PRO_WARM, PREF>(a, pl.grid, pl.lds_bytes, s);
    }
}

template <int T, int J>
hipError_t launch_imp_t(int kind, const ImpArgs &a, const PassPlan &pl, hipStream_t s) {
    // prefetching variant whenever the current row of S fits next to the partials
    if constexpr (J <= 5) {
        if (pl.lds_bytes >= (size_t)32 * (size_t)((a.n + 3) / 4)) return launch_imp_tj<T, J, true>(kind, a, pl, s);
    }
    return launch_imp_tj<T, J, false>(kind, a, pl, s);
}

template <int T, int J, bool GP, bool WB>
hipError_t launch_ia_k(const ImpArgs &a, int grid, size_t lds, hipStream_t s) {
    static bool attr_set = false;   // per process; the attribute is per function
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_row_ia<T, J, GP, WB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLdsIa);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    k_row_ia<T, J, GP, WB><<<grid, T, lds, s>>>(a);
    return hipGetLastError();
}

// LDS of the implicit-A pass: partials (unless GP), NXS mask slots, the
// list lengths of a workgroup's rows.
size_t ia_lds(int64_t n, int grid, bool gp) {
    const int64_t q = (n + 3) / 4, mw = (q + 3) / 4;
    const int64_t rows = (n + grid - 1) / grid + 1;
    return (size_t)(gp ? 0 : 16 * q) + (size_t)(NXS * mw * 4) + (size_t)(4 * rows);
}

// The block warm start has 1024-thread variants only (n > 4096).
template <int T, int J>
hipError_t launch_ia_t(const ImpArgs &a, const PassPlan &pl, hipStream_t s) {
    const bool gp = pl.lds_bytes < ia_lds(a.n, pl.grid, false);
    const bool wb = a.blk != nullptr;
    if constexpr (T == 1024) {
        if (wb) {
            if constexpr (J >= 7) {
                if (gp) return launch_ia_k<T, J, true, true>(a, pl.grid, pl.lds_bytes, s);
            } else {
                if (gp) return hipErrorInvalidValue;
            }
            return launch_ia_k<T, J, false, true>(a, pl.grid, pl.lds_bytes, s);
        }
    } else {
        if (wb) return hipErrorInvalidValue;
    }
    if constexpr (J >= 7) {
        if (gp) return launch_ia_k<T, J, true, false>(a, pl.grid, pl.lds_bytes, s);
    } else {
        if (gp) return hipErrorInvalidValue;
    }
    return launch_ia_k<T, J, false, false>(a, pl.grid, pl.lds_bytes, s);
}

}  // namespace

// Chunks (float4 per thread per row) instantiated for each workgroup size.
int max_chunks(int threads) { return threads == 256 ? 4 : threads == 512 ? 8 : threads == 1024 ? 16 : 0; }

PassPlan plan_pass_variant(int64_t n, int num_cus, int threads, bool lds) {
    PassPlan pl{};
    const int64_t q = (n + 3) / 4;   // float4 chunks per row
    // The row -> workgroup map depends on n only, so every variant computes
    // the same column partial sums and gives bit-identical results.
    const int64_t g = n <= 4096 ? 2LL * num_cus : (int64_t)num_cus;
    pl.grid = (int)(n < g ? n : g);
    pl.threads = threads;
    pl.chunks = (int)((q + threads - 1) / threads);
    if (pl.chunks > max_chunks(threads)) {
        pl.threads = 0;           // not instantiated
        return pl;
    }
    const size_t bytes = (size_t)2 * 16 * (size_t)q;
    pl.lds_bytes = (lds && bytes <= (size_t)kMaxDynLds && pl.chunks <= 5) ? bytes : 0;
    return pl;
}

// Above 12 chunks per thread (n > 49152) the register-resident pass holds
// u and the partials of up to 16 chunks with low occupancy and falls below
// the two-sweep pass, which reads S and R_t twice: at 13-16 chunks the
// register pass moves 3.4-3.8 TB/s of its 20 B per element, the two-sweep
// pass 4.0 TB/s; at 12 chunks and below the register pass is faster.
constexpr int kRegPassMaxChunks = 12;

PassPlan plan_pass(int64_t n, int num_cus) {
    PassPlan pl = plan_pass_variant(n, num_cus, n <= 4096 ? 256 : 1024, true);
    // APX_ROW_PASS=reg selects the register variant, APX_ROW_PASS=2s the
    // two-sweep pass (cross-checks; 1024-thread plans only).
    const char *v = getenv("APX_ROW_PASS");
    if (v && v[0] == 'r') pl.lds_bytes = 0;
    const bool force_2s = v && v[0] == '2' && n > 4096;
    if (n > 4096 && (pl.threads == 0 || pl.chunks > kRegPassMaxChunks || force_2s)) {
        // rows longer than the register-resident variants hold well (or
        // forced): the same row -> workgroup map, two sweeps per row
        const int64_t q = (n + 3) / 4;
        pl.grid = (int)(n < num_cus ? n : num_cus);
        pl.threads = 1024;
        pl.chunks = (int)((q + 1023) / 1024);
        pl.lds_bytes = 0;
        pl.two_sweep = 1;
    }
    return pl;
}

hipError_t launch_row_pass(const PassPlan &pl, int mode, const PassArgs &a, hipStream_t s) {
    if (pl.two_sweep) return pl.threads == 1024 ? launch_2s(mode, a, pl.grid, s) : hipErrorInvalidValue;
    if (pl.threads == 256) {
        switch (pl.chunks) {
        case 1: return launch_t<256, 1>(mode, a, pl, s);
        case 2: return launch_t<256, 2>(mode, a, pl, s);
        case 3: return launch_t<256, 3>(mode, a, pl, s);
        case 4: return launch_t<256, 4>(mode, a, pl, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (pl.threads == 512) {
        switch (pl.chunks) {
        case 1: return launch_t<512, 1>(mode, a, pl, s);
        case 2: return launch_t<512, 2>(mode, a, pl, s);
        case 3: return launch_t<512, 3>(mode, a, pl, s);
        case 4: return launch_t<512, 4>(mode, a, pl, s);
        case 5: return launch_t<512, 5>(mode, a, pl, s);
        case 6: return launch_t<512, 6>(mode, a, pl, s);
        case 7: return launch_t<512, 7>(mode, a, pl, s);
        case 8: return launch_t<512, 8>(mode, a, pl, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (pl.threads != 1024) return hipErrorInvalidValue;
    switch (pl.chunks) {
    case 1: return launch_t<1024, 1>(mode, a, pl, s);
    case 2: return launch_t<1024, 2>(mode, a, pl, s);
    case 3: return launch_t<1024, 3>(mode, a, pl, s);
    case 4: return launch_t<1024, 4>(mode, a, pl, s);
    case 5: return launch_t<1024, 5>(mode, a, pl, s);
    case 6: return launch_t<1024, 6>(mode, a, pl, s);
    case 7: return launch_t<1024, 7>(mode, a, pl, s);
    case 8: return launch_t<1024, 8>(mode, a, pl, s);
    case 9: return launch_t<1024, 9>(mode, a, pl, s);
    case 10: return launch_t<1024, 10>(mode, a, pl, s);
    case 11: return launch_t<1024, 11>(mode, a, pl, s);
    case 12: return launch_t<1024, 12>(mode, a, pl, s);
    case 13: return launch_t<1024, 13>(mode, a, pl, s);
    case 14: return launch_t<1024, 14>(mode, a, pl, s);
    case 15: return launch_t<1024, 15>(mode, a, pl, s);
    case 16: return launch_t<1024, 16>(mode, a, pl, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_col_reduce(const ColArgs &a, hipStream_t s) {
    const int grid = (a.n + 63) / 64;
    k_col_reduce<<<grid, 1024, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_state_init(ApState *st, int32_t max_iter, int32_t conv_iter, float lam, hipStream_t s,
                             int msg_on, float msg_tol, int alpha_one) {
    k_state_init<<<1, 64, 0, s>>>(st, max_iter, conv_iter, lam, msg_on, msg_tol, alpha_one);
    return hipGetLastError();
}

hipError_t launch_extract_cols(const float *A, int64_t ld, int32_t n, float *acol, float *adiag, hipStream_t s) {
    const int g = (n + 255) / 256;
    k_extract_cols<<<g > 0 ? g : 1, 256, 0, s>>>(A, ld, n, acol, adiag);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float *M, int64_t rows, int64_t cols, int64_t ld, int32_t *flag,
                               hipStream_t s) {
    const int g = (int)(rows < 8192 ? (rows > 0 ? rows : 1) : 8192);
    k_check_finite<<<g, 256, 0, s>>>(M, rows, cols, ld, flag);
    return hipGetLastError();
}

hipError_t launch_decide(const float *A, const float *R, int64_t n, int64_t ld, int32_t *dec, hipStream_t s) {
    k_decide<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(A, R, n, ld, dec);
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

hipError_t launch_compact(const FinalArgs &a, hipStream_t s) {
    k_compact<<<1, 1024, 0, s>>>(a.eflag, a.n, a.ex, a.nex);
    return hipGetLastError();
}
hipError_t launch_labels(const FinalArgs &a, hipStream_t s) {
    const int64_t rows = (a.row1 > 0 ? a.row1 : a.n) - a.row0;
    if (rows <= 0) return hipSuccess;
    k_labels<<<(unsigned)((rows + 3) / 4), 256, 0, s>>>(a);
    return hipGetLastError();
}
hipError_t launch_sum2(const FinalArgs &a, hipStream_t s) {
    k_sum2<<<1, 1024, 0, s>>>(a.contrib, a.n, a.sums);
    return hipGetLastError();
}
hipError_t launch_finalize(const FinalArgs &a, hipStream_t s) {
    hipError_t e = launch_compact(a, s);
    if (e != hipSuccess) return e;
    e = launch_labels(a, s);
    if (e != hipSuccess) return e;
    return launch_sum2(a, s);
}


bool imp_plan(int64_t n, int num_cus, PassPlan *pl) {
    const int64_t q = (n + 3) / 4;
    const int threads = n <= 4096 ? 256 : 1024;
    const int maxj = threads == 256 ? 4 : 10;
    PassPlan p{};
    const int64_t g = n <= 4096 ? 2LL * num_cus : (int64_t)num_cus;
    p.grid = (int)(n < g ? n : g);
    p.threads = threads;
    p.chunks = (int)((q + threads - 1) / threads);
    if (p.chunks > maxj) return false;
    const size_t with_s = (size_t)32 * (size_t)q, part_only = (size_t)16 * (size_t)q;
    // APX_IMP_PREFETCH=0 keeps S out of LDS (the non-prefetching variant; cross-checks)
    const char *v = getenv("APX_IMP_PREFETCH");
    const bool pref = !(v && v[0] == '0');
    if (pref && p.chunks <= 5 && with_s <= (size_t)kMaxDynLdsImp) p.lds_bytes = with_s;
    else if (part_only <= (size_t)kMaxDynLdsImp) p.lds_bytes = part_only;
    else return false;
    *pl = p;
    return true;
}

hipError_t launch_row_imp(const PassPlan &pl, int kind, const ImpArgs &a, hipStream_t s) {
    if (pl.threads == 256) {
        switch (pl.chunks) {
        case 1: return launch_imp_t<256, 1>(kind, a, pl, s);
        case 2: return launch_imp_t<256, 2>(kind, a, pl, s);
        case 3: return launch_imp_t<256, 3>(kind, a, pl, s);
        case 4: return launch_imp_t<256, 4>(kind, a, pl, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (pl.threads != 1024) return hipErrorInvalidValue;
    switch (pl.chunks) {
    case 1: return launch_imp_t<1024, 1>(kind, a, pl, s);
    case 2: return launch_imp_t<1024, 2>(kind, a, pl, s);
    case 3: return launch_imp_t<1024, 3>(kind, a, pl, s);
    case 4: return launch_imp_t<1024, 4>(kind, a, pl, s);
    case 5: return launch_imp_t<1024, 5>(kind, a, pl, s);
    case 6: return launch_imp_t<1024, 6>(kind, a, pl, s);
    case 7: return launch_imp_t<1024, 7>(kind, a, pl, s);
    case 8: return launch_imp_t<1024, 8>(kind, a, pl, s);
    case 9: return launch_imp_t<1024, 9>(kind, a, pl, s);
    case 10: return launch_imp_t<1024, 10>(kind, a, pl, s);
    default: return hipErrorInvalidValue;
    }
}

bool ia_plan(int64_t n, int num_cus, PassPlan *pl) {
    const int64_t q = (n + 3) / 4;
    const int threads = n <= 4096 ? 256 : 1024;
    const int maxj = threads == 256 ? 4 : 10;
    PassPlan p{};
    const int64_t g = n <= 4096 ? 2LL * num_cus : (int64_t)num_cus;
    p.grid = (int)(n < g ? n : g);
    p.threads = threads;
    p.chunks = (int)((q + threads - 1) / threads);
    if (n < 1 || p.chunks > maxj) return false;
    // APX_IMPLICIT_A_GP=1 keeps the partials in global memory (cross-checks)
    const char *v = getenv("APX_IMPLICIT_A_GP");
    bool gp = ia_lds(n, p.grid, false) > (size_t)kMaxDynLdsIa || (v && v[0] == '1' && p.chunks >= 7);
    p.lds_bytes = ia_lds(n, p.grid, gp);
    if (p.lds_bytes > (size_t)kMaxDynLdsIa) return false;
    *pl = p;
    return true;
}

hipError_t launch_row_ia(const PassPlan &pl, const ImpArgs &a, hipStream_t s) {
    if (pl.threads == 256) {
        switch (pl.chunks) {
        case 1: return launch_ia_t<256, 1>(a, pl, s);
        case 2: return launch_ia_t<256, 2>(a, pl, s);
        case 3: return launch_ia_t<256, 3>(a, pl, s);
        case 4: return launch_ia_t<256, 4>(a, pl, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (pl.threads != 1024) return hipErrorInvalidValue;
    switch (pl.chunks) {
    case 1: return launch_ia_t<1024, 1>(a, pl, s);
    case 2: return launch_ia_t<1024, 2>(a, pl, s);
    case 3: return launch_ia_t<1024, 3>(a, pl, s);
    case 4: return launch_ia_t<1024, 4>(a, pl, s);
    case 5: return launch_ia_t<1024, 5>(a, pl, s);
    case 6: return launch_ia_t<1024, 6>(a, pl, s);
    case 7: return launch_ia_t<1024, 7>(a, pl, s);
    case 8: return launch_ia_t<1024, 8>(a, pl, s);
    case 9: return launch_ia_t<1024, 9>(a, pl, s);
    case 10: return launch_ia_t<1024, 10>(a, pl, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ia_materialize(float *A, int64_t ld, int32_t n, const float *acol, const float *adiag,
                                 const char *x_parity, hipStream_t s, const int32_t *blk, float lam, int32_t t) {
    const int g = n < 8192 ? n : 8192;
    k_ia_materialize<<<g > 0 ? g : 1, 256, 0, s>>>(A, ld, n, acol, adiag, x_parity, blk, lam, t);
    return hipGetLastError();
}

__global__ void k_extract_diag(const float *A, int64_t ld, int32_t n, float *adiag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) adiag[k] = A[(int64_t)k * ld + k];
}

hipError_t launch_extract_diag(const float *A, int64_t ld, int32_t n, float *adiag, hipStream_t s) {
    const int g = (n + 255) / 256;
    k_extract_diag<<<g > 0 ? g : 1, 256, 0, s>>>(A, ld, n, adiag);
    return hipGetLastError();
}

hipError_t launch_imp_materialize(const float *S, float *R, int64_t ld, int32_t n, const float *alpha,
                                  const char *state_parity, hipStream_t s) {
    const int g = n < 8192 ? n : 8192;
    k_imp_materialize<<<g > 0 ? g : 1, 256, 0, s>>>(S, R, ld, n, alpha, state_parity);
    return hipGetLastError();
}

hipError_t launch_state_resume(ApState *st, hipStream_t s) {
    k_state_resume<<<1, 64, 0, s>>>(st);
    return hipGetLastError();
}

}  // namespace apx
