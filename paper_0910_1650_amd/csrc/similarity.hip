// similarity.hip -- S from points, preferences and tie-break noise.
//
//   s(i,k) = -||x_i - x_k||^2 = 2<x_i,x_k> - (||x_i||^2 + ||x_k||^2)   (Section 2)
//
// The Gram part runs on FP32 matrix cores (v_mfma_f32_32x32x2f32, FP32
// accumulate).  Only tiles on or above the block diagonal are computed; each
// result is written at (i,k) and mirrored to (k,i) from the accumulators,
// so S is exactly symmetric.  The preference is the median of the n(n-1) off-diagonal
// entries, found exactly by a three-pass radix select over the upper
// triangle (which holds every off-diagonal value twice by symmetry).
#include <cmath>

#include "apx_internal.h"

namespace apx {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int BM = 128;      // tile edge
// K chunk staged in LDS.  16 rather than 32 halves the registers that
// carry the next chunk's loads, so three workgroups fit a CU instead of two
// (168 registers instead of 192): the writes of S of one workgroup overlap
// the MFMAs of two others.  The MFMA sequence (two K values per step, in
// ascending order) is the same for any chunk size, so S is unchanged.
constexpr int KB = 16;
constexpr int NT = 256;      // threads per tile (4 wavefronts)
constexpr int SEL_BINS = 8192;   // bins per rank in the global select histogram (13-bit first digit)

// Ordered 32-bit key of a float: unsigned order equals float order.
__device__ __forceinline__ uint32_t fkey(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float keyf(uint32_t k) {
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

__global__ void k_sqnorm(const float *X, int64_t n, int64_t d, int64_t ldx, float *nrm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float *x = X + i * ldx;
    float acc = 0.0f;
    for (int64_t j = 0; j < d; ++j) acc = fmaf(x[j], x[j], acc);
    nrm[i] = acc;
}

struct SimArgs {
    const float *X;
    int64_t n, d, ldx;
    const float *nrm;
    float *S;
    int64_t ld;
    int64_t tiles_per_side;
    uint32_t *minmax;     // [0] = min key, [1] = max key of off-diagonal entries
    // median preference: the first digit pass of the exact select (13-bit
    // digits of the upper entries' keys; both ranks share the empty prefix)
    // counted here, into hist[b] and hist[SEL_BINS + b]; null: no counting
    unsigned long long *hist;
    const int32_t *bad;   // nonzero: the input failed the finite check, write nothing
};

// One 128 x 128 tile per workgroup.  X rows are staged through LDS one K
// chunk at a time, the next chunk's global loads in flight during the
// current chunk's MFMAs; the epilogue writes S straight from the
// accumulators (no LDS tile): lane l of
// block (x, y) holds column c = l mod 32 and rows 8g + 4(l / 32) + q
// (g, q = 0..3), written directly (one float per row, 128-byte row
// segments per half wavefront) and mirrored (the four rows q are
// consecutive columns of S's row c: one float4).  With the median
// preference (COUNT) the epilogue also counts the first 13-bit digit of
// every upper entry's key in an LDS histogram whose nonzero bins the tile
// adds to the global one: the select's first pass over S is not needed.
constexpr int LDA = BM + 1;   // padded LDS rows: conflict-free transposed stores

// Gram block <x_i, x_k> of rows row0.. and columns col0.. (BM each) into the
// accumulators: wavefront (wm, wn) holds the 2 x 2 32x32 blocks at rows
// wm*64 + 32x, columns wn*64 + 32y.  Every entry sums its products in the
// same order (K chunks of KB, two per MFMA), whichever tile it lies in and
// whichever of x_i, x_k is the A operand, so an entry has one value.
__device__ __forceinline__ void gram_tile(const float *X, int64_t n, int64_t d, int64_t ldx, int64_t row0,
                                          int64_t col0, v16f (&acc)[2][2], float *As, float *Bs) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[x][y][v] = 0.0f;

    // X[row0 .. +BM, k0 .. +KB] and X[col0 .. +BM, k0 .. +KB] into registers
    constexpr int SU = BM * KB / NT;
    float va[SU], vb[SU];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int e = tid + u * NT;
            const int m = e / KB, kk = e % KB;
            const int64_t kg = k0 + kk;
            const int64_t ra = row0 + m, rb = col0 + m;
            va[u] = (ra < n && kg < d) ? X[ra * ldx + kg] : 0.0f;
            vb[u] = (rb < n && kg < d) ? X[rb * ldx + kg] : 0.0f;
        }
    };
    fetch(0);
    for (int64_t k0 = 0; k0 < d; k0 += KB) {
        // staged k-major; the previous chunk's MFMAs are done (barrier below)
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const int e = tid + u * NT;
            const int m = e / KB, kk = e % KB;
            As[kk * LDA + m] = va[u];
            Bs[kk * LDA + m] = vb[u];
        }
        __syncthreads();
        if (k0 + KB < d) fetch(k0 + KB);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 2) {
            const int kr = kk + (lane >> 5);
            float av[2], bv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) av[x] = As[kr * LDA + wm * 64 + x * 32 + (lane & 31)];
#pragma unroll
            for (int y = 0; y < 2; ++y) bv[y] = Bs[kr * LDA + wn * 64 + y * 32 + (lane & 31)];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x], bv[y], acc[x][y], 0, 0, 0);
        }
        __syncthreads();
    }
}

template <bool COUNT>
__global__ __launch_bounds__(NT) void k_sim_gemm(SimArgs a) {
    if (*a.bad) return;
    // Decode the upper-triangle tile (bi <= bj) from the linear block index.
    const int64_t T = a.tiles_per_side;
    int64_t t = blockIdx.x, bi = 0;
    while (t >= T - bi) {
        t -= T - bi;
        ++bi;
    }
    const int64_t bj = bi + t;
    const int64_t row0 = bi * BM, col0 = bj * BM;

    __shared__ float As[KB * LDA], Bs[KB * LDA];    // 16.5 KB of staging
    __shared__ float nr[BM], nc[BM];                // squared norms of the tile's rows and columns
    __shared__ uint32_t hsh[COUNT ? SEL_BINS : 1];  // first-digit counts of the tile's upper entries
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    if constexpr (COUNT)
        for (int b = tid; b < SEL_BINS; b += NT) hsh[b] = 0u;   // published by gram_tile's barriers (d >= 1)
    for (int e = tid; e < BM; e += NT) {
        nr[e] = row0 + e < a.n ? a.nrm[row0 + e] : 0.0f;
        nc[e] = col0 + e < a.n ? a.nrm[col0 + e] : 0.0f;
    }
    v16f acc[2][2];
    gram_tile(a.X, a.n, a.d, a.ldx, row0, col0, acc, As, Bs);

    uint32_t kmin = 0xffffffffu, kmax = 0u;
    const bool diag_tile = (bi == bj);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int c = wn * 64 + y * 32 + (lane & 31);   // tile column
            const int64_t k = col0 + c;
            const float ncc = nc[c];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int mb = wm * 64 + x * 32 + 8 * g + 4 * (lane >> 5);   // first of four rows
                const int64_t ib = row0 + mb;
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = 2.0f * acc[x][y][4 * g + q] - (nr[mb + q] + ncc);
                if (k >= a.n) continue;
                if (!diag_tile) {
                    // every (i, k) here has i < k: direct, mirror, bounds
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (ib + q < a.n) {
                            a.S[(ib + q) * a.ld + k] = v[q];
                            const uint32_t key = fkey(v[q]);
                            kmin = min(kmin, key);
                            kmax = max(kmax, key);
                            if constexpr (COUNT) atomicAdd(&hsh[key >> 19], 1u);
                        }
                    }
                    float *dst = a.S + k * a.ld + ib;
                    if (ib + 3 < a.n) {
                        *reinterpret_cast<float4 *>(dst) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (ib + q < a.n) dst[q] = v[q];
                    }
                } else {
                    // diagonal tile: the upper entries (m < c) are written at
                    // (m, c) and (c, m), so S is symmetric; the diagonal gets
                    // a value that the preference pass overwrites
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int m = mb + q;
                        if (ib + q >= a.n || m > c) continue;
                        a.S[(ib + q) * a.ld + k] = v[q];
                        if (m < c) {
                            a.S[k * a.ld + ib + q] = v[q];
                            const uint32_t key = fkey(v[q]);
                            kmin = min(kmin, key);
                            kmax = max(kmax, key);
                            if constexpr (COUNT) atomicAdd(&hsh[key >> 19], 1u);
                        }
                    }
                }
            }
        }
    // Block min/max of the upper off-diagonal entries: wavefronts, then the
    // tile, then one atomic per bound, skipped when it cannot change the value
    // (all tiles update the same two words).
    for (int off = 32; off >= 1; off >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
    }
    __shared__ uint32_t red[2][NT / 64];
    if (lane == 0) {
        red[0][wave] = kmin;
        red[1][wave] = kmax;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) {
            kmin = min(kmin, red[0][w]);
            kmax = max(kmax, red[1][w]);
        }
        if (kmin < __atomic_load_n(&a.minmax[0], __ATOMIC_RELAXED)) atomicMin(&a.minmax[0], kmin);
        if (kmax > __atomic_load_n(&a.minmax[1], __ATOMIC_RELAXED)) atomicMax(&a.minmax[1], kmax);
    }
    // the tile's counts (integers: the sums do not depend on the order);
    // the barrier above ordered every LDS count before these reads
    if constexpr (COUNT) {
        for (int b = tid; b < SEL_BINS; b += NT) {
            const uint32_t c = hsh[b];
            if (c) {
                atomicAdd(&a.hist[b], (unsigned long long)c);
                atomicAdd(&a.hist[SEL_BINS + b], (unsigned long long)c);
            }
        }
    }
}

// ---- exact order statistics of the upper triangle -------------------------
// sel[0..1]: state of the two ranks (lo, hi): prefix key bits so far.
struct SelState {
    uint32_t prefix[2];
    uint32_t pad0[2];
    unsigned long long rank[2];   // remaining rank inside the current prefix
};

// Digits of the 32-bit key: 13 bits (the first pass, when both ranks share
// the empty prefix and one histogram counts for both: more bins spread the
// counter contention of keys that share their exponent), then 10 and 9.
__device__ __forceinline__ void sel_digit(int pass, int &shift, int &bits, uint32_t &hmask) {
    shift = pass == 0 ? 19 : (pass == 1 ? 9 : 0);
    bits = pass == 0 ? 13 : (pass == 1 ? 10 : 9);
    hmask = pass == 0 ? 0u : (pass == 1 ? 0xfff80000u : 0xfffffe00u);
}

__global__ void k_sel_init(SelState *st, uint32_t *minmax, unsigned long long lo,
                           unsigned long long hi, unsigned long long *hist) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->prefix[0] = st->prefix[1] = 0u;
        st->rank[0] = lo;
        st->rank[1] = hi;
        minmax[0] = 0xffffffffu;
        minmax[1] = 0u;
    }
    for (int b = threadIdx.x; b < 2 * SEL_BINS; b += blockDim.x) hist[b] = 0ull;
}

// Histogram of the keys of upper-triangle entries whose high bits match the
// current prefix of each rank.  shift/bits select the digit of this pass.
// f(k, v) for the entries v = row[k], k = i+1 .. n-1, of row i: the unaligned
// head one by one, then 16-byte pieces (rows start 16-byte aligned: ld is a
// multiple of 4), U per thread in flight in every step, the row's ragged end
// included (its last piece read element by element, nothing at or beyond n).
typedef float sv4 __attribute__((ext_vector_type(4)));
template <int U, class F>
__device__ __forceinline__ void upper_row(const float *row, int64_t i, int64_t n, F &&f) {
    const int64_t k4 = (i + 4) & ~int64_t(3);          // first multiple of 4 above i
    const int64_t kh = k4 < n ? k4 : n;
    if (i + 1 + threadIdx.x < kh) f(i + 1 + threadIdx.x, row[i + 1 + threadIdx.x]);
    const int64_t st = 4 * (int64_t)blockDim.x;
    for (int64_t kb = k4 + 4 * (int64_t)threadIdx.x; kb < n; kb += U * st) {
        float4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = kb + u * st;
            if (k + 3 < n) {
                // read once per pass: nontemporal
                const sv4 w = __builtin_nontemporal_load(reinterpret_cast<const sv4 *>(row + k));
                v[u] = make_float4(w.x, w.y, w.z, w.w);
            } else {
                v[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (k < n) v[u].x = row[k];
                if (k + 1 < n) v[u].y = row[k + 1];
                if (k + 2 < n) v[u].z = row[k + 2];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = kb + u * st;
            if (k < n) f(k, v[u].x);
            if (k + 1 < n) f(k + 1, v[u].y);
            if (k + 2 < n) f(k + 2, v[u].z);
            if (k + 3 < n) f(k + 3, v[u].w);
        }
    }
}

// Workgroups of a row-walking pass: as many as are resident on the chip
// at once (workgroup b walks rows b, b + grid, ...: a second, partial round
// would leave most CUs idle while it finishes), at most one per row.
int walk_grid(const void *kern, size_t lds, int64_t rows) {
    int dev = 0, cus = 0, occ = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 256, lds) != hipSuccess || occ < 1) occ = 1;
    const int64_t g = (int64_t)occ * cus;
    return (int)(rows < g ? rows : g);
}

// Rows [r0, r1) of S (row i at S + i * ld).
__global__ __launch_bounds__(256) void k_sel_hist(const float *S, int64_t n, int64_t ld,
                                                  const SelState *st, int pass,
                                                  unsigned long long *hist, int64_t r0, int64_t r1) {
    // dynamic LDS: one histogram of nb bins on the first pass (both ranks
    // start from the same empty prefix), two on the others
    extern __shared__ uint32_t hsh[];
    int shift, bits;
    uint32_t hmask;
    sel_digit(pass, shift, bits, hmask);
    const uint32_t nb = 1u << bits;
    const uint32_t nh = pass == 0 ? 1u : 2u;
    for (uint32_t b = threadIdx.x; b < nh * nb; b += blockDim.x) hsh[b] = 0u;
    __syncthreads();
    const uint32_t p0 = st->prefix[0], p1 = st->prefix[1];
    // both ranks inside one prefix (always on the first pass): one count
    // serves both histograms
    const bool same = p0 == p1;
    uint32_t *const h0 = hsh;
    uint32_t *const h1 = hsh + (nh - 1) * nb;
    auto count = [&](int64_t, float v) {
        const uint32_t key = fkey(v);
        const uint32_t dig = (key >> shift) & (nb - 1u);
        if ((key & hmask) == p0) atomicAdd(&h0[dig], 1u);
        if (!same && (key & hmask) == p1) atomicAdd(&h1[dig], 1u);
    };
    const int64_t re = r1 < n - 1 ? r1 : n - 1;
    for (int64_t i = r0 + blockIdx.x; i < re; i += gridDim.x) upper_row<8>(S + i * ld, i, n, count);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const uint32_t c0 = h0[b], c1 = same ? c0 : h1[b];
        if (c0) atomicAdd(&hist[b], (unsigned long long)c0);
        if (c1) atomicAdd(&hist[SEL_BINS + b], (unsigned long long)c1);
    }
}

// Inclusive prefix sum over the 256 threads: wavefront shuffles, then the
// wavefront totals through LDS (ws: 4 entries).
__device__ __forceinline__ unsigned long long block_scan256(unsigned long long x, unsigned long long *ws) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) ws[w] = x;
    __syncthreads();
    unsigned long long add = 0ull;
    for (int k = 0; k < w; ++k) add += ws[k];
    __syncthreads();
    return x + add;
}

// Pick the digit holding each rank; extend the prefixes; clear the histogram.
// 256 threads: each sums nb/256 consecutive digits, a block scan of the
// sums finds the segment holding the rank, its owner walks its digits
// (held in registers since the sum).
__global__ __launch_bounds__(256) void k_sel_pick(SelState *st, int pass, unsigned long long *hist) {
    int shift, bits;
    uint32_t hmask;
    sel_digit(pass, shift, bits, hmask);
    const uint32_t nb = 1u << bits;
    const uint32_t per = nb / 256;               // digits per thread (32, 4 or 2)
    constexpr int MAXPER = SEL_BINS / 256;
    __shared__ unsigned long long ws[4];
    const int t = threadIdx.x;
    for (int r = 0; r < 2; ++r) {
        const unsigned long long *hr = hist + r * SEL_BINS;
        // the thread's segment of digits, all loads in flight at once
        unsigned long long v[MAXPER];
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) v[q] = (uint32_t)q < per ? hr[t * per + q] : 0ull;
        unsigned long long own = 0ull;
#pragma unroll
        for (int q = 0; q < MAXPER; ++q) own += v[q];
        // read before the scan's barriers: the owner rewrites it below
        const unsigned long long rank = st->rank[r];
        const unsigned long long incl = block_scan256(own, ws);
        const unsigned long long before = incl - own;   // digits below this thread's segment
        if (rank >= before && rank < incl) {
            unsigned long long cum = before;
            uint32_t b = t * per;
            bool found = false;
#pragma unroll
            for (int q = 0; q < MAXPER; ++q) {
                if (!found && (uint32_t)q < per) {
                    if (rank < cum + v[q]) {
                        found = true;
                        b = t * per + q;
                    } else {
                        cum += v[q];
                    }
                }
            }
            st->rank[r] = rank - cum;
            st->prefix[r] |= (b << shift);
        }
        __syncthreads();
    }
    for (int b = t; b < 2 * SEL_BINS; b += blockDim.x) hist[b] = 0ull;
}

struct PrefArgs {
    float *S;
    int64_t n, ld;
    int mode;                 // APX_PREF_*
    const float *pref_vec;
    float pref_scalar;
    const SelState *sel;      // median mode
    const uint32_t *minmax;
    uint64_t seed;
    double noise_rel;
    double *pref_dev;         // out: the scalar preference (median/scalar)
    const int32_t *bad = nullptr;   // nonzero: the input failed the finite check, write nothing
};

__device__ __forceinline__ double pref_of(const PrefArgs &a, int64_t i, double pm) {
    if (a.mode == APX_PREF_VECTOR) return (double)a.pref_vec[i];
    return pm;
}

__device__ __forceinline__ double median_of(const PrefArgs &a) {
    if (a.mode == APX_PREF_MEDIAN)
        return 0.5 * ((double)keyf(a.sel->prefix[0]) + (double)keyf(a.sel->prefix[1]));
    return (double)a.pref_scalar;
}

// SplitMix64 output function (Steele, Lea, Flood 2014) on the counter
// seed + (i*n+k+1) * golden gamma; top 53 bits as a double in [0,1).
__device__ __forceinline__ double noise_u(uint64_t seed, int64_t n, int64_t i, int64_t k) {
    uint64_t z = seed + (uint64_t)(i * n + k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// fl32((double)v + scale * u) for u in [0, 1).  When scale <= |v| 2^-27 the
// sum stays below v + 2^(e-26) (2^e <= |v|), far from the midpoint to v's
// upper neighbour (at least 2^(e-25) away, also when |v| is a power of two
// and v < 0), so it rounds back to v and the counter generator is skipped:
// the same value, without its 64-bit arithmetic (the tie noise is far below
// one FP32 ulp of most entries).
__device__ __forceinline__ float add_noise(float v, double scale, uint64_t seed, int64_t n, int64_t i, int64_t k) {
    const double dv = (double)v;
    if (scale <= fabs(dv) * 0x1p-27) return v;
    return (float)(dv + scale * noise_u(seed, n, i, k));
}

// The noise of an upper entry v = s(i,k) that the noise changes, written at
// (i,k) and, with its own draw, at (k,i).  Out of line: the row walks call
// it for few entries, and inlined into each of their unrolled element slots
// its 64-bit arithmetic would take the registers of their loads in flight.
__device__ __noinline__ void put_noise(float *S, int64_t ld, float v, double scale, uint64_t seed, int64_t n,
                                       int64_t i, int64_t k) {
    S[i * ld + k] = add_noise(v, scale, seed, n, i, k);
    S[k * ld + i] = add_noise(v, scale, seed, n, k, i);
}

// Range of S with the preferences on the diagonal (FP64).
__global__ void k_pref_range(PrefArgs a, double *range_out) {
    __shared__ float lo[256], hi[256];
    const double pm = median_of(a);
    float mn = keyf(a.minmax[0]), mx = keyf(a.minmax[1]);
    for (int64_t i = threadIdx.x; i < a.n; i += blockDim.x) {
        const float p = (float)pref_of(a, i, pm);
        mn = fminf(mn, p);
        mx = fmaxf(mx, p);
    }
    lo[threadIdx.x] = mn;
    hi[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lo[threadIdx.x] = fminf(lo[threadIdx.x], lo[threadIdx.x + w]);
            hi[threadIdx.x] = fmaxf(hi[threadIdx.x], hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *range_out = (double)hi[0] - (double)lo[0];
        *a.pref_dev = pm;
    }
}

// Diagonal := preference (+ its noise); with noise, every off-diagonal entry
// v becomes fl32(v + scale * u(i,k)).  S is symmetric before the noise, so
// the upper triangle alone is read: an entry the noise changes (add_noise)
// is written at (i,k) and, with its own draw, at (k,i); the others keep v.
__global__ __launch_bounds__(256) void k_pref_noise(PrefArgs a, const double *range) {
    if (a.bad != nullptr && *a.bad) return;
    const double pm = median_of(a);
    const double scale = a.noise_rel * (*range);
    const bool noise = a.noise_rel > 0.0;
    for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
        float *row = a.S + i * a.ld;
        if (threadIdx.x == 0) {
            const double base = pref_of(a, i, pm);
            row[i] = noise ? (float)(base + scale * noise_u(a.seed, a.n, i, i)) : (float)base;
        }
        if (!noise) continue;
        upper_row<8>(row, i, a.n, [&](int64_t k, float v) {
            if (scale <= fabs((double)v) * 0x1p-27) return;
            put_noise(a.S, a.ld, v, scale, a.seed, a.n, i, k);
        });
    }
}

// Median mode, last select pass fused with the tie noise: the upper triangle
// is read once and counted for the last digit (values before noise); an
// entry the noise changes is written at (i,k) and, with its own draw, at
// (k,i) (S is symmetric before the noise; no pass reads the lower triangle
// or an entry after its row's block has read it).  The diagonal is left for
// k_pref_diag once the median is known.  The noise scale needs only the
// off-diagonal range (the median lies inside it).
__global__ __launch_bounds__(256) void k_sel_hist_noise(PrefArgs a, unsigned long long *hist) {
    if (a.bad != nullptr && *a.bad) return;
    extern __shared__ uint32_t hsh[];
    constexpr int pass = 2;
    int shift, bits;
    uint32_t hmask;
    sel_digit(pass, shift, bits, hmask);
    const uint32_t nb = 1u << bits;
    for (uint32_t b = threadIdx.x; b < 2 * nb; b += blockDim.x) hsh[b] = 0u;
    __syncthreads();
    const uint32_t p0 = a.sel->prefix[0], p1 = a.sel->prefix[1];
    const bool same = p0 == p1;
    uint32_t *const h0 = hsh;
    uint32_t *const h1 = hsh + nb;
    const double scale = a.noise_rel * ((double)keyf(a.minmax[1]) - (double)keyf(a.minmax[0]));
    for (int64_t i = blockIdx.x; i < a.n - 1; i += gridDim.x) {
        float *row = a.S + i * a.ld;
        upper_row<8>(row, i, a.n, [&](int64_t k, float v) {
            const uint32_t key = fkey(v);
            const uint32_t dig = (key >> shift) & (nb - 1u);
            if ((key & hmask) == p0) atomicAdd(&h0[dig], 1u);
            if (!same && (key & hmask) == p1) atomicAdd(&h1[dig], 1u);
            if (scale <= fabs((double)v) * 0x1p-27) return;
            put_noise(a.S, a.ld, v, scale, a.seed, a.n, i, k);
        });
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        const uint32_t c0 = h0[b], c1 = same ? c0 : h1[b];
        if (c0) atomicAdd(&hist[b], (unsigned long long)c0);
        if (c1) atomicAdd(&hist[SEL_BINS + b], (unsigned long long)c1);
    }
}

// The diagonal after the fused pass: s(i,i) = p (+ its noise).
__global__ void k_pref_diag(PrefArgs a, const double *range) {
    if (a.bad != nullptr && *a.bad) return;
    const double pm = median_of(a);
    const double scale = a.noise_rel * (*range);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const double base = pref_of(a, i, pm);
        a.S[i * a.ld + i] = a.noise_rel > 0.0 ? (float)(base + scale * noise_u(a.seed, a.n, i, i)) : (float)base;
    }
}

// ---- matrix-free S: row panels ---------------------------------------------
// Rows [p0, p1) of S into a panel (row i at Sp + (i - p0) * ld), every tile
// of the panel computed (nothing mirrored).  An entry gets the value that
// ap_similarity stores: the same Gram sum (gram_tile), then, with final set,
// the preference on the diagonal and the tie noise as the median or the
// preference pass adds it (the off-diagonal noise scale is the range of the
// off-diagonal entries in median mode, of S with the preferences otherwise).
// final = 0: the values before both, and the bounds of the off-diagonal keys.
struct PanelArgs {
    const float *X;
    int64_t n, d, ldx;
    const float *nrm;
    float *Sp;
    int64_t ld, p0, p1;
    int final;
    PrefArgs pa;              // preference mode and values, select state, bounds, noise
    const double *range;      // final: range of S with the preferences
    uint32_t *minmax;         // final = 0: bounds of the off-diagonal keys (atomic)
    const ApState *st;        // nullable: a frozen run skips the panel
};

__global__ __launch_bounds__(NT) void k_sim_panel(PanelArgs a) {
    if (a.st != nullptr && a.st->frozen) return;
    const int64_t tn = (a.n + BM - 1) / BM;
    const int64_t bi = blockIdx.x / tn, bj = blockIdx.x % tn;
    const int64_t row0 = a.p0 + bi * BM, col0 = bj * BM;
    __shared__ float As[KB * LDA], Bs[KB * LDA];
    __shared__ float nr[BM], nc[BM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    for (int e = tid; e < BM; e += NT) {
        nr[e] = row0 + e < a.n ? a.nrm[row0 + e] : 0.0f;
        nc[e] = col0 + e < a.n ? a.nrm[col0 + e] : 0.0f;
    }
    v16f acc[2][2];
    gram_tile(a.X, a.n, a.d, a.ldx, row0, col0, acc, As, Bs);

    double pm = 0.0, sc_off = 0.0, sc_diag = 0.0;
    if (a.final) {
        pm = median_of(a.pa);
        sc_diag = a.pa.noise_rel * (*a.range);
        sc_off = a.pa.mode == APX_PREF_MEDIAN
            ? a.pa.noise_rel * ((double)keyf(a.pa.minmax[1]) - (double)keyf(a.pa.minmax[0]))
            : sc_diag;
    }
    const bool noise = a.pa.noise_rel > 0.0;
    uint32_t kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int c = wn * 64 + y * 32 + (lane & 31);
            const int64_t k = col0 + c;
            const float ncc = nc[c];
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int mb = wm * 64 + x * 32 + 8 * g + 4 * (lane >> 5);
                const int64_t ib = row0 + mb;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t i = ib + q;
                    if (k >= a.n || i >= a.p1) continue;
                    const float v = 2.0f * acc[x][y][4 * g + q] - (nr[mb + q] + ncc);
                    float out = v;
                    if (!a.final) {
                        if (k != i) {
                            const uint32_t key = fkey(v);
                            kmin = min(kmin, key);
                            kmax = max(kmax, key);
                        }
                    } else if (k == i) {
                        const double base = pref_of(a.pa, i, pm);
                        out = noise ? (float)(base + sc_diag * noise_u(a.pa.seed, a.n, i, i)) : (float)base;
                    } else if (noise) {
                        out = add_noise(v, sc_off, a.pa.seed, a.n, i, k);
                    }
                    a.Sp[(i - a.p0) * a.ld + k] = out;
                }
            }
        }
    if (!a.final) {
        for (int off = 32; off >= 1; off >>= 1) {
            kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
            kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
        }
        if (lane == 0) {
            if (kmin < __atomic_load_n(&a.minmax[0], __ATOMIC_RELAXED)) atomicMin(&a.minmax[0], kmin);
            if (kmax > __atomic_load_n(&a.minmax[1], __ATOMIC_RELAXED)) atomicMax(&a.minmax[1], kmax);
        }
    }
}

}  // namespace
}  // namespace apx

using namespace apx;

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return hip_err(ctx, _e, what);  \
    } while (0)

namespace {
struct SimLayout {
    size_t o_n, o_mm, o_sel, o_h, o_r, bytes;
};
SimLayout sim_layout(int64_t n) {
    WsLayout L;
    SimLayout o{};
    o.o_n = L.take(sizeof(float) * (size_t)n);
    o.o_mm = L.take(sizeof(uint32_t) * 2);
    o.o_sel = L.take(sizeof(SelState));
    o.o_h = L.take(sizeof(unsigned long long) * 2 * SEL_BINS);
    o.o_r = L.take(sizeof(double) * 2);
    o.bytes = L.off;
    return o;
}
}  // namespace

size_t apx::similarity_ws_bytes(int64_t n) { return sim_layout(n).bytes; }

extern "C" apx_status ap_similarity(apx_ctx *ctx, const float *X, int64_t n, int64_t d, int64_t ldx,
                                    float *S, int64_t ld, int32_t pref_mode, const float *pref_vec,
                                    float pref_scalar, uint64_t noise_seed, double noise_rel,
                                    double *pref_out) {
    if (!ctx) return APX_EINVAL;
    if (!X || !S) return set_err(ctx, APX_EINVAL, "X and S must be non-null");
    if (n < 2 || d < 1) return set_err(ctx, APX_EINVAL, "need n >= 2 and d >= 1");
    if (n > (int64_t)1 << 31) return set_err(ctx, APX_ENOTIMPL, "n too large");
    if (ldx < d) return set_err(ctx, APX_EINVAL, "ldx < d");
    if (ld < n || ld % 4) return set_err(ctx, APX_EINVAL, "ld must be >= n and a multiple of 4");
    if ((reinterpret_cast<uintptr_t>(S) & 15u) != 0) return set_err(ctx, APX_EINVAL, "S not 16-byte aligned");
    if (pref_mode < APX_PREF_MEDIAN || pref_mode > APX_PREF_VECTOR)
        return set_err(ctx, APX_EINVAL, "bad pref_mode");
    if (pref_mode == APX_PREF_VECTOR && !pref_vec) return set_err(ctx, APX_EINVAL, "pref_vec is null");
    if (pref_mode == APX_PREF_SCALAR && !std::isfinite(pref_scalar))
        return set_err(ctx, APX_EINVAL, "pref_scalar is not finite");
    if (!(noise_rel >= 0.0) || !std::isfinite(noise_rel)) return set_err(ctx, APX_EINVAL, "bad noise_rel");
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != ctx->device) (void)hipSetDevice(ctx->device);
    hipStream_t s = ctx->stream;

    const SimLayout SL = sim_layout(n);
    const size_t o_n = SL.o_n, o_mm = SL.o_mm, o_sel = SL.o_sel, o_h = SL.o_h, o_r = SL.o_r;
    apx_status st = ws_reserve(ctx, ctx->ws_base + SL.bytes);
    if (st != APX_OK) return st;

    // Non-finite input is rejected before S is written.
    int32_t *hflag = reinterpret_cast<int32_t *>(static_cast<char *>(ctx->pinned) + 2048);
    HIP_TRY(launch_fill_u8(reinterpret_cast<uint8_t *>(ctx->dflag), sizeof(int32_t), 0, s), "finite check");
    HIP_TRY(launch_check_finite(X, n, d, ldx, ctx->dflag, s), "finite check");
    if (pref_mode == APX_PREF_VECTOR) HIP_TRY(launch_check_finite(pref_vec, 1, n, n, ctx->dflag, s), "finite check");
    // (no wait here: every kernel that writes S reads the flag first and
    // returns when it is set; the host reads it at the end)
    const int32_t *bad = static_cast<const int32_t *>(ctx->dflag);
    char *b = static_cast<char *>(ctx->ws) + ctx->ws_base;
    float *nrm = reinterpret_cast<float *>(b + o_n);
    uint32_t *mm = reinterpret_cast<uint32_t *>(b + o_mm);
    SelState *sel = reinterpret_cast<SelState *>(b + o_sel);
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(b + o_h);
    double *dvals = reinterpret_cast<double *>(b + o_r);   // [0] range, [1] preference

    const unsigned long long M = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
    const unsigned long long lo = (M % 2) ? (M - 1) / 2 : M / 2 - 1;
    const unsigned long long hi = (M % 2) ? (M - 1) / 2 : M / 2;
    k_sel_init<<<1, 256, 0, s>>>(sel, mm, lo, hi, hist);
    HIP_TRY(hipGetLastError(), "select init");
    k_sqnorm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(X, n, d, ldx, nrm);
    HIP_TRY(hipGetLastError(), "sqnorm");
    // median preference: the GEMM counts the select's first digit
    SimArgs sa{X, n, d, ldx, nrm, S, ld, (n + BM - 1) / BM, mm, pref_mode == APX_PREF_MEDIAN ? hist : nullptr, bad};
    const int64_t ntiles = sa.tiles_per_side * (sa.tiles_per_side + 1) / 2;
    if (sa.hist) k_sim_gemm<true><<<(unsigned)ntiles, NT, 0, s>>>(sa);
    else k_sim_gemm<false><<<(unsigned)ntiles, NT, 0, s>>>(sa);
    HIP_TRY(hipGetLastError(), "similarity gemm");
    PrefArgs pa{S, n, ld, pref_mode, pref_vec, pref_scalar, sel, mm, noise_seed, noise_rel, &dvals[1], bad};
    if (pref_mode == APX_PREF_MEDIAN) {
        // three digits: the first counted by the GEMM, two passes over the
        // upper triangle; with noise the last one also adds the noise to
        // every off-diagonal entry
        for (int pass = 0; pass < 3; ++pass) {
            const size_t lds = sizeof(uint32_t) * (pass == 0 ? 8192 : 2 * (pass == 1 ? 1024 : 512));
            if (pass == 0) {
                // first digit: counted by the GEMM
            } else if (pass == 2 && noise_rel > 0.0) {
                const int g = walk_grid((const void *)k_sel_hist_noise, lds, n - 1);
                k_sel_hist_noise<<<g, 256, lds, s>>>(pa, hist);
            } else {
                const int g = walk_grid((const void *)k_sel_hist, lds, n - 1);
                k_sel_hist<<<g, 256, lds, s>>>(S, n, ld, sel, pass, hist, 0, n);
            }
            HIP_TRY(hipGetLastError(), "select histogram");
            k_sel_pick<<<1, 256, 0, s>>>(sel, pass, hist);
            HIP_TRY(hipGetLastError(), "select pick");
        }
        k_pref_range<<<1, 256, 0, s>>>(pa, &dvals[0]);
        HIP_TRY(hipGetLastError(), "preference range");
        k_pref_diag<<<(unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), 256, 0, s>>>(pa, &dvals[0]);
        HIP_TRY(hipGetLastError(), "preference");
    } else {
        k_pref_range<<<1, 256, 0, s>>>(pa, &dvals[0]);
        HIP_TRY(hipGetLastError(), "preference range");
        const int g = (int)(n < 8192 ? n : 8192);
        k_pref_noise<<<g, 256, 0, s>>>(pa, &dvals[0]);
        HIP_TRY(hipGetLastError(), "preference/noise");
    }
    // The bounds of the off-diagonal keys tell whether a similarity overflowed
    // (a key at or beyond the one of +inf or -inf: infinities and NaNs).
    double *h = reinterpret_cast<double *>(static_cast<char *>(ctx->pinned) + 1024);
    uint32_t *hk = reinterpret_cast<uint32_t *>(static_cast<char *>(ctx->pinned) + 1088);
    HIP_TRY(hipMemcpyAsync(h, &dvals[1], sizeof(double), hipMemcpyDeviceToHost, s), "pref copy");
    HIP_TRY(hipMemcpyAsync(hk, mm, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s), "bounds copy");
    HIP_TRY(hipMemcpyAsync(hflag, ctx->dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s), "finite check");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (*hflag) return set_err(ctx, APX_EINVAL, "X or pref_vec holds a NaN or infinite value");
    const uint32_t key_pinf = 0xff800000u, key_ninf = 0x007fffffu;   // fkey(+inf), fkey(-inf)
    if (hk[1] >= key_pinf || hk[0] <= key_ninf)
        return set_err(ctx, APX_EINVAL, "similarities overflow FP32 (S holds non-finite values)");
    if (pref_out) *pref_out = pref_mode == APX_PREF_VECTOR ? NAN : *h;
    return APX_OK;
}

// ---- matrix-free similarity: the row panels of ap_solve_mf -----------------
namespace apx {

size_t mf_sim_bytes(int64_t n) { return sim_layout(n).bytes; }

namespace {
struct MfPtrs {
    float *nrm;
    uint32_t *mm;
    SelState *sel;
    unsigned long long *hist;
    double *dvals;   // [0] range, [1] preference
};
MfPtrs mf_ptrs(const MfSim &m) {
    const SimLayout L = sim_layout(m.n);
    MfPtrs q;
    q.nrm = reinterpret_cast<float *>(m.ws + L.o_n);
    q.mm = reinterpret_cast<uint32_t *>(m.ws + L.o_mm);
    q.sel = reinterpret_cast<SelState *>(m.ws + L.o_sel);
    q.hist = reinterpret_cast<unsigned long long *>(m.ws + L.o_h);
    q.dvals = reinterpret_cast<double *>(m.ws + L.o_r);
    return q;
}
PanelArgs panel_args(const MfSim &m, const MfPtrs &q, float *panel, int64_t ld, int64_t p0, int64_t p1, int final,
                     const ApState *st) {
    PanelArgs a{};
    a.X = m.X;
    a.n = m.n;
    a.d = m.d;
    a.ldx = m.ldx;
    a.nrm = q.nrm;
    a.Sp = panel;
    a.ld = ld;
    a.p0 = p0;
    a.p1 = p1;
    a.final = final;
    a.pa = PrefArgs{nullptr, m.n, ld, m.pref_mode, m.pref_vec, m.pref_scalar, q.sel, q.mm, m.seed, m.noise_rel,
                    &q.dvals[1]};
    a.range = &q.dvals[0];
    a.minmax = q.mm;
    a.st = st;
    return a;
}
hipError_t launch_panel(const PanelArgs &a, hipStream_t s) {
    const int64_t tiles = ((a.p1 - a.p0 + BM - 1) / BM) * ((a.n + BM - 1) / BM);
    k_sim_panel<<<(unsigned)tiles, NT, 0, s>>>(a);
    return hipGetLastError();
}
}  // namespace

const double *mf_sim_pref(const MfSim &m) { return &mf_ptrs(m).dvals[1]; }
const uint32_t *mf_sim_bounds(const MfSim &m) { return mf_ptrs(m).mm; }

// Norms, the bounds of the off-diagonal entries, the median (three digit
// sweeps of the upper triangle, one panel at a time) and the range of S with
// the preferences: what ap_similarity derives from the stored S.
hipError_t mf_sim_setup(const MfSim &m, float *panel, int64_t ld, int64_t prows, hipStream_t s) {
    const MfPtrs q = mf_ptrs(m);
    const int64_t n = m.n;
    const unsigned long long M = (unsigned long long)n * (unsigned long long)(n - 1) / 2ull;
    const unsigned long long lo = (M % 2) ? (M - 1) / 2 : M / 2 - 1;
    const unsigned long long hi = (M % 2) ? (M - 1) / 2 : M / 2;
    k_sel_init<<<1, 256, 0, s>>>(q.sel, q.mm, lo, hi, q.hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sqnorm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(m.X, n, m.d, m.ldx, q.nrm);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int sweeps = m.pref_mode == APX_PREF_MEDIAN ? 3 : 1;
    for (int pass = 0; pass < sweeps; ++pass) {
        for (int64_t p0 = 0; p0 < n; p0 += prows) {
            const int64_t p1 = p0 + prows < n ? p0 + prows : n;
            if ((e = launch_panel(panel_args(m, q, panel, ld, p0, p1, 0, nullptr), s)) != hipSuccess) return e;
            if (m.pref_mode == APX_PREF_MEDIAN) {
                const size_t lds = sizeof(uint32_t) * (pass == 0 ? 8192 : 2 * (pass == 1 ? 1024 : 512));
                const int g = walk_grid((const void *)k_sel_hist, lds, p1 - p0);
                k_sel_hist<<<g, 256, lds, s>>>(panel - p0 * ld, n, ld, q.sel, pass, q.hist, p0, p1);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
        }
        if (m.pref_mode == APX_PREF_MEDIAN) {
            k_sel_pick<<<1, 256, 0, s>>>(q.sel, pass, q.hist);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    const PanelArgs a = panel_args(m, q, panel, ld, 0, 0, 1, nullptr);
    k_pref_range<<<1, 256, 0, s>>>(a.pa, &q.dvals[0]);
    return hipGetLastError();
}

hipError_t mf_sim_panel(const MfSim &m, float *panel, int64_t ld, int64_t p0, int64_t p1, const ApState *st,
                        hipStream_t s) {
    return launch_panel(panel_args(m, mf_ptrs(m), panel, ld, p0, p1, 1, st), s);
}

}  // namespace apx
