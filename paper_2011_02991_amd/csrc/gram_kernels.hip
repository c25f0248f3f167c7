// gram_kernels.hip -- the Gram matrix of the explicit derivative states, on
// the matrix cores (MFMA, FP64).
//
// The derivative-state variant of the metric (appendix: every derivative state
// prepared and kept, then all (P^2 + P)/2 inner products) ends with Q = P + 1
// states X_0 = lambda* (the forward state in the sweeps' final frame) and
// X_{1+s} = the swept derivative state of column s, stored one after another
// (each 2^n complex amplitudes, i.e. K = 2^(n+1) interleaved reals).  Every
// inner product <X_a|X_b> is then one entry of a dense contraction over K:
//   Re <X_a|X_b> = sum_k x_a[k] x_b[k]                 (mode 0),
//   Im <X_a|X_b> = sum_k x_a[k] (J x_b)[k]              (mode 1),
// with (J x)[2j] = x[2j+1], (J x)[2j+1] = -x[2j] (complex multiplication by -i
// read as reals).  That is a symmetric (mode 0) or antisymmetric (mode 1) K x Q
// by Q x K product with K far larger than Q, computed here with
// v_mfma_f64_16x16x4_f64: every product is formed in FP64 (complex64 states
// are converted, exactly, when a tile is staged) and accumulated in FP64.
// When the states are kept a chunk of columns at a time, the same kernel takes
// one chunk with lambda* and column 0 (symmetric) or two chunks against each
// other (rectangular: every pair of a state of each), with the columns of each
// operand's positions passed along, so the entries land where they belong.
//
// Work split: the Q columns are cut into tiles of 64; a work-group owns one
// pair of tiles (ta <= tb, or a tile of each operand) and one chunk of K,
// stages 32 reals of each of its 128 columns per step in LDS (FP64) and
// accumulates a 64 x 64 block of the
// result in the MFMA accumulators (4 wavefronts, 32 x 32 each, as 2 x 2 MFMA
// blocks).  Pairs vary fastest over the work-groups, so the work-groups of one
// chunk run together and share its columns in the caches.  Each work-group
// writes its block to a partial buffer; k_gram_reduce adds the chunks of every
// entry in a fixed order (bitwise reproducible) and writes the raw metric
// entries in the layout of the recurrent method's raw L and T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "gram_kernels.hpp"

namespace qng {

namespace {

constexpr int kGramThreads = 256;
constexpr int kTile = 64;         // columns per tile
constexpr int kStep = 32;         // reals of K staged per step
constexpr int kPad = kStep + 1;   // LDS row stride in doubles: lanes on 16 columns hit distinct banks

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void tile_pair(int pair, int ntile, int &ta, int &tb) {
    ta = 0;
    while (pair >= ntile - ta) {
        pair -= ntile - ta;
        ++ta;
    }
    tb = ta + pair;
}

// An operand's states on the device (see GramSet): position q at p1 + q *
// stride below n1, else at p2 + (q - n1) * stride.
template <typename R> struct DevSet {
    const R *p1, *p2;
    int n1, n;
};
template <typename R>
__device__ __forceinline__ const R *state_ptr(const DevSet<R> &s, int q, uint64_t stride) {
    return q < s.n1 ? s.p1 + (uint64_t)q * stride : s.p2 + (uint64_t)(q - s.n1) * stride;
}

// Eight consecutive reals of position q from real k (k a multiple of 8), as
// FP64; zeros past the last position or past K (K = 2^(n+1) is a multiple of
// 8 from n = 2 on; below that the tail is read element by element).
__device__ __forceinline__ void load8(const DevSet<float> &s, uint64_t stride, int q, uint64_t k, uint64_t K,
                                      double (&v)[8]) {
    if (q < s.n && k + 8 <= K) {
        const float4 *p = (const float4 *)(state_ptr(s, q, stride) + k);
        const float4 a = p[0], b = p[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (q < s.n && k + j < K) ? (double)state_ptr(s, q, stride)[k + j] : 0.0;
    }
}
__device__ __forceinline__ void load8(const DevSet<double> &s, uint64_t stride, int q, uint64_t k, uint64_t K,
                                      double (&v)[8]) {
    if (q < s.n && k + 8 <= K) {
        const double2 *p = (const double2 *)(state_ptr(s, q, stride) + k);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double2 a = p[j];
            v[2 * j] = a.x;
            v[2 * j + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (q < s.n && k + j < K) ? state_ptr(s, q, stride)[k + j] : 0.0;
    }
}

// A, B: the operands (B read only when rect), K reals per state, states
// `stride` reals apart.  kc: reals per chunk (a multiple of kStep).  rect: the
// tile pairs are every (ta, tb) of A's ntA and B's ntB tiles; else the pairs
// ta <= tb of A's.  partials: [chunk][pair][64][64] doubles.
template <typename R>
__global__ __launch_bounds__(kGramThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_gram(
    const DevSet<R> A, const DevSet<R> B, bool rect, uint64_t stride, uint64_t K, uint64_t kc, int ntA, int ntB,
    int npairs, int mode, bool nchunks_xcd, double *__restrict__ partials) {
    __shared__ double sA[kTile * kPad];
    __shared__ double sB[kTile * kPad];
    // Work-groups are dealt to the 8 XCDs round robin (work-group b runs on XCD
    // b mod 8).  All tile pairs of one chunk go to one XCD, so the work-groups
    // reading the same columns of a chunk share that XCD's L2: XCD x takes
    // chunks x, x + 8, x + 16, ... (nchunks is a multiple of 8 when above 8).
    int pair, chunk;
    if (nchunks_xcd) {
        const unsigned b = blockIdx.x, xcd = b & 7u, local = b >> 3;
        pair = (int)(local % (unsigned)npairs);
        chunk = (int)((local / (unsigned)npairs) * 8u + xcd);
    } else {
        pair = (int)(blockIdx.x % (unsigned)npairs);
        chunk = (int)(blockIdx.x / (unsigned)npairs);
    }
    int ta, tb;
    if (rect) {
        ta = pair / ntB;
        tb = pair % ntB;
    } else {
        tile_pair(pair, ntA, ta, tb);
    }
    // (field by field: a reference chosen between the two arguments would put
    // them in scratch memory)
    const DevSet<R> SB{rect ? B.p1 : A.p1, rect ? B.p2 : A.p2, rect ? B.n1 : A.n1, rect ? B.n : A.n};
    const bool same = !rect && ta == tb && mode == 0;   // one tile serves both operands
    const double *sBv = same ? sA : sB;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;   // this wave's 32 x 32 quarter of the block
    const int lcol = tid >> 2, part = tid & 3;  // staging: column lcol, reals part*8 .. part*8+7 of the step

    d4 acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
    const uint64_t kbeg = (uint64_t)chunk * kc;
    const uint64_t kend = kbeg + kc < K ? kbeg + kc : K;
    // the next step's reals are loaded into registers while the current step's
    // MFMAs run, then written to LDS between the two barriers
    double va[8], vb[8];
    load8(A, stride, ta * kTile + lcol, kbeg + part * 8, K, va);
    if (!same) load8(SB, stride, tb * kTile + lcol, kbeg + part * 8, K, vb);
    for (uint64_t k0 = kbeg; k0 < kend; k0 += kStep) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sA[lcol * kPad + part * 8 + j] = va[j];
        if (!same) {
            if (mode == 1) {
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const double re = vb[j], im = vb[j + 1];
                    vb[j] = im;
                    vb[j + 1] = -re;
                }
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) sB[lcol * kPad + part * 8 + j] = vb[j];
        }
        __syncthreads();
        const uint64_t kn = k0 + kStep;
        if (kn < kend) {
            load8(A, stride, ta * kTile + lcol, kn + part * 8, K, va);
            if (!same) load8(SB, stride, tb * kTile + lcol, kn + part * 8, K, vb);
        }
        // A(row = lane % 16, k = lane / 16), B(k = lane / 16, col = lane % 16)
        const int r0 = wr * 32 + (lane & 15), c0 = wc * 32 + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < kStep; kk += 4) {
            const int kl = kk + (lane >> 4);
            const double a0 = sA[r0 * kPad + kl], a1 = sA[(r0 + 16) * kPad + kl];
            const double b0 = sBv[c0 * kPad + kl], b1 = sBv[(c0 + 16) * kPad + kl];
            acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
            acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
            acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
            acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
        }
        __syncthreads();
    }
    // D(row = 4 i + lane / 16, col = lane % 16) of each 16 x 16 block (item i of
    // the accumulator)
    double *out = partials + ((uint64_t)chunk * npairs + pair) * (kTile * kTile);
    const int rr = wr * 32 + (lane >> 4), cc = wc * 32 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        out[(rr + 4 * i) * kTile + cc] = acc00[i];
        out[(rr + 4 * i) * kTile + cc + 16] = acc01[i];
        out[(rr + 16 + 4 * i) * kTile + cc] = acc10[i];
        out[(rr + 16 + 4 * i) * kTile + cc + 16] = acc11[i];
    }
}

// Positions and columns of an operand (see GramSet).
struct SetCols {
    int n1, n, col1, col2;
};
__device__ __forceinline__ int column_of(const SetCols &s, int q) { return q < s.n1 ? s.col1 + q : s.col2 + q - s.n1; }

// One thread per entry of a computed block: the chunks' partials summed in
// order, times sign[ca + 1] sign[cb + 1] (each kept state is its column's
// derivative state up to a known sign), and the entry of columns ca < cb goes
// to the raw metric: ca = -1 -> T of column cb, else L of (ca, cb); the real
// part (mode 0) or the imaginary part (mode 1) of the complex result.
__global__ void k_gram_reduce(const double *__restrict__ partials, int npairs, int nchunks, bool rect, int ntA,
                              int ntB, SetCols A, SetCols B, int P, int mode, const int8_t *__restrict__ sign,
                              double *__restrict__ lraw, double *__restrict__ traw) {
    const uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)npairs * kTile * kTile) return;
    const int pair = (int)(idx / (kTile * kTile));
    const int e = (int)(idx % (kTile * kTile));
    int ta, tb;
    if (rect) {
        ta = pair / ntB;
        tb = pair % ntB;
    } else {
        tile_pair(pair, ntA, ta, tb);
    }
    const SetCols SB{rect ? B.n1 : A.n1, rect ? B.n : A.n, rect ? B.col1 : A.col1, rect ? B.col2 : A.col2};
    const int qa = ta * kTile + e / kTile, qb = tb * kTile + e % kTile;
    if (qa >= A.n || qb >= SB.n || (!rect && qa >= qb)) return;
    const int ca = column_of(A, qa), cb = column_of(SB, qb);
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partials[((uint64_t)c * npairs + pair) * (kTile * kTile) + e];
    if (sign[ca + 1] != sign[cb + 1]) s = -s;
    double *dst = ca < 0 ? traw + 2 * (uint64_t)cb : lraw + 2 * ((uint64_t)ca * P + cb);
    dst[mode] = s;
}

inline void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

struct GramShape {
    int ntA, ntB, npairs, nchunks;
    uint64_t K, kc;
};

GramShape gram_shape(int n, int QA, int QB) {
    GramShape g;
    g.ntA = (QA + kTile - 1) / kTile;
    g.ntB = QB > 0 ? (QB + kTile - 1) / kTile : g.ntA;
    g.npairs = QB > 0 ? g.ntA * g.ntB : g.ntA * (g.ntA + 1) / 2;
    g.K = uint64_t(2) << n;
    // about 12288 work-groups in all, chunks a power of two of at least kStep
    // reals: short chunks keep the work-groups that share a tile at nearby
    // reals, so more of its re-reads hit the L2 (3072: 3 % slower at n = 26)
    uint64_t want = (12288 + (uint64_t)g.npairs - 1) / (uint64_t)g.npairs;
    uint64_t nch = 1;
    while (nch < want) nch <<= 1;
    while (nch > 1 && g.K / nch < (uint64_t)kStep) nch >>= 1;
    // partial sums within max(32 bytes per amplitude, 8 MiB): next to nothing
    // beside the states from 22 qubits on, and small registers stay small
    const uint64_t cap = std::max<uint64_t>(uint64_t(32) << n, uint64_t(8) << 20) / (kTile * kTile * sizeof(double));
    while (nch > 1 && nch * (uint64_t)g.npairs > cap) nch >>= 1;
    g.nchunks = (int)nch;
    g.kc = g.K / nch;
    if (g.kc < (uint64_t)kStep) g.kc = kStep;
    return g;
}

template <typename R> DevSet<R> dev_set(const GramSet &s) {
    return DevSet<R>{(const R *)s.p1, (const R *)s.p2, s.n1, s.n};
}

}  // namespace

size_t gram_partial_bytes(int n, int QA, int QB) {
    const GramShape g = gram_shape(n, QA, QB);
    return (size_t)g.nchunks * g.npairs * kTile * kTile * sizeof(double);
}

void launch_gram(const GramSet &A, const GramSet *B, bool complex64, int n, int P, int mode, const int8_t *sign,
                 double *partials, double *lraw, double *traw, hipStream_t st) {
    const bool rect = B != nullptr;
    if (rect ? (A.n < 1 || B->n < 1) : A.n < 2) return;
    const GramSet &Bs = rect ? *B : A;
    const GramShape g = gram_shape(n, A.n, rect ? Bs.n : 0);
    const uint64_t stride = g.K;
    const unsigned blocks = (unsigned)((uint64_t)g.npairs * g.nchunks);
    const bool xcd = g.nchunks % 8 == 0;
    if (complex64)
        hipLaunchKernelGGL(k_gram<float>, dim3(blocks), dim3(kGramThreads), 0, st, dev_set<float>(A),
                           dev_set<float>(Bs), rect, stride, g.K, g.kc, g.ntA, g.ntB, g.npairs, mode, xcd, partials);
    else
        hipLaunchKernelGGL(k_gram<double>, dim3(blocks), dim3(kGramThreads), 0, st, dev_set<double>(A),
                           dev_set<double>(Bs), rect, stride, g.K, g.kc, g.ntA, g.ntB, g.npairs, mode, xcd, partials);
    check_launch();
    const uint64_t entries = (uint64_t)g.npairs * kTile * kTile;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((entries + 255) / 256)), dim3(256), 0, st, partials, g.npairs,
                       g.nchunks, rect, g.ntA, g.ntB, SetCols{A.n1, A.n, A.col1, A.col2},
                       SetCols{Bs.n1, Bs.n, Bs.col1, Bs.col2}, P, mode, sign, lraw, traw);
    check_launch();
}

double gram_flops(int n, int QA, int QB) {
    const GramShape g = gram_shape(n, QA, QB);
    return 2.0 * (double)g.npairs * kTile * kTile * (double)g.K;
}

}  // namespace qng
