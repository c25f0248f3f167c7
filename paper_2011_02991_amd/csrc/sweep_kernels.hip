// sweep_kernels.hip -- the fused sweep-pass kernel for gfx950 (see sweep.hpp).
//
// One work-group of 256 threads (4 wave64) owns one tile: the 2^m amplitudes
// of lambda (A) and of the W phi registers (B; W = 1, or 2 for a block of two
// columns sharing lambda) whose indices agree outside the pass's m tile
// qubits.  The tile lives in registers: every thread holds T = 2^RB amplitudes
// of each register, in the register precision CT (FP64 for complex128
// storage; FP32 or FP64 for complex64 storage).  A thread mapping says which
// local bits are "register bits" (the thread's own T amplitudes differ in
// them) and which are "thread bits" (bits of the thread index).
//
// The operations of a pass are interpreted from a list of device op codes
// (sweep.hpp): the register position, the Pauli axis and where a control or a
// Z bit lives are resolved on the host, so every code runs one straight-line
// path with its register indices fixed at compile time.
//
//  * Load: amplitudes go from HBM straight into registers under the pass's
//    load mapping, whose lowest thread bits are the lowest qubits, so the 64
//    lanes of a wave read contiguous runs.
//  * X/Y rotations, X/Y inner products and CNOT targets act on register bits:
//    the pair (i, i ^ 2^j) of one thread, no communication, no barrier.
//  * Diagonal operations (RZ, CZ, Z inner products) act on any bit: its value
//    comes from the register index, the thread index or the tile base.
//  * Between phases the tile is exchanged through LDS (one register at a time)
//    to the next mapping, the only place where barriers are needed.
//  * Inner products: each thread's share (register precision, then FP64) is
//    summed within each 16-lane row with DPP exchanges and across the
//    wavefront's rows with two lane exchanges, kept per (slot, wavefront) in
//    LDS; at the end one FP64 partial per (slot, tile) is written, and
//    k_reduce_tasks adds the partials of a slot over the tiles in a fixed
//    order (bitwise reproducible).
//  * Store: registers -> HBM under the final mapping (lanes on the lowest
//    qubits again), in place: the tile is touched by this work-group only.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sweep.hpp"

namespace qng {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename R> struct Amp;
template <> struct Amp<double> { using T = double2; };
template <> struct Amp<float>  { using T = float2; };

constexpr int kRows = kThreads / 16;   // DPP rows of 16 lanes per work-group

// v + (v of lane l ^ 16) in every lane, by v_permlane16_swap (gfx950: odd rows
// of the first operand trade places with even rows of the second).  With both
// operands holding v, the two results hold v of rows (0, 0, 2, 2) and of rows
// (1, 1, 3, 3), so their sum is the pair sum; the same with v_permlane32_swap
// (upper half against lower half) gives lane l ^ 32.  Both are VALU moves, so
// the sum needs no LDS round trip.
template <bool HALVES>
__device__ __forceinline__ double pair_sum(double v) {
    const uint32_t lo = __double2loint(v), hi = __double2hiint(v);
    if constexpr (HALVES) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
    }
}

// Sum of a value over the four 16-lane rows of the wavefront (lane l with
// l ^ 16, then l ^ 32): every lane l then holds the sum of lane l mod 16 of
// every row, added in the same order on every lane.
__device__ __forceinline__ double across_rows(double v) {
    v = pair_sum<false>(v);
    return pair_sum<true>(v);
}

// Row reduction with DPP: after row_shr by 1, 2, 4 and 8 (zero shifted in at
// the start of each 16-lane row), lane 15 of every row holds the row's sum.
template <int CTRL>
__device__ __forceinline__ double dpp_shifted(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ void row_sum(double &a, double &b) {
    a += dpp_shifted<0x111>(a);
    b += dpp_shifted<0x111>(b);
    a += dpp_shifted<0x112>(a);
    b += dpp_shifted<0x112>(b);
    a += dpp_shifted<0x114>(a);
    b += dpp_shifted<0x114>(b);
    a += dpp_shifted<0x118>(a);
    b += dpp_shifted<0x118>(b);
}

// LDS layout of the sweep kernel: the exchange buffer [2^m] (at least the
// kMaxBlockWidth x kWaves tile sums <lambda|phi_b>, which use its start while
// no exchange runs: both sit between barriers), one sink entry per thread,
// the per-wavefront partials of the inner products [kMaxSlots][kWaves].
constexpr int kLdsTailEntries = kThreads + kMaxSlots * kWaves;
template <typename CX> __host__ __device__ constexpr size_t xbuf_bytes(int m) {
    return ((size_t)1 << m) * sizeof(CX) > (size_t)kMaxBlockWidth * kWaves * 16
               ? ((size_t)1 << m) * sizeof(CX)
               : (size_t)kMaxBlockWidth * kWaves * 16;
}

// Store a per-lane partial of slot `slot` of `dst`: one value per wavefront.
// Every lane stores (lane 15 of the wavefront's first row to the slot, the
// others to the sink), so the op loop has no divergent branch.
__device__ __forceinline__ void row_store(double2 *sink, double2 *dst, int slot, int tid, double a, double b) {
    row_sum(a, b);
    a = across_rows(a);
    b = across_rows(b);
    double2 *p = ((tid & 63) == 15) ? dst + slot * kWaves + (tid >> 6) : sink;
    *p = make_double2(a, b);
}

// The inner products pr[b], pi[b] of the W phi registers, summed over each
// wavefront (16-lane rows, then across the rows) and stored, the active ones
// (b >= fa) to slot slot + b - fa, the others to the sink.  The sums use halving exchanges: lanes pair up across the
// row (DPP row_mirror: lane i with 15 - i; row_half_mirror: i with i ^ 7
// inside each half; quad_perm: i ^ 2, then i ^ 1), and in the first steps a
// lane keeps half of its values and sends the other half, which its partner
// keeps, so the values to exchange halve at each step.  At the end each
// quarter (W = 2) or half (W = 1) of the row holds one of the sums.
template <int CTRL>
__device__ __forceinline__ double dpp_xchg(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141, kDppXor2 = 0x4E, kDppXor1 = 0xB1;

// Built with QNG_REAL_PRODUCTS = 1 (sweep_kernels_real.hip), the metric's
// inner products keep their real parts only (the natural-gradient step needs
// Re G alone): half the multiply-adds and half the row sums; the imaginary
// parts are stored as zero.  The products that give T (column seeds) and the
// Z products on qubits outside the tile stay complex.
#ifndef QNG_REAL_PRODUCTS
#define QNG_REAL_PRODUCTS 0
#endif
constexpr bool kRealProducts = QNG_REAL_PRODUCTS != 0;

template <int W>
__device__ __forceinline__ void row_reduce_store(double2 *sink, double2 *red, int slot, int fa, int tid,
                                                 const double (&pr)[W], const double (&pi)[W]) {
    static_assert(W == 1 || W == 2 || W == 4, "one, two or four phi registers");
    const int lane = tid & 15;
    const bool h8 = lane & 8;
    if constexpr (W == 4) {
        // lanes 0-7 keep registers 0 and 1, lanes 8-15 registers 2 and 3; then
        // each quarter of the row one register (real and imaginary parts
        // together when complex), then (complex) the lower pair of each
        // quarter the real part
        const bool h4 = lane & 4;
        const double a = (h8 ? pr[2] : pr[0]) + dpp_xchg<kDppRowMirror>(h8 ? pr[0] : pr[2]);
        const double b = (h8 ? pr[3] : pr[1]) + dpp_xchg<kDppRowMirror>(h8 ? pr[1] : pr[3]);
        double v;
        int part = 0;
        if constexpr (kRealProducts) {
            v = (h4 ? b : a) + dpp_xchg<kDppRowHalfMirror>(h4 ? a : b);
            v += dpp_xchg<kDppXor2>(v);
        } else {
            const double ai = (h8 ? pi[2] : pi[0]) + dpp_xchg<kDppRowMirror>(h8 ? pi[0] : pi[2]);
            const double bi = (h8 ? pi[3] : pi[1]) + dpp_xchg<kDppRowMirror>(h8 ? pi[1] : pi[3]);
            const double re = (h4 ? b : a) + dpp_xchg<kDppRowHalfMirror>(h4 ? a : b);
            const double im = (h4 ? bi : ai) + dpp_xchg<kDppRowHalfMirror>(h4 ? ai : bi);
            // i ^ 2 pairs lanes of one quarter: the lower pair keeps re, the upper im
            const bool h2 = lane & 2;
            v = (h2 ? im : re) + dpp_xchg<kDppXor2>(h2 ? re : im);
            part = h2 ? 1 : 0;
        }
        v += dpp_xchg<kDppXor1>(v);
        v = across_rows(v);
        // quarter q of the row holds register q (h8 picks the pair, then h4 within it)
        const int reg = (lane >> 3) * 2 + ((lane >> 2) & 1);
        const bool keep = reg >= fa;
        if constexpr (kRealProducts) {
            const bool last = (lane & 3) == 3 && (tid & 63) < 16;
            double2 *p = (last && keep) ? &red[(slot + reg - fa) * kWaves + (tid >> 6)] : sink;
            *p = make_double2(v, 0.0);
        } else {
            const bool last = (lane & 1) == 1 && (tid & 63) < 16;
            double *p = (last && keep) ? &red[(slot + reg - fa) * kWaves + (tid >> 6)].x + part : (double *)sink;
            *p = v;
        }
        return;
    } else {
        if constexpr (kRealProducts) {
            // W = 1: every lane ends with the row's sum; W = 2: lanes 0-7 with
            // register 0's, lanes 8-15 with register 1's
            double v = W == 1 ? pr[0] : (h8 ? pr[W - 1] : pr[0]) + dpp_xchg<kDppRowMirror>(h8 ? pr[0] : pr[W - 1]);
            if constexpr (W == 1) v += dpp_xchg<kDppRowMirror>(v);
            v += dpp_xchg<kDppRowHalfMirror>(v);
            v += dpp_xchg<kDppXor2>(v);
            v += dpp_xchg<kDppXor1>(v);
            v = across_rows(v);
            const int b = W == 1 ? 0 : lane >> 3;
            const bool last = (lane & 7) == 7 && (tid & 63) < 16;
            const bool keep = W == 1 ? lane == 15 : b >= fa;
            double2 *p = (last && keep) ? &red[(slot + b - fa) * kWaves + (tid >> 6)] : sink;
            *p = make_double2(v, 0.0);
            return;
        }
        double v;
        if constexpr (W == 1) {
            // lanes 0-7 keep the real part, lanes 8-15 the imaginary part
            v = (h8 ? pi[0] : pr[0]) + dpp_xchg<kDppRowMirror>(h8 ? pr[0] : pi[0]);
        } else {
            // lanes 0-7 keep register 0's pair, lanes 8-15 register 1's ...
            const double a = (h8 ? pr[1] : pr[0]) + dpp_xchg<kDppRowMirror>(h8 ? pr[0] : pr[1]);
            const double b = (h8 ? pi[1] : pi[0]) + dpp_xchg<kDppRowMirror>(h8 ? pi[0] : pi[1]);
            // ... then the lower quarter of each half the real part
            const bool h4 = lane & 4;
            v = (h4 ? b : a) + dpp_xchg<kDppRowHalfMirror>(h4 ? a : b);
        }
        if constexpr (W == 1) v += dpp_xchg<kDppRowHalfMirror>(v);
        v += dpp_xchg<kDppXor2>(v);
        v += dpp_xchg<kDppXor1>(v);
        v = across_rows(v);
        // W = 1: lane 7 holds the real sum, lane 15 the imaginary one; W = 2: lanes
        // 3, 7 hold register 0's, lanes 11, 15 register 1's (those of the
        // wavefront's first row store the wavefront's sums)
        const int b = W == 1 ? 0 : lane >> 3;
        const bool last = (W == 1 ? (lane & 7) == 7 : (lane & 3) == 3) && (tid & 63) < 16;
        const bool keep = W == 1 || b >= fa;
        const int part = W == 1 ? lane >> 3 : (lane >> 2) & 1;
        double *p = (last && keep) ? &red[(slot + b - fa) * kWaves + (tid >> 6)].x + part : (double *)sink;
        *p = v;
    }
}

// The tile is kept as four arrays of T scalars per thread: real and imaginary
// parts of lambda (A) and phi (B), indexed only by compile-time constants, so
// every element is a register of its own.  With the one-hot handler dispatch
// each element stays in one register through the whole op loop; as short
// vectors, the CNOT handlers of the T=16 tile rebuilt whole vectors (a copy of
// the tile per op).
template <typename CT, int T, int W>
struct Regs {
    CT ar[T], ai[T];           // lambda
    CT br[W > 0 ? W : 1][T], bi[W > 0 ? W : 1][T];     // phi registers (W = 0: none; HIP has no empty arrays)
};

// 2x2 complex matrix entries of the gate table in the register precision
// (row-major: a, b / c, d as re, im).
template <typename CT>
__device__ __forceinline__ CT mat_entry(const CT *__restrict__ mt, int gate, int k) {
    return mt[(size_t)gate * 8 + k];
}

// ------------------------------------------------------- inner products
//
// A thread's share of a product (its T amplitudes, two chains of fused
// multiply-adds) is formed in the register precision CT and converted to FP64
// once; every sum beyond the thread (row, work-group, tiles, launches) is
// FP64.  Built with QNG_EXACT_PRODUCTS = 1 (sweep_kernels_exact.hip), the
// share is formed in FP64 from the register values (each product of two FP32
// values exact) instead.  For FP32 registers this rounds each term relative to the thread's
// own partial, a few units of 2^-24 of a sum of T = 16 terms, which is far
// below what storing the state in FP32 already costs (the state is rounded
// at every gate), and it spares converting every register value to FP64 for
// each product.  The first term of a chain is a plain product, so no chain
// starts from zero.

#ifndef QNG_EXACT_PRODUCTS
#define QNG_EXACT_PRODUCTS 0
#endif
template <typename CT> using ProdT = typename std::conditional<QNG_EXACT_PRODUCTS != 0, double, CT>::type;

__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __fma_rn(a, b, c); }

// acc = (first ? 0 : acc) + conj(a) b, with signs sa on the whole term; the
// operands are taken in the accumulator's precision A
template <typename T> using AccArg = typename std::common_type<T>::type;   // not deduced
template <bool FIRST, bool NEG, typename A>
__device__ __forceinline__ void cfma(A &r, A &i, AccArg<A> ar, AccArg<A> ai, AccArg<A> br, AccArg<A> bi) {
    const A s = NEG ? A(-1) : A(1);
    if (FIRST) {
        r = (s * ar) * br;
        i = (s * ar) * bi;
    } else {
        r = fma_rn(s * ar, br, r);
        i = fma_rn(s * ar, bi, i);
    }
    r = fma_rn(s * ai, bi, r);
    i = fma_rn(-s * ai, br, i);
}

// X: sum over pairs of conj(a0) b1 + conj(a1) b0.
// Y: i * sum over pairs of (conj(a1) b0 - conj(a0) b1).
// (<A|X|B> and <A|Y|B> on register bit J; Y = [[0, -i], [i, 0]].)
template <int J, int AX, int T, typename CT>
__device__ __forceinline__ void prod_xy(const CT (&ar)[T], const CT (&ai)[T], const CT (&br)[T], const CT (&bi)[T],
                                        double &pr, double &pi) {
    ProdT<CT> r0 = 0, i0 = 0, r1 = 0, i1 = 0;
    int pair = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);
        const ProdT<CT> a0r = ar[i], a0i = ai[i], a1r = ar[k], a1i = ai[k];
        const ProdT<CT> b0r = br[i], b0i = bi[i], b1r = br[k], b1i = bi[k];
        ProdT<CT> &r = (pair & 1) ? r1 : r0;
        ProdT<CT> &m = (pair & 1) ? i1 : i0;
        if (pair < 2) cfma<true, AX == 1>(r, m, a0r, a0i, b1r, b1i);
        else cfma<false, AX == 1>(r, m, a0r, a0i, b1r, b1i);
        cfma<false, false>(r, m, a1r, a1i, b0r, b0i);
        ++pair;
    }
    const double sr = (T >= 4) ? (double)r0 + (double)r1 : (double)r0;
    const double si = (T >= 4) ? (double)i0 + (double)i1 : (double)i0;
    if (AX == 0) {
        pr = sr;
        pi = si;
    } else {
        pr = -si;
        pi = sr;
    }
}

// Z on register bit J: sum_i (-1)^{bit J of i} conj(a_i) b_i
template <int J, int T, typename CT>
__device__ __forceinline__ void prod_z_reg(const CT (&ar)[T], const CT (&ai)[T], const CT (&br)[T],
                                           const CT (&bi)[T], double &pr, double &pi) {
    ProdT<CT> r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        ProdT<CT> &r = (i & 1) ? r1 : r0;
        ProdT<CT> &m = (i & 1) ? i1 : i0;
        const bool neg = (i >> J) & 1;
        if (i < 2) {
            if (neg) cfma<true, true>(r, m, ar[i], ai[i], br[i], bi[i]);
            else cfma<true, false>(r, m, ar[i], ai[i], br[i], bi[i]);
        } else {
            if (neg) cfma<false, true>(r, m, ar[i], ai[i], br[i], bi[i]);
            else cfma<false, false>(r, m, ar[i], ai[i], br[i], bi[i]);
        }
    }
    pr = (T >= 2) ? (double)r0 + (double)r1 : (double)r0;
    pi = (T >= 2) ? (double)i0 + (double)i1 : (double)i0;
}

// sum_i conj(a_i) b_i (the caller applies a sign common to all registers)
template <int T, typename CT>
__device__ __forceinline__ void prod_plain(const CT (&ar)[T], const CT (&ai)[T], const CT (&br)[T],
                                           const CT (&bi)[T], double &pr, double &pi) {
    ProdT<CT> r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        ProdT<CT> &r = (i & 1) ? r1 : r0;
        ProdT<CT> &m = (i & 1) ? i1 : i0;
        if (i < 2) cfma<true, false>(r, m, ar[i], ai[i], br[i], bi[i]);
        else cfma<false, false>(r, m, ar[i], ai[i], br[i], bi[i]);
    }
    pr = (T >= 2) ? (double)r0 + (double)r1 : (double)r0;
    pi = (T >= 2) ? (double)i0 + (double)i1 : (double)i0;
}

// Real parts only (QNG_REAL_PRODUCTS): Re(s conj(a) b) = s (a.x b.x + a.y b.y)
// and Im(s conj(a) b) = s (a.x b.y - a.y b.x), one chain each.
template <bool NEG, typename A>
__device__ __forceinline__ void cfma_re(A &r, AccArg<A> ar, AccArg<A> ai, AccArg<A> br, AccArg<A> bi) {
    r = fma_rn(NEG ? -ar : ar, br, r);
    r = fma_rn(NEG ? -ai : ai, bi, r);
}
template <bool NEG, typename A>
__device__ __forceinline__ void cfma_im(A &r, AccArg<A> ar, AccArg<A> ai, AccArg<A> br, AccArg<A> bi) {
    r = fma_rn(NEG ? -ar : ar, bi, r);
    r = fma_rn(NEG ? ai : -ai, br, r);
}

// The same products for every phi register of the tile at once, lambda's
// values converted once per pair for all of them.
template <int J, int AX, int T, typename CT, int W>
__device__ __forceinline__ void prodw_xy(const Regs<CT, T, W> &x, double (&pr)[W], double (&pi)[W]) {
    if constexpr (kRealProducts) {
        // X: the real part of sum conj(a0) b1 + conj(a1) b0; Y: minus the
        // imaginary part of sum -conj(a0) b1 + conj(a1) b0
        ProdT<CT> c0[W], c1[W];
#pragma unroll
        for (int b = 0; b < W; ++b) c0[b] = c1[b] = 0;
        int pair = 0;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i & (1 << J)) continue;
            const int k = i | (1 << J);
            const ProdT<CT> a0r = x.ar[i], a0i = x.ai[i], a1r = x.ar[k], a1i = x.ai[k];
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const ProdT<CT> b0r = x.br[b][i], b0i = x.bi[b][i], b1r = x.br[b][k], b1i = x.bi[b][k];
                ProdT<CT> &c = (pair & 1) ? c1[b] : c0[b];
                if (AX == 0) {
                    cfma_re<false>(c, a0r, a0i, b1r, b1i);
                    cfma_re<false>(c, a1r, a1i, b0r, b0i);
                } else {
                    cfma_im<true>(c, a0r, a0i, b1r, b1i);
                    cfma_im<false>(c, a1r, a1i, b0r, b0i);
                }
            }
            ++pair;
        }
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const double v = (double)c0[b] + (double)c1[b];
            pr[b] = AX == 0 ? v : -v;
            pi[b] = 0.0;
        }
        return;
    }
    ProdT<CT> r0[W], i0[W], r1[W], i1[W];
    int pair = 0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);
        const ProdT<CT> a0r = x.ar[i], a0i = x.ai[i], a1r = x.ar[k], a1i = x.ai[k];
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const ProdT<CT> b0r = x.br[b][i], b0i = x.bi[b][i], b1r = x.br[b][k], b1i = x.bi[b][k];
            ProdT<CT> &r = (pair & 1) ? r1[b] : r0[b];
            ProdT<CT> &m = (pair & 1) ? i1[b] : i0[b];
            if (pair < 2) cfma<true, AX == 1>(r, m, a0r, a0i, b1r, b1i);
            else cfma<false, AX == 1>(r, m, a0r, a0i, b1r, b1i);
            cfma<false, false>(r, m, a1r, a1i, b0r, b0i);
        }
        ++pair;
    }
#pragma unroll
    for (int b = 0; b < W; ++b) {
        const double sr = (T >= 4) ? (double)r0[b] + (double)r1[b] : (double)r0[b];
        const double si = (T >= 4) ? (double)i0[b] + (double)i1[b] : (double)i0[b];
        pr[b] = AX == 0 ? sr : -si;
        pi[b] = AX == 0 ? si : sr;
    }
}

template <int J, int T, typename CT, int W>
__device__ __forceinline__ void prodw_z_reg(const Regs<CT, T, W> &x, double (&pr)[W], double (&pi)[W]) {
    if constexpr (kRealProducts) {
        ProdT<CT> c0[W], c1[W];
#pragma unroll
        for (int b = 0; b < W; ++b) c0[b] = c1[b] = 0;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const ProdT<CT> ar = x.ar[i], ai = x.ai[i];
#pragma unroll
            for (int b = 0; b < W; ++b) {
                ProdT<CT> &c = (i & 1) ? c1[b] : c0[b];
                if ((i >> J) & 1) cfma_re<true>(c, ar, ai, x.br[b][i], x.bi[b][i]);
                else cfma_re<false>(c, ar, ai, x.br[b][i], x.bi[b][i]);
            }
        }
#pragma unroll
        for (int b = 0; b < W; ++b) {
            pr[b] = (double)c0[b] + (double)c1[b];
            pi[b] = 0.0;
        }
        return;
    }
    ProdT<CT> r0[W], i0[W], r1[W], i1[W];
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const ProdT<CT> ar = x.ar[i], ai = x.ai[i];
        const bool neg = (i >> J) & 1;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            ProdT<CT> &r = (i & 1) ? r1[b] : r0[b];
            ProdT<CT> &m = (i & 1) ? i1[b] : i0[b];
            if (i < 2) {
                if (neg) cfma<true, true>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
                else cfma<true, false>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
            } else {
                if (neg) cfma<false, true>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
                else cfma<false, false>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < W; ++b) {
        pr[b] = (T >= 2) ? (double)r0[b] + (double)r1[b] : (double)r0[b];
        pi[b] = (T >= 2) ? (double)i0[b] + (double)i1[b] : (double)i0[b];
    }
}

template <int T, typename CT, int W>
__device__ __forceinline__ void prodw_plain(const Regs<CT, T, W> &x, double (&pr)[W], double (&pi)[W]) {
    if constexpr (kRealProducts) {
        ProdT<CT> c0[W], c1[W];
#pragma unroll
        for (int b = 0; b < W; ++b) c0[b] = c1[b] = 0;
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const ProdT<CT> ar = x.ar[i], ai = x.ai[i];
#pragma unroll
            for (int b = 0; b < W; ++b) cfma_re<false>((i & 1) ? c1[b] : c0[b], ar, ai, x.br[b][i], x.bi[b][i]);
        }
#pragma unroll
        for (int b = 0; b < W; ++b) {
            pr[b] = (double)c0[b] + (double)c1[b];
            pi[b] = 0.0;
        }
        return;
    }
    ProdT<CT> r0[W], i0[W], r1[W], i1[W];
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const ProdT<CT> ar = x.ar[i], ai = x.ai[i];
#pragma unroll
        for (int b = 0; b < W; ++b) {
            ProdT<CT> &r = (i & 1) ? r1[b] : r0[b];
            ProdT<CT> &m = (i & 1) ? i1[b] : i0[b];
            if (i < 2) cfma<true, false>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
            else cfma<false, false>(r, m, ar, ai, x.br[b][i], x.bi[b][i]);
        }
    }
#pragma unroll
    for (int b = 0; b < W; ++b) {
        pr[b] = (T >= 2) ? (double)r0[b] + (double)r1[b] : (double)r0[b];
        pi[b] = (T >= 2) ? (double)i0[b] + (double)i1[b] : (double)i0[b];
    }
}

// The inner products <lambda|sigma|phi_b> of every phi register into
// pr[b], pi[b] (PROD(re_a, im_a, re_b, im_b, pr, pi) forms one), and their
// stores: the active registers fa .. W-1 into consecutive slots from `slot`,
// the others into the sink (no branch).
// The stores come after the op's tile update, as in the one-register kernel
// (its register allocation depends on that order).
// Built with QNG_NO_PRODUCTS = 1 (sweep_kernels_states.hip), the passes take
// no inner product at all: they only carry the registers through the adjoint
// gates and the in-pass seeds, for the variant that keeps every column's phi
// register as an explicit derivative state and forms the metric as their Gram
// matrix afterwards.
#ifndef QNG_NO_PRODUCTS
#define QNG_NO_PRODUCTS 0
#endif
constexpr bool kNoProducts = QNG_NO_PRODUCTS != 0;

// Each build names its kernel after its arithmetic, so kernel traces tell them
// apart: k_sweep_reg (complex products), k_sweep_reg_real (real parts),
// k_sweep_reg_exact / k_sweep_reg_real_exact (every product in FP64 from FP32
// registers), k_sweep_reg_states (no products).
#if QNG_NO_PRODUCTS
#define QNG_SWEEP_KERNEL k_sweep_reg_states
#elif QNG_REAL_PRODUCTS && QNG_EXACT_PRODUCTS
#define QNG_SWEEP_KERNEL k_sweep_reg_real_exact
#elif QNG_REAL_PRODUCTS
#define QNG_SWEEP_KERNEL k_sweep_reg_real
#elif QNG_EXACT_PRODUCTS
#define QNG_SWEEP_KERNEL k_sweep_reg_exact
#else
#define QNG_SWEEP_KERNEL k_sweep_reg
#endif
// waves per SIMD the FP32 kernels without products are held to (four: at most
// 128 VGPRs, a few values spill in the exchanges; three: 130 VGPRs, none)
#ifndef QNG_STATES_WAVES
#define QNG_STATES_WAVES 4
#endif

#define QNG_PRODS(PRODW)                                                                                     \
    double pr[W > 0 ? W : 1], pi[W > 0 ? W : 1];                                                             \
    if constexpr (!kNoProducts) { PRODW(x, pr, pi); }
#define QNG_STORE_PRODS()                                                                                    \
    if constexpr (!kNoProducts) row_reduce_store<W>(sink, red, slot, fa, tid, pr, pi)

// ------------------------------------------------------- gates on registers

// Every adjoint rotation is, on pairs of reals, the plane rotation
// [[c, s], [-s, c]] applied in place as three shears (u = s / (1 + c), w = -s;
// rotations with c < 0 arrive negated, a sign both registers share):
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename CT>
struct Pair {
    CT a, b;
};
template <typename CT>
__device__ __forceinline__ Pair<CT> shear3(CT a, CT b, CT u, CT w) {
    a = fmadd(u, b, a);
    b = fmadd(w, a, b);
    a = fmadd(u, b, a);
    return Pair<CT>{a, b};
}
// (A, B) <- shears of (A, B); A and B are register-vector elements
#define QNG_SHEAR(A, B, U, W)                   \
    do {                                        \
        const Pair<CT> r_ = shear3(A, B, U, W); \
        A = r_.a;                               \
        B = r_.b;                               \
    } while (0)

// Adjoint X/Y rotation on the pairs of register bit J of one register (re,
// im): RX on (re x0, im x1) and (re x1, im x0), RY on (re x0, re x1) and
// (im x0, im x1).
template <int J, int AX, int T, typename CT>
__device__ __forceinline__ void rot_xy1(CT (&re)[T], CT (&im)[T], CT u, CT w) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);
        if (AX == 0) {
            QNG_SHEAR(re[i], im[k], u, w);
            QNG_SHEAR(re[k], im[i], u, w);
        } else {
            QNG_SHEAR(re[i], re[k], u, w);
            QNG_SHEAR(im[i], im[k], u, w);
        }
    }
}
template <int J, int AX, int T, typename CT, int W>
__device__ __forceinline__ void rot_xy(Regs<CT, T, W> &x, CT u, CT w) {
    rot_xy1<J, AX, T, CT>(x.ar, x.ai, u, w);
#pragma unroll
    for (int b = 0; b < W; ++b) rot_xy1<J, AX, T, CT>(x.br[b], x.bi[b], u, w);
}

// RZ adjoint on register bit J: (re, im) of the |0> amplitude rotated by
// (u, w), of the |1> amplitude by (-u, -w)
template <int J, int T, typename CT, int W>
__device__ __forceinline__ void diag_reg(Regs<CT, T, W> &x, CT u, CT w) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const bool one = (i >> J) & 1;
        const CT ui = one ? -u : u, wi = one ? -w : w;
        QNG_SHEAR(x.ar[i], x.ai[i], ui, wi);
#pragma unroll
        for (int b = 0; b < W; ++b) QNG_SHEAR(x.br[b][i], x.bi[b][i], ui, wi);
    }
}

// one rotation for every register (bit held by the thread index or the tile base)
template <int T, typename CT, int W>
__device__ __forceinline__ void diag_all(Regs<CT, T, W> &x, CT u, CT w) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        QNG_SHEAR(x.ar[i], x.ai[i], u, w);
#pragma unroll
        for (int b = 0; b < W; ++b) QNG_SHEAR(x.br[b][i], x.bi[b][i], u, w);
    }
}

// value select (by-value operands keep the choice on registers, not on addresses)
template <typename R>
__device__ __forceinline__ R sel(bool c, R a, R b) {
    return c ? a : b;
}

// Swap of two register values in place (v_swap_b32 on each dword).  Every
// tile update of the op loop is then an in-place rewrite of each register
// (rotations and phases are shears, swaps exchange register contents), so the
// register allocator keeps one set of registers for the tile across the whole
// loop instead of copying it at every dispatch.  A conditional swap (CNOT with
// a control held by the thread index or the tile base) runs under a branch:
// lanes whose control is clear are masked off, so they keep their values.
__device__ __forceinline__ void swap_in_place(float &a, float &b) {
    asm("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap_in_place(double &a, double &b) {
    uint32_t alo = (uint32_t)__builtin_bit_cast(uint64_t, a), ahi = (uint32_t)(__builtin_bit_cast(uint64_t, a) >> 32);
    uint32_t blo = (uint32_t)__builtin_bit_cast(uint64_t, b), bhi = (uint32_t)(__builtin_bit_cast(uint64_t, b) >> 32);
    asm("v_swap_b32 %0, %1" : "+v"(alo), "+v"(blo));
    asm("v_swap_b32 %0, %1" : "+v"(ahi), "+v"(bhi));
    a = __builtin_bit_cast(double, (uint64_t)alo | ((uint64_t)ahi << 32));
    b = __builtin_bit_cast(double, (uint64_t)blo | ((uint64_t)bhi << 32));
}

// The pairs of register bit J whose bit K is set (K < 0: every pair) trade
// places in one register.
template <int J, int K, int T, typename CT>
__device__ __forceinline__ void swap_pairs(CT (&re)[T], CT (&im)[T]) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if ((i & (1 << J)) || (K >= 0 && !(i & (1 << K)))) continue;
        const int k = i | (1 << J);
        swap_in_place(re[i], re[k]);
        swap_in_place(im[i], im[k]);
    }
}

// dst <- src written into the register that holds dst (an opaque in-place
// move: a plain copy would let the compiler hand dst the register of src, and
// the tile would then need a second register set wherever the paths merge).
__device__ __forceinline__ void move_in_place(float &dst, float src) {
    asm("v_mov_b32 %0, %1" : "+v"(dst) : "v"(src));
}
__device__ __forceinline__ void move_in_place(double &dst, double src) {
    uint32_t dlo = (uint32_t)__builtin_bit_cast(uint64_t, dst), dhi = (uint32_t)(__builtin_bit_cast(uint64_t, dst) >> 32);
    const uint32_t slo = (uint32_t)__builtin_bit_cast(uint64_t, src), shi = (uint32_t)(__builtin_bit_cast(uint64_t, src) >> 32);
    asm("v_mov_b32 %0, %1" : "+v"(dlo) : "v"(slo));
    asm("v_mov_b32 %0, %1" : "+v"(dhi) : "v"(shi));
    dst = __builtin_bit_cast(double, (uint64_t)dlo | ((uint64_t)dhi << 32));
}

// CNOT adjoint (itself) with target register bit J and control register bit K:
// the pairs of bit J whose bit K is set trade places.
template <int J, int K, int T, typename CT, int W>
__device__ __forceinline__ void cnot_reg(Regs<CT, T, W> &x) {
    swap_pairs<J, K, T, CT>(x.ar, x.ai);
#pragma unroll
    for (int b = 0; b < W; ++b) swap_pairs<J, K, T, CT>(x.br[b], x.bi[b]);
}

// CNOT with target register bit J and a control common to all registers of
// the thread (thread bit or tile base): every pair of bit J trades places
// where the control is set.
template <int J, int T, typename CT, int W>
__device__ __forceinline__ void cnot_cond(Regs<CT, T, W> &x, bool control) {
    if (control) {
        swap_pairs<J, -1, T, CT>(x.ar, x.ai);
#pragma unroll
        for (int b = 0; b < W; ++b) swap_pairs<J, -1, T, CT>(x.br[b], x.bi[b]);
    }
}

// A DevOp read as four dwords (scalar loads need dword granularity) and its
// fields extracted with shifts.
struct OpD {
    uint32_t w0, w1;
    int32_t gate, aux;
    uint64_t hf;   // one-hot handler bit (sweep.hpp, HB_*)
    uint32_t h2;   // one-hot bit of the second word (HB2_*), or 0
    __device__ __forceinline__ int type() const { return (int)(w0 & 0xffu); }
    __device__ __forceinline__ uint8_t b0() const { return (uint8_t)((w0 >> 8) & 0xffu); }
    __device__ __forceinline__ uint8_t b1() const { return (uint8_t)((w0 >> 16) & 0xffu); }
    __device__ __forceinline__ int slot() const { return (int)(w1 & 0xffffu); }
    __device__ __forceinline__ uint8_t q0() const { return (uint8_t)((w1 >> 16) & 0xffu); }
    __device__ __forceinline__ uint8_t q1() const { return (uint8_t)(w1 >> 24); }
};

__device__ __forceinline__ OpD load_op(const DevOp *p) {
    const uint4 v = *reinterpret_cast<const uint4 *>(p);
    const uint4 h = *(reinterpret_cast<const uint4 *>(p) + 1);
    return OpD{v.x, v.y, (int32_t)v.z, (int32_t)v.w, (uint64_t)h.x | ((uint64_t)h.y << 32), h.z};
}

constexpr uint64_t hbit(int b) { return uint64_t(1) << b; }
constexpr uint64_t hbits(int b, int count) { return ((uint64_t(1) << count) - 1) << b; }

// The byte tables of a pass (tile qubits, qubits outside the tile) and of a
// thread mapping (local bit per position), read as dwords and kept as wide
// integers, so that a byte with a uniform index is a shift (no indexed array,
// which the compiler would place in scratch memory).
typedef unsigned __int128 u128;

__device__ __forceinline__ uint32_t byte_at(u128 v, int k) { return (uint32_t)(v >> (8 * k)) & 0xffu; }

__device__ __forceinline__ u128 wide(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    return (u128)a | ((u128)b << 32) | ((u128)c << 64) | ((u128)d << 96);
}

struct PassBytes {
    u128 tq;          // DevPass::tile_q[0..15]
    u128 rq0;         // DevPass::rest_q[0..15]
    uint64_t rq1;     // DevPass::rest_q[16..23]
    __device__ __forceinline__ uint32_t rest(int k) const {
        return k < 16 ? byte_at(rq0, k) : (uint32_t)(rq1 >> (8 * (k - 16))) & 0xffu;
    }
};
__device__ __forceinline__ PassBytes load_pass_bytes(const DevPass *pp) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(pp);
    PassBytes b;
    b.tq = wide(w[6], w[7], w[8], w[9]);
    b.rq0 = wide(w[10], w[11], w[12], w[13]);
    b.rq1 = (uint64_t)w[14] | ((uint64_t)w[15] << 32);
    return b;
}
struct MapBytes {
    u128 pos;         // DevMap::pos
};
__device__ __forceinline__ MapBytes load_map(const DevMap *mp) {
    const uint4 v = *reinterpret_cast<const uint4 *>(mp);
    return MapBytes{wide(v.x, v.y, v.z, v.w)};
}

// Global (element) offset of each of a thread's registers under a mapping.
template <int RB, int T>
__device__ __forceinline__ void global_offsets(const PassBytes &pb, const MapBytes &mp, int tbits, int tid,
                                               uint64_t base, uint64_t (&off)[T]) {
    uint64_t dth = base;
#pragma unroll
    for (int t = 0; t < kMaxTileQubits; ++t)
        if (t < tbits) dth |= (uint64_t)((tid >> t) & 1) << byte_at(pb.tq, (int)byte_at(mp.pos, RB + t));
    uint64_t u[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) u[j] = (uint64_t)1 << byte_at(pb.tq, (int)byte_at(mp.pos, j));
#pragma unroll
    for (int i = 0; i < T; ++i) {
        uint64_t d = dth;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if ((i >> j) & 1) d |= u[j];
        off[i] = d;
    }
}

// Exchange-buffer slot of an in-tile index: the index with its higher bit
// fields folded onto the low kSwizzleBits by XOR.  The map is linear over
// GF(2) and leaves the high bits alone, so it is a bijection of the tile, and
// a set of lanes whose tile positions fall in distinct classes modulo
// kSwizzleBits lands in distinct banks whichever positions the mapping gives
// them (without it, lanes on high tile positions all hit one bank).
#ifndef QNG_SWIZZLE_BITS
#define QNG_SWIZZLE_BITS 4
#endif
constexpr int kSwizzleBits = QNG_SWIZZLE_BITS;
__device__ __forceinline__ uint32_t swizzle(uint32_t l) {
    constexpr uint32_t mask = (1u << kSwizzleBits) - 1u;
    uint32_t f = l;
#pragma unroll
    for (int k = kSwizzleBits; k < kMaxTileQubits; k += kSwizzleBits) f ^= (l >> k) & mask;
    return f;
}

// Exchange-buffer slot of each of a thread's registers under a mapping: the
// swizzled local (in-tile) index.  The swizzle is linear and the register and
// thread bits are disjoint, so the slot is the XOR of the swizzled parts.
template <int RB, int T>
__device__ __forceinline__ void local_offsets(const MapBytes &mp, int tbits, int tid, uint32_t (&off)[T]) {
    uint32_t lth = 0;
#pragma unroll
    for (int t = 0; t < kMaxTileQubits; ++t)
        if (t < tbits) lth |= (uint32_t)((tid >> t) & 1) << byte_at(mp.pos, RB + t);
    lth = swizzle(lth);
    uint32_t u[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) u[j] = swizzle(1u << byte_at(mp.pos, j));
#pragma unroll
    for (int i = 0; i < T; ++i) {
        uint32_t l = lth;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if ((i >> j) & 1) l ^= u[j];
        off[i] = l;
    }
}

// Mask over registers (bit i for register i) of the value of a location: a
// register position, a thread position or a bit of the tile base.
template <int T>
__device__ __forceinline__ uint32_t loc_mask(uint8_t loc, uint8_t q, int tid, uint64_t base) {
    constexpr uint32_t all = (T >= 32) ? 0xffffffffu : ((1u << T) - 1u);
    if (loc < kLocThread) {
        uint32_t mask = 0;
#pragma unroll
        for (int i = 0; i < T; ++i) mask |= (uint32_t)((i >> loc) & 1) << i;
        return mask;
    }
    const uint32_t v = (loc == kLocBase) ? (uint32_t)((base >> q) & 1u) : (uint32_t)((tid >> (loc & 15)) & 1);
    return v ? all : 0u;
}

// ------------------------------------------------------- op handlers
//
// Each op carries one handler bit; the op loop tests it group by group, then
// register bit by register bit, then kind by kind (independent tests, nested),
// so an op costs about a dozen scalar tests and every handler is a
// straight-line update of the tile in place.

constexpr uint64_t rot_bits(int j) {
    return hbit(HB_ROT_X + j) | hbit(HB_ROT_Y + j) | hbit(HB_PRODROT_X + j) | hbit(HB_PRODROT_Y + j);
}
constexpr uint64_t diag_bits(int j) { return hbit(HB_DIAG_REG + j) | hbit(HB_PRODDIAG_REG + j); }
constexpr uint64_t cnot_uni_bits(int j) { return hbit(HB_CNOT_THR + j) | hbit(HB_CNOT_BASE + j); }
constexpr uint64_t cnot_reg_bits(int j) { return hbits(HB_CNOT_REG + 3 * j, 3); }   // target register bit j

// X/Y rotation adjoints on register bit J, alone or after their inner product
template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void rot_handlers(Regs<CT, T, W> &x, uint64_t hf, CT u, CT w, double2 *sink, double2 *red, int slot,
                                             int fa, int tid) {
    if constexpr (J < RB) {
        if (hf & hbit(HB_PRODROT_Y + J)) {
            QNG_PRODS((prodw_xy<J, 1, T, CT, W>));
            rot_xy<J, 1, T, CT, W>(x, u, w);
            QNG_STORE_PRODS();
        }
        if (hf & hbit(HB_PRODROT_X + J)) {
            QNG_PRODS((prodw_xy<J, 0, T, CT, W>));
            rot_xy<J, 0, T, CT, W>(x, u, w);
            QNG_STORE_PRODS();
        }
        if (hf & hbit(HB_ROT_Y + J)) rot_xy<J, 1, T, CT, W>(x, u, w);
        if (hf & hbit(HB_ROT_X + J)) rot_xy<J, 0, T, CT, W>(x, u, w);
    }
}

// RZ adjoints on register bit J, alone or after their Z inner product
template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void diag_handlers(Regs<CT, T, W> &x, uint64_t hf, CT u, CT w, double2 *sink, double2 *red, int slot,
                                              int fa, int tid) {
    if constexpr (J < RB) {
        if (hf & hbit(HB_PRODDIAG_REG + J)) {
            QNG_PRODS((prodw_z_reg<J, T, CT, W>));
            diag_reg<J, T, CT, W>(x, u, w);
            QNG_STORE_PRODS();
        }
        if (hf & hbit(HB_DIAG_REG + J)) diag_reg<J, T, CT, W>(x, u, w);
    }
}

constexpr uint64_t prod_bits(int j) { return hbit(HB_PROD_X + j) | hbit(HB_PROD_Y + j) | hbit(HB_PRODZ_REG + j); }

// Inner products on register bit J without an adjoint after them
template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void prod_handlers(const Regs<CT, T, W> &x, uint64_t hf, double2 *sink, double2 *red, int slot, int fa,
                                              int tid) {
    if constexpr (J < RB) {
        if (hf & hbit(HB_PROD_X + J)) {
            QNG_PRODS((prodw_xy<J, 0, T, CT, W>));
            QNG_STORE_PRODS();
        }
        if (hf & hbit(HB_PROD_Y + J)) {
            QNG_PRODS((prodw_xy<J, 1, T, CT, W>));
            QNG_STORE_PRODS();
        }
        if (hf & hbit(HB_PRODZ_REG + J)) {
            QNG_PRODS((prodw_z_reg<J, T, CT, W>));
            QNG_STORE_PRODS();
        }
    }
}

template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void cnot_uni(Regs<CT, T, W> &x, bool control) {
    if constexpr (J < RB) cnot_cond<J, T, CT, W>(x, control);
}

// CNOT adjoints with target register bit J and a register control
template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void cnot_reg_handlers(Regs<CT, T, W> &x, uint64_t hf) {
    if constexpr (J < RB) {
        constexpr int K0 = J == 0 ? 1 : 0, K1 = J <= 1 ? 2 : 1, K2 = J <= 2 ? 3 : 2;   // controls != J
        if constexpr (K0 < RB)
            if (hf & hbit(HB_CNOT_REG + 3 * J + 0)) cnot_reg<J, K0, T, CT, W>(x);
        if constexpr (K1 < RB)
            if (hf & hbit(HB_CNOT_REG + 3 * J + 1)) cnot_reg<J, K1, T, CT, W>(x);
        if constexpr (K2 < RB)
            if (hf & hbit(HB_CNOT_REG + 3 * J + 2)) cnot_reg<J, K2, T, CT, W>(x);
    }
}

// Seed of phi register SB of a column block: phi_SB <- sigma lambda, sigma
// of Pauli axis `axis` (0 X, 1 Y, 2 Z) on the local bit at `loc` (X and Y:
// a register bit; Z: any location, qubit q for a bit of the tile base).
template <int SB, int RB, int T, typename CT, int W>
__device__ __forceinline__ void seed_phi(Regs<CT, T, W> &x, int axis, uint8_t loc, uint8_t q, int tid,
                                         uint64_t base) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        move_in_place(x.br[SB][i], x.ar[i]);
        move_in_place(x.bi[SB][i], x.ai[i]);
    }
    if (axis == 2) {
        const uint32_t neg = loc_mask<T>(loc, q, tid, base);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const CT sg = sel<CT>((neg >> i) & 1u, (CT)-1, (CT)1);
            x.br[SB][i] *= sg;
            x.bi[SB][i] *= sg;
        }
        return;
    }
#define QNG_SEED_XY(J)                                                                                       \
    if constexpr (J < RB) {                                                                                  \
        if (loc == J) {                                                                                      \
            swap_pairs<J, -1, T, CT>(x.br[SB], x.bi[SB]);                                                    \
            if (axis == 1) {                                                                                 \
                /* (Y v)_0 = -i v_1, (Y v)_1 = i v_0: after the swap, times -i where bit J is clear, */      \
                /* times i where it is set */                                                                \
                for (int i = 0; i < T; ++i) {                                                                \
                    swap_in_place(x.br[SB][i], x.bi[SB][i]);                                                 \
                    if (i & (1 << J)) x.br[SB][i] = -x.br[SB][i];                                            \
                    else x.bi[SB][i] = -x.bi[SB][i];                                                         \
                }                                                                                            \
            }                                                                                                \
        }                                                                                                    \
    }
    QNG_SEED_XY(0)
    QNG_SEED_XY(1)
    QNG_SEED_XY(2)
    QNG_SEED_XY(3)
#undef QNG_SEED_XY
}

// ------------------------------------------------------- controlled rotations
//
// A controlled rotation acts where its control bit is 1.  The control may sit
// at any location (register, thread or tile-base bit), so its value per
// register is a mask `on` (bit i for register i).  The adjoint is the plane
// rotation (c, s) on the same pairs of reals as the plain rotation's, taken as
// (1, 0) where the control is 0: there it leaves the values exactly as they
// are.  (Three shears cannot take the sign trick of the plain rotations here,
// since a sign on half of the amplitudes is not common to the registers.)  The
// generator |1><1|_c (x) sigma enters an inner product as lambda with its
// amplitudes of control 0 set to zero.

#define QNG_PLANE(A, B, C, S)                       \
    do {                                            \
        const CT a_ = A, b_ = B;                    \
        A = fmadd(C, a_, (S) * b_);                 \
        B = fmadd(C, b_, -(S) * a_);                \
    } while (0)

template <int J, int AX, int T, typename CT>
__device__ __forceinline__ void crot_xy1(CT (&re)[T], CT (&im)[T], uint32_t on, CT c, CT s) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);   // the control (not bit J) is the same for i and k
        const bool o = (on >> i) & 1u;
        const CT ci = sel<CT>(o, c, (CT)1), si = sel<CT>(o, s, (CT)0);
        if (AX == 0) {
            QNG_PLANE(re[i], im[k], ci, si);
            QNG_PLANE(re[k], im[i], ci, si);
        } else {
            QNG_PLANE(re[i], re[k], ci, si);
            QNG_PLANE(im[i], im[k], ci, si);
        }
    }
}
template <int J, int AX, int T, typename CT, int W>
__device__ __forceinline__ void crot_xy(Regs<CT, T, W> &x, uint32_t on, CT c, CT s) {
    crot_xy1<J, AX, T, CT>(x.ar, x.ai, on, c, s);
#pragma unroll
    for (int b = 0; b < W; ++b) crot_xy1<J, AX, T, CT>(x.br[b], x.bi[b], on, c, s);
}

// CRZ adjoint: where the control is 1, (re, im) rotated by (c, s) for target
// bit 0 and by (c, -s) for target bit 1 (`one`: mask of the target bit)
template <int T, typename CT, int W>
__device__ __forceinline__ void cdiag(Regs<CT, T, W> &x, uint32_t on, uint32_t one, CT c, CT s) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const bool o = (on >> i) & 1u;
        const CT ci = sel<CT>(o, c, (CT)1);
        const CT si = sel<CT>(o, sel<CT>((one >> i) & 1u, -s, s), (CT)0);
        QNG_PLANE(x.ar[i], x.ai[i], ci, si);
#pragma unroll
        for (int b = 0; b < W; ++b) QNG_PLANE(x.br[b][i], x.bi[b][i], ci, si);
    }
}

// The tile with lambda's amplitudes of control 0 set to zero and those with
// bit `neg` set negated (f in {0, 1, -1}: exact in any precision); the phi
// registers as they are.  A value copy: the products read it, the tile itself
// is left in place.
template <int T, typename CT, int W>
__device__ __forceinline__ Regs<CT, T, W> masked_lambda(const Regs<CT, T, W> &x, uint32_t on, uint32_t neg) {
    Regs<CT, T, W> y;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const CT f = sel<CT>((on >> i) & 1u, sel<CT>((neg >> i) & 1u, (CT)-1, (CT)1), (CT)0);
        y.ar[i] = x.ar[i] * f;
        y.ai[i] = x.ai[i] * f;
#pragma unroll
        for (int b = 0; b < W; ++b) {
            y.br[b][i] = x.br[b][i];
            y.bi[b][i] = x.bi[b][i];
        }
    }
    return y;
}

constexpr uint32_t h2bit(int b) { return uint32_t(1) << b; }
constexpr uint32_t crot_bits(int j) {
    return h2bit(HB2_CROT_X + j) | h2bit(HB2_CROT_Y + j) | h2bit(HB2_PRODCROT_X + j) | h2bit(HB2_PRODCROT_Y + j) |
           h2bit(HB2_PRODC_X + j) | h2bit(HB2_PRODC_Y + j);
}

// Controlled X/Y operations with the target on register bit J: products of
// the generator (alone or before the adjoint), adjoints
template <int J, int RB, int T, typename CT, int W>
__device__ __forceinline__ void crot_handlers(Regs<CT, T, W> &x, uint32_t h2, uint32_t on, CT c, CT s,
                                              double2 *sink, double2 *red, int slot, int fa, int tid) {
    if constexpr (J < RB) {
        if constexpr (!kNoProducts) {
            if (h2 & (h2bit(HB2_PRODCROT_X + J) | h2bit(HB2_PRODC_X + J))) {
                const Regs<CT, T, W> y = masked_lambda<T, CT, W>(x, on, 0u);
                double pr[W], pi[W];
                prodw_xy<J, 0, T, CT, W>(y, pr, pi);
                row_reduce_store<W>(sink, red, slot, fa, tid, pr, pi);
            }
            if (h2 & (h2bit(HB2_PRODCROT_Y + J) | h2bit(HB2_PRODC_Y + J))) {
                const Regs<CT, T, W> y = masked_lambda<T, CT, W>(x, on, 0u);
                double pr[W], pi[W];
                prodw_xy<J, 1, T, CT, W>(y, pr, pi);
                row_reduce_store<W>(sink, red, slot, fa, tid, pr, pi);
            }
        }
        if (h2 & (h2bit(HB2_PRODCROT_X + J) | h2bit(HB2_CROT_X + J))) crot_xy<J, 0, T, CT, W>(x, on, c, s);
        if (h2 & (h2bit(HB2_PRODCROT_Y + J) | h2bit(HB2_CROT_Y + J))) crot_xy<J, 1, T, CT, W>(x, on, c, s);
    }
}

// One register of the tile through the exchange buffer, from mapping `from`
// to mapping `to`.  With RECOMPUTE the slots are recomputed for every
// register from an opaque copy of the thread index (the kernels with two phi
// registers near the VGPR bound: kept across the exchanges of all three
// registers the slots hold 2T more VGPRs next to the tile, and spill);
// otherwise the compiler computes them once for all registers.
template <int RB, int T, typename CT, typename CX, bool RECOMPUTE>
__device__ __forceinline__ void exchange(CT (&re)[T], CT (&im)[T], CX *xbuf, const MapBytes &from,
                                         const MapBytes &to, int tbits, int tid, bool active) {
    int t = tid;
    if constexpr (RECOMPUTE) asm volatile("" : "+v"(t));
    if (active) {
        uint32_t lo[T];
        local_offsets<RB, T>(from, tbits, t, lo);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            CX v;
            v.x = re[i];
            v.y = im[i];
            xbuf[lo[i]] = v;
        }
    }
    __syncthreads();
    if (active) {
        uint32_t lo[T];
        local_offsets<RB, T>(to, tbits, t, lo);
#pragma unroll
        for (int i = 0; i < T; ++i) {
            const CX v = xbuf[lo[i]];
            re[i] = v.x;
            im[i] = v.y;
        }
    }
    __syncthreads();
}

template <typename R, typename CT, int T>
__device__ __forceinline__ void load_reg(const void *g, const uint64_t (&off)[T], CT (&re)[T], CT (&im)[T]) {
    using C = typename Amp<R>::T;
    const C *p = (const C *)g;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        const C v = p[off[i]];
        re[i] = v.x;
        im[i] = v.y;
    }
}

template <typename R, typename CT, int T>
__device__ __forceinline__ void store_reg(void *g, const uint64_t (&off)[T], const CT (&re)[T], const CT (&im)[T]) {
    using C = typename Amp<R>::T;
    C *p = (C *)g;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        C v;
        v.x = (R)re[i];
        v.y = (R)im[i];
        p[off[i]] = v;
    }
}

// Tile sums <lambda|phi_b>_tile of phi registers B0 .. B1-1, summed over the
// work-group (uniform control flow: contains barriers).
template <int T, typename CT, int W, int B0, int B1, int N>
__device__ __forceinline__ void tile_sums(const Regs<CT, T, W> &x, double2 *sink, double2 *zs, int tid,
                                          double (&Sr)[N], double (&Si)[N]) {
    __syncthreads();   // earlier readers of zs are done
#pragma unroll
    for (int b = B0; b < B1; ++b) {
        double sr, si;
        prod_plain<T, CT>(x.ar, x.ai, x.br[b], x.bi[b], sr, si);
        row_store(sink, zs, b, tid, sr, si);
    }
    __syncthreads();
#pragma unroll
    for (int b = B0; b < B1; ++b) {
        double ar = 0.0, ai = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            ar += zs[b * kWaves + w].x;
            ai += zs[b * kWaves + w].y;
        }
        Sr[b] = ar;
        Si[b] = ai;
    }
    __syncthreads();   // zs lies in the exchange buffer: read before the next exchange
}

// Seed of a lower column of a block: phi register SB <- sigma lambda when the
// op names register SB, then <lambda|phi> into the op's slot and the pass's
// tile sums of that register (uniform control flow: contains barriers).
template <int SB, int RB, int T, typename CT, int W>
__device__ __forceinline__ void seed_handler(Regs<CT, T, W> &x, const OpD &op, int tid, uint64_t base,
                                             double2 *sink, double2 *red, double2 *zs, bool pass_zsum,
                                             double (&Sr)[W], double (&Si)[W]) {
    if constexpr (SB + 1 < W) {
        if (op.aux == SB) {
            seed_phi<SB, RB, T, CT, W>(x, op.w0 >> 24, op.b0(), op.q0(), tid, base);
            if constexpr (!kNoProducts) {
                double pr, pi;
                prod_plain<T, CT>(x.ar, x.ai, x.br[SB], x.bi[SB], pr, pi);
                row_store(sink, red, op.slot(), tid, pr, pi);
                if (pass_zsum) tile_sums<T, CT, W, SB, SB + 1>(x, sink, zs, tid, Sr, Si);
            }
        }
    }
}

// Occupancy target: three waves per SIMD (the 53 KB of LDS of a work-group
// allow three per CU).  The 16-amplitude kernel with one phi register reaches
// it by itself (114 VGPRs; 158 with every product in FP64) and gets no bound;
// with two phi registers it is held to 168 VGPRs (it needs 146; with every
// product in FP64 a few values spill in the exchanges).
template <typename R, typename CT, int RB, bool FULL, int W, bool CTRL>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kNoProducts ? (sizeof(CT) == 4 ? QNG_STATES_WAVES : 3) : W == 1 ? (RB >= 4 ? 1 : 3) : 3, 8))) void QNG_SWEEP_KERNEL(const LaunchItem *__restrict__ items, int n_items,
                                                        const DevPass *__restrict__ passes,
                                                        const DevOp *__restrict__ ops,
                                                        const DevMap *__restrict__ maps,
                                                        const void *__restrict__ mats,
                                                        double2 *__restrict__ partials) {
    constexpr int T = 1 << RB;
    extern __shared__ __align__(16) unsigned char smem[];

    // ---- which item (one pass of one column block) this work-group serves
    const uint32_t wg = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    const LaunchItem it = items[lo];
    const DevPass *pp = passes + it.pass;
    // consecutive passes of a column walk their tiles in opposite orders, so a
    // pass starts on the tiles the previous one wrote last (still in the
    // last-level cache)
    const uint32_t tile = (it.pass & 1u) ? it.ntiles - 1 - (wg - it.tile_begin) : wg - it.tile_begin;
    const uint4 ph0 = *reinterpret_cast<const uint4 *>(pp);          // op_begin, n_ops, slots|m|n, nrest|zsum|rb
    const uint4 ph1 = *(reinterpret_cast<const uint4 *>(pp) + 1);    // map_load, pad, tile_q[0..7]
    const int m = (int)((ph0.z >> 16) & 0xffu);
    const int pass_nrest = (int)(ph0.w & 0xffu);
    const bool pass_zsum = ((ph0.w >> 8) & 0xffu) != 0;
    const int pass_slots = (int)(ph0.z & 0xffffu);
    const int tbits = m - RB;
    const int tid = threadIdx.x;
    // FULL: the tile has exactly kThreads * T amplitudes, every thread holds a
    // part of it (no divergent branches around the exchanges)
    const bool active = FULL || (tid >> tbits) == 0;

    using CX = typename Amp<CT>::T;
    CX *xbuf = (CX *)smem;                                // [2^m] exchange buffer
    double2 *tail = (double2 *)(smem + xbuf_bytes<CX>(m));
    double2 *sink = tail + tid;                           // this thread's sink entry
    double2 *red = tail + kThreads;                       // [kMaxSlots][kWaves]
    double2 *zs = (double2 *)xbuf;                        // [W][kWaves], inside the exchange buffer

    uint64_t base = 0;
    const PassBytes pbytes = load_pass_bytes(pp);
#pragma unroll
    for (int k = 0; k < kMaxRest; ++k)
        if (k < pass_nrest) base |= (uint64_t)((tile >> k) & 1u) << pbytes.rest(k);

    void *gphi[W > 0 ? W : 1];
#pragma unroll
    for (int b = 0; b < W; ++b) gphi[b] = b == 0 ? it.regB : b == 1 ? it.regC : b == 2 ? it.regD : it.regE;
    Regs<CT, T, W> x;

    // ---- load
    MapBytes cur = load_map(maps + ph1.x);
    {
        uint64_t off[T];
        global_offsets<RB, T>(pbytes, cur, tbits, tid, base, off);
        if (active) {
            load_reg<R, CT, T>(it.regA, off, x.ar, x.ai);
#pragma unroll
            for (int b = 0; b < W; ++b) load_reg<R, CT, T>(gphi[b], off, x.br[b], x.bi[b]);
        } else {
#pragma unroll
            for (int i = 0; i < T; ++i) {
                x.ar[i] = x.ai[i] = (CT)0;
#pragma unroll
                for (int b = 0; b < W; ++b) x.br[b][i] = x.bi[b][i] = (CT)0;
            }
        }
    }
    // plain tile sums <A|B_b>_tile for Z inner products on qubits outside the
    // tile (a phi register seeded in this pass gets its sum at the seed)
    double Sr[W > 0 ? W : 1], Si[W > 0 ? W : 1];
#pragma unroll
    for (int b = 0; b < W; ++b) Sr[b] = Si[b] = 0.0;
    if (!kNoProducts && pass_zsum) tile_sums<T, CT, W, 0, W>(x, sink, zs, tid, Sr, Si);

    // ---- operations.  Each op carries a one-hot handler bit; the handlers run
    // under independent tests of that word (by group, register bit, kind),
    // each one a straight-line update of the register tile in place.
    const CT *__restrict__ mt = (const CT *)mats;
    const int n_ops = (int)ph0.y;
    const DevOp *op_ptr = ops + ph0.x;
    // The descriptor of the next op is fetched while the current one runs, and
    // the current op's shear parameters (unused by ops without a gate) before
    // the handlers, so scalar-load latency overlaps the work.
    OpD nxt = load_op(op_ptr);
    for (int oi = 0; oi < n_ops; ++oi) {
        const OpD op = nxt;
        nxt = load_op(op_ptr + (oi + 1 < n_ops ? oi + 1 : oi));
        const CT *mrow = mt + (size_t)(op.gate > 0 ? op.gate : 0) * 8;
        const CT u = mrow[0], w = mrow[1];
        const uint64_t hf = op.hf;
        const int fa = (W == 1) ? 0 : op.aux;   // inner products: first active phi register
        // Handlers under independent tests of the handler word, nested by
        // group and register bit (an if / else-if chain would merge several
        // tile updates at one point, and the compiler then gives the tile a
        // second register set and copies it at every op).
        if (hf & hbits(HB_ROT_X, 16)) {
            // X/Y rotations, alone or after their inner product
            if (hf & rot_bits(0)) rot_handlers<0, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & rot_bits(1)) rot_handlers<1, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & rot_bits(2)) rot_handlers<2, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & rot_bits(3)) rot_handlers<3, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
        }
        if (hf & hbits(HB_DIAG_REG, 10)) {
            // RZ adjoints, alone or after their Z inner product
            if (hf & (hbit(HB_DIAG_UNI) | hbit(HB_PRODDIAG_UNI))) {
                // the Z bit is common to all registers of the thread
                const bool one = (op.b0() == kLocBase) ? ((base >> op.q0()) & 1u) : ((tid >> (op.b0() & 15)) & 1);
                if (!kNoProducts && (hf & hbit(HB_PRODDIAG_UNI))) {
                    const double sg = one ? -1.0 : 1.0;
                    const int slot = op.slot();
                    QNG_PRODS((prodw_plain<T, CT, W>));
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        pr[b] *= sg;
                        pi[b] *= sg;
                    }
                    QNG_STORE_PRODS();
                }
                diag_all<T, CT, W>(x, one ? -u : u, one ? -w : w);
            }
            if (hf & diag_bits(0)) diag_handlers<0, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & diag_bits(1)) diag_handlers<1, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & diag_bits(2)) diag_handlers<2, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
            if (hf & diag_bits(3)) diag_handlers<3, RB, T, CT, W>(x, hf, u, w, sink, red, op.slot(), fa, tid);
        }
        if (hf & hbits(HB_CNOT_REG, 20)) {
            // CNOT adjoints (register target)
            if (hf & hbits(HB_CNOT_THR, 8)) {
                // control held by the thread index or the tile base
                const bool control = (hf & hbits(HB_CNOT_THR, 4)) ? ((tid >> (op.b1() & 15)) & 1) != 0
                                                                   : ((base >> op.q0()) & 1u) != 0;
                if (hf & cnot_uni_bits(0)) cnot_cond<0, T, CT, W>(x, control);
                if (hf & cnot_uni_bits(1)) cnot_uni<1, RB, T, CT, W>(x, control);
                if (hf & cnot_uni_bits(2)) cnot_uni<2, RB, T, CT, W>(x, control);
                if (hf & cnot_uni_bits(3)) cnot_uni<3, RB, T, CT, W>(x, control);
            }
            if (hf & cnot_reg_bits(0)) cnot_reg_handlers<0, RB, T, CT, W>(x, hf);
            if (hf & cnot_reg_bits(1)) cnot_reg_handlers<1, RB, T, CT, W>(x, hf);
            if (hf & cnot_reg_bits(2)) cnot_reg_handlers<2, RB, T, CT, W>(x, hf);
            if (hf & cnot_reg_bits(3)) cnot_reg_handlers<3, RB, T, CT, W>(x, hf);
        }
        if (hf & hbits(HB_PROD_X, 13)) {
            // inner products without an adjoint after them (independent tests
            // like the other handlers: under one multi-way branch the compiler
            // hoists the conversions of the whole tile above it, 128 more VGPRs)
            const int slot = op.slot();
            if (hf & hbits(HB_PROD_X, 12)) {
                if (hf & prod_bits(0)) prod_handlers<0, RB, T, CT, W>(x, hf, sink, red, slot, fa, tid);
                if (hf & prod_bits(1)) prod_handlers<1, RB, T, CT, W>(x, hf, sink, red, slot, fa, tid);
                if (hf & prod_bits(2)) prod_handlers<2, RB, T, CT, W>(x, hf, sink, red, slot, fa, tid);
                if (hf & prod_bits(3)) prod_handlers<3, RB, T, CT, W>(x, hf, sink, red, slot, fa, tid);
            }
            if (!kNoProducts && (hf & hbit(HB_PRODZ_UNI))) {
                // Z bit held by the thread index or the tile base
                const bool one =
                    (op.b0() == kLocBase) ? ((base >> op.q0()) & 1u) : ((tid >> (op.b0() & 15)) & 1);
                const double sg = one ? -1.0 : 1.0;
                QNG_PRODS((prodw_plain<T, CT, W>));
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    pr[b] *= sg;
                    pi[b] *= sg;
                }
                QNG_STORE_PRODS();
            }
        }
        if constexpr (CTRL) {
            // controlled rotations (second handler word): the control's value per
            // register, the adjoint's plane rotation from the table's third and
            // fourth entries (without products: the adjoints and seeds alone)
            const uint32_t h2 = op.h2;
            if (h2) {
                const uint32_t on = loc_mask<T>(op.b1(), op.q1(), tid, base);
                const CT c = mrow[2], s = mrow[3];
                const int slot = op.slot();
                if (h2 & crot_bits(0)) crot_handlers<0, RB, T, CT, W>(x, h2, on, c, s, sink, red, slot, fa, tid);
                if (h2 & crot_bits(1)) crot_handlers<1, RB, T, CT, W>(x, h2, on, c, s, sink, red, slot, fa, tid);
                if (h2 & crot_bits(2)) crot_handlers<2, RB, T, CT, W>(x, h2, on, c, s, sink, red, slot, fa, tid);
                if (h2 & crot_bits(3)) crot_handlers<3, RB, T, CT, W>(x, h2, on, c, s, sink, red, slot, fa, tid);
                if (h2 & (h2bit(HB2_CDIAG) | h2bit(HB2_PRODCDIAG) | h2bit(HB2_PRODCZ))) {
                    const uint32_t one = loc_mask<T>(op.b0(), op.q0(), tid, base);
                    if (!kNoProducts && (h2 & (h2bit(HB2_PRODCDIAG) | h2bit(HB2_PRODCZ)))) {
                        const Regs<CT, T, W> y = masked_lambda<T, CT, W>(x, on, one);
                        double pr[W], pi[W];
                        prodw_plain<T, CT, W>(y, pr, pi);
                        row_reduce_store<W>(sink, red, slot, fa, tid, pr, pi);
                    }
                    if (h2 & (h2bit(HB2_CDIAG) | h2bit(HB2_PRODCDIAG))) cdiag<T, CT, W>(x, on, one, c, s);
                }
                if constexpr (W > 1) {
                    if (h2 & h2bit(HB2_CSEED)) {
                        // phi register 0 <- K lambda: sigma on the target, then the
                        // amplitudes of control 0 cleared; <lambda|phi> into the slot
                        seed_phi<0, RB, T, CT, W>(x, op.w0 >> 24, op.b0(), op.q0(), tid, base);
#pragma unroll
                        for (int i = 0; i < T; ++i) {
                            const CT f = sel<CT>((on >> i) & 1u, (CT)1, (CT)0);
                            x.br[0][i] *= f;
                            x.bi[0][i] *= f;
                        }
                        if constexpr (!kNoProducts) {
                            double pr, pi;
                            prod_plain<T, CT>(x.ar, x.ai, x.br[0], x.bi[0], pr, pi);
                            row_store(sink, red, slot, tid, pr, pi);
                            if (pass_zsum) tile_sums<T, CT, W, 0, 1>(x, sink, zs, tid, Sr, Si);
                        }
                    }
                }
            }
        }
        if (hf & (hbit(HB_XPOSE) | hbit(HB_CZ) | hbit(HB_ZSUM) | hbit(HB_SEED))) {
            if (hf & hbit(HB_CZ)) {
                const uint32_t neg = loc_mask<T>(op.b0(), op.q0(), tid, base) & loc_mask<T>(op.b1(), op.q1(), tid, base);
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const CT sg = sel<CT>((neg >> i) & 1u, (CT)-1, (CT)1);
                    x.ar[i] *= sg;
                    x.ai[i] *= sg;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        x.br[b][i] *= sg;
                        x.bi[b][i] *= sg;
                    }
                }
            }
            if (!kNoProducts && (hf & hbit(HB_ZSUM))) {
                if (tid == 0) {
                    const double sg = ((base >> op.q0()) & 1u) ? -1.0 : 1.0;
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        if (W > 1 && b < fa) continue;
                        const int sl = op.slot() + b - fa;
                        red[sl * kWaves] = make_double2(sg * Sr[b], sg * Si[b]);
                        for (int k = 1; k < kWaves; ++k) red[sl * kWaves + k] = make_double2(0.0, 0.0);
                    }
                }
            }
            if constexpr (W > 1) {
                if (hf & hbit(HB_SEED)) {
                    // phi register op.aux (below the top one) <- sigma lambda;
                    // <lambda|phi> = <y|sigma|y> into the op's slot
                    seed_handler<0, RB, T, CT, W>(x, op, tid, base, sink, red, zs, pass_zsum, Sr, Si);
                    if constexpr (W > 2) {
                        seed_handler<1, RB, T, CT, W>(x, op, tid, base, sink, red, zs, pass_zsum, Sr, Si);
                        seed_handler<2, RB, T, CT, W>(x, op, tid, base, sink, red, zs, pass_zsum, Sr, Si);
                    }
                }
            }
            if (hf & hbit(HB_XPOSE)) {
                const MapBytes next = load_map(maps + op.aux);
                constexpr bool kRecompute = W > 1 && (RB >= 4 || sizeof(R) < sizeof(CT));
                exchange<RB, T, CT, CX, kRecompute>(x.ar, x.ai, xbuf, cur, next, tbits, tid, active);
#pragma unroll
                for (int b = 0; b < W; ++b)
                    exchange<RB, T, CT, CX, kRecompute>(x.br[b], x.bi[b], xbuf, cur, next, tbits, tid, active);
                cur = next;
            }
        }
    }

    // ---- store
    {
        uint64_t off[T];
        global_offsets<RB, T>(pbytes, cur, tbits, tid, base, off);
        if (active) {
            store_reg<R, CT, T>(it.regA, off, x.ar, x.ai);
#pragma unroll
            for (int b = 0; b < W; ++b) store_reg<R, CT, T>(gphi[b], off, x.br[b], x.bi[b]);
        }
    }
    // ---- per-tile partial sums
    if constexpr (kNoProducts) return;
    __syncthreads();
    for (int k = tid; k < pass_slots; k += kThreads) {
        double xr = 0.0, xi = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            xr += red[k * kWaves + w].x;
            xi += red[k * kWaves + w].y;
        }
        partials[it.partial_off + (uint64_t)k * it.ntiles + tile] = make_double2(xr, xi);
    }
}

// One work-group per task sums the task's per-tile partials in a fixed order
// (bitwise reproducible): 1024 threads, four independent loads in flight per
// thread, then a tree over the threads.
constexpr int kReduceThreads = 1024;

__global__ __launch_bounds__(kReduceThreads) void k_reduce_tasks(const ReduceTask *__restrict__ tasks,
                                                                 const double2 *__restrict__ partials,
                                                                 double2 *__restrict__ results) {
    __shared__ double sr[kReduceThreads], si[kReduceThreads];
    const ReduceTask t = tasks[blockIdx.x];
    const double2 *p = partials + t.off;
    double a0 = 0.0, b0 = 0.0, a1 = 0.0, b1 = 0.0, a2 = 0.0, b2 = 0.0, a3 = 0.0, b3 = 0.0;
    uint32_t k = threadIdx.x;
    for (; k + 3 * kReduceThreads < t.count; k += 4 * kReduceThreads) {
        const double2 v0 = p[k], v1 = p[k + kReduceThreads], v2 = p[k + 2 * kReduceThreads],
                      v3 = p[k + 3 * kReduceThreads];
        a0 += v0.x; b0 += v0.y;
        a1 += v1.x; b1 += v1.y;
        a2 += v2.x; b2 += v2.y;
        a3 += v3.x; b3 += v3.y;
    }
    for (; k < t.count; k += kReduceThreads) {
        const double2 v = p[k];
        a0 += v.x;
        b0 += v.y;
    }
    sr[threadIdx.x] = (a0 + a1) + (a2 + a3);
    si[threadIdx.x] = (b0 + b1) + (b2 + b3);
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) results[t.dest] = make_double2(sr[0], si[0]);
}

template <typename CT> size_t smem_bytes(int m) {
    // without products only the exchange buffer is used
    return xbuf_bytes<typename Amp<CT>::T>(m) + (kNoProducts ? 0 : (size_t)kLdsTailEntries * sizeof(double2));
}

template <typename R, typename CT, int RB, bool FULL, int W, bool CTRL>
void launch_full(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
                 const DevMap *maps, const CT *mats, double *partials, int m, hipStream_t st) {
    const size_t smem = smem_bytes<CT>(m);
    static size_t attr_set = 0;
    if (smem > attr_set) {
        (void)hipFuncSetAttribute((const void *)QNG_SWEEP_KERNEL<R, CT, RB, FULL, W, CTRL>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        (void)hipGetLastError();
        attr_set = smem;
    }
    hipLaunchKernelGGL((QNG_SWEEP_KERNEL<R, CT, RB, FULL, W, CTRL>), dim3(total_tiles), dim3(kThreads), smem, st,
                       items, n_items, passes, ops, maps, (const void *)mats, (double2 *)partials);
}

// The kernels with the second handler word (controlled rotations) are built
// apart, so plans without controlled rotations keep the plain op loop.
template <typename R, typename CT, int RB, bool FULL, int W>
void launch_ctrl(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
                 const DevMap *maps, const CT *mats, double *partials, int m, bool ctrl, hipStream_t st) {
    if (ctrl) {
        launch_full<R, CT, RB, FULL, W, true>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st);
        return;
    }
    launch_full<R, CT, RB, FULL, W, false>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st);
}

// Every pass of a launch has the launch's tile width m (one plan, or one
// register class of a batch), so "every thread holds part of the tile" is a
// property of the launch.  Blocks of two columns run with full tiles of 8 or
// 16 amplitudes per thread (registers of at least 11 qubits).
template <typename R, typename CT, int RB>
void launch_rb(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
               const DevMap *maps, const CT *mats, double *partials, int m, int width, bool ctrl, hipStream_t st) {
    const bool full = m - RB == 8;
    if (width == 0) {
        // lambda alone (forward plans), passes without products only
        if constexpr (kNoProducts) {
            if (!ctrl) {
                if (full)
                    launch_full<R, CT, RB, true, 0, false>(items, n_items, total_tiles, passes, ops, maps, mats,
                                                           partials, m, st);
                else
                    launch_full<R, CT, RB, false, 0, false>(items, n_items, total_tiles, passes, ops, maps, mats,
                                                            partials, m, st);
                return;
            }
        }
        throw hipErrorInvalidValue;
    }
    if (width == 2) {
        if constexpr (RB >= 3) {
            if (full) {
                launch_ctrl<R, CT, RB, true, 2>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m,
                                                ctrl, st);
                return;
            }
        }
        throw hipErrorInvalidValue;
    }
    if (width == 4) {
        // four-column blocks: 8 amplitudes per thread, FP32 registers, no
        // controlled rotations
        if constexpr (RB == 3 && sizeof(CT) == 4) {
            if (full && !ctrl) {
                launch_full<R, CT, RB, true, 4, false>(items, n_items, total_tiles, passes, ops, maps, mats, partials,
                                                       m, st);
                return;
            }
        }
        throw hipErrorInvalidValue;
    }
    if (full)
        launch_ctrl<R, CT, RB, true, 1>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, ctrl, st);
    else
        launch_ctrl<R, CT, RB, false, 1>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, ctrl, st);
}

template <typename R, typename CT>
void launch_ct(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
               const DevMap *maps, const CT *mats, double *partials, int m, int rb, int width, bool ctrl,
               hipStream_t st) {
    switch (rb) {
    case 1: launch_rb<R, CT, 1>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, width, ctrl, st); break;
    case 2: launch_rb<R, CT, 2>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, width, ctrl, st); break;
    case 3: launch_rb<R, CT, 3>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, width, ctrl, st); break;
    case 4:
        // FP64 registers stop at 8 amplitudes per thread: at 16 the kernel
        // needs 178-226 VGPRs (two waves per SIMD) and measured 1.8-2.2x slower
        // per pass at n = 26
        if constexpr (sizeof(CT) == 4) {
            launch_rb<R, CT, 4>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, width, ctrl, st);
            break;
        }
        [[fallthrough]];
    default: throw hipErrorInvalidValue;
    }
}

}  // namespace

#if QNG_NO_PRODUCTS
template <typename R>
void launch_sweep_pass_states(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                              const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32, int m,
                              int rb, int width, hipStream_t st, bool ctrl) {
    if (n_items <= 0 || total_tiles == 0) return;
    if constexpr (sizeof(R) == 8)
        launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats64, nullptr, m, rb, width, ctrl, st);
    else
        launch_ct<R, float>(items, n_items, total_tiles, passes, ops, maps, mats32, nullptr, m, rb, width, ctrl, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}
template void launch_sweep_pass_states<double>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                               const DevMap *, const double *, const float *, int, int, int,
                                               hipStream_t, bool);
template void launch_sweep_pass_states<float>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                              const DevMap *, const double *, const float *, int, int, int,
                                              hipStream_t, bool);
#elif QNG_REAL_PRODUCTS && QNG_EXACT_PRODUCTS
void launch_sweep_pass_real_exact(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                                  const DevOp *ops, const DevMap *maps, const float *mats32, double *partials, int m,
                                  int rb, int width, hipStream_t st, bool ctrl) {
    if (n_items <= 0 || total_tiles == 0) return;
    launch_ct<float, float>(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb, width, ctrl, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}
#elif QNG_REAL_PRODUCTS
template <typename R>
void launch_sweep_pass_real(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                            const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32,
                            double *partials, int m, int rb, int reg_mode, int width, hipStream_t st, bool ctrl) {
    if (n_items <= 0 || total_tiles == 0) return;
    if constexpr (sizeof(R) == 8) {
        (void)reg_mode;
        launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats64, partials, m, rb, width, ctrl, st);
    } else {
        if (reg_mode == REG_F64)
            launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats64, partials, m, rb, width, ctrl, st);
        else if (reg_mode == REG_F32)
            launch_ct<R, float>(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb, width, ctrl, st);
        else
            throw hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}
template void launch_sweep_pass_real<double>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                             const DevMap *, const double *, const float *, double *, int, int, int,
                                             int, hipStream_t, bool);
template void launch_sweep_pass_real<float>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                            const DevMap *, const double *, const float *, double *, int, int, int,
                                            int, hipStream_t, bool);
#elif !QNG_EXACT_PRODUCTS
template <typename R>
void launch_sweep_pass(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                       const DevOp *ops, const DevMap *maps, const double *mats64, const float *mats32,
                       double *partials, int m, int rb, int reg_mode, int width, hipStream_t st, bool real_products,
                       bool ctrl) {
    if (n_items <= 0 || total_tiles == 0) return;
    if (real_products) {
        if (reg_mode == REG_F32_EXACT)
            launch_sweep_pass_real_exact(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb,
                                         width, st, ctrl);
        else
            launch_sweep_pass_real<R>(items, n_items, total_tiles, passes, ops, maps, mats64, mats32, partials, m,
                                      rb, reg_mode, width, st, ctrl);
        return;
    }
    if constexpr (sizeof(R) == 8) {
        (void)reg_mode;
        launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats64, partials, m, rb, width, ctrl, st);
    } else {
        if (reg_mode == REG_F64)
            launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats64, partials, m, rb, width, ctrl, st);
        else if (reg_mode == REG_F32_EXACT)
            launch_sweep_pass_exact(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb, width,
                                    st, ctrl);
        else
            launch_ct<R, float>(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb, width, ctrl, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

void launch_reduce_tasks(const ReduceTask *tasks, int n_tasks, const double *partials, double *results,
                         hipStream_t st) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(k_reduce_tasks, dim3(n_tasks), dim3(kReduceThreads), 0, st, tasks,
                       (const double2 *)partials, (double2 *)results);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

template void launch_sweep_pass<double>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                        const DevMap *, const double *, const float *, double *, int, int, int, int,
                                        hipStream_t, bool, bool);
template void launch_sweep_pass<float>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                       const DevMap *, const double *, const float *, double *, int, int, int, int,
                                       hipStream_t, bool, bool);
#else
void launch_sweep_pass_exact(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                             const DevOp *ops, const DevMap *maps, const float *mats32, double *partials, int m,
                             int rb, int width, hipStream_t st, bool ctrl) {
    if (n_items <= 0 || total_tiles == 0) return;
    launch_ct<float, float>(items, n_items, total_tiles, passes, ops, maps, mats32, partials, m, rb, width, ctrl, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}
#endif

}  // namespace qng
