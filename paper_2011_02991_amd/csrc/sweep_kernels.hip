// sweep_kernels.hip -- the fused sweep-pass kernel for gfx950 (see sweep.hpp).
//
// One work-group of 256 threads (4 wave64) owns one tile: the 2^m amplitudes
// of lambda (A) and phi (B) whose indices agree outside the pass's m tile
// qubits.  The tile lives in registers: every thread holds T = 2^RB amplitudes
// of each register, in FP64 whatever the storage precision (complex64 states
// are widened at the load and rounded once at the store of each pass).  A thread mapping says which local bits are "register
// bits" (the thread's own T amplitudes differ in them) and which are "thread
// bits" (bits of the thread index).
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
//  * Inner products accumulate per thread in FP64, are summed within each
//    16-lane row with DPP shifts and kept per (slot, row) in LDS; at the end
//    one FP64 partial per (slot, tile) is written, and k_reduce_tasks adds the
//    partials of a slot over the tiles in a fixed order (bitwise reproducible).
//  * Store: registers -> HBM under the final mapping (lanes on the lowest
//    qubits again), in place: the tile is touched by this work-group only.
#include <hip/hip_runtime.h>

#include "sweep.hpp"

namespace qng {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename R> struct Amp;
template <> struct Amp<double> { using T = double2; };
template <> struct Amp<float>  { using T = float2; };

constexpr int kRows = kThreads / 16;   // DPP rows of 16 lanes per work-group

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

// Store a per-lane partial of slot `slot`: one value per 16-lane row.
__device__ __forceinline__ void row_store(double2 *red, int slot, int tid, double a, double b) {
    row_sum(a, b);
    if ((tid & 15) == 15) red[slot * kRows + (tid >> 4)] = make_double2(a, b);
}

// The tile is kept as four scalar arrays per thread: real and imaginary parts
// of lambda (A) and phi (B), T values each (scalar arrays stay in VGPRs).
template <typename CT, int T>
struct Regs {
    CT ar[T], ai[T], br[T], bi[T];
};

// conj(x) * y accumulated in FP64
template <typename R>
__device__ __forceinline__ void cmac(double &sr, double &si, R xr_, R xi_, R yr_, R yi_) {
    const double xr = xr_, xi = xi_, yr = yr_, yi = yi_;
    sr += xr * yr + xi * yi;
    si += xr * yi - xi * yr;
}

// 2x2 complex matrix [[a, b], [c, d]] as scalars
template <typename R>
struct M2 {
    R ar, ai, br, bi, cr, ci, dr, di;
};

template <typename R>
__device__ __forceinline__ M2<R> load_m2(const double *p) {
    return M2<R>{(R)p[0], (R)p[1], (R)p[2], (R)p[3], (R)p[4], (R)p[5], (R)p[6], (R)p[7]};
}

// 2x2 complex matrix on the pair (x0, x1)
template <typename R>
__device__ __forceinline__ void mat_apply(const M2<R> m, R &x0r, R &x0i, R &x1r, R &x1i) {
    const R ur = x0r, ui = x0i, vr = x1r, vi = x1i;
    x0r = m.ar * ur - m.ai * ui + m.br * vr - m.bi * vi;
    x0i = m.ar * ui + m.ai * ur + m.br * vi + m.bi * vr;
    x1r = m.cr * ur - m.ci * ui + m.dr * vr - m.di * vi;
    x1i = m.cr * ui + m.ci * ur + m.dr * vi + m.di * vr;
}

// value select (by-value operands keep the choice on registers, not on addresses)
template <typename R>
__device__ __forceinline__ R sel(bool c, R a, R b) {
    return c ? a : b;
}

template <typename R>
__device__ __forceinline__ void cmul(R &xr, R &xi, R fr, R fi) {
    const R ur = xr, ui = xi;
    xr = fr * ur - fi * ui;
    xi = fr * ui + fi * ur;
}

// ---------------------------------------------------------- register-bit ops

// <A|sigma|B> over the pairs of register bit J (a* meaning conj(a)):
//   X: a0*b1 + a1*b0;   Y: i (a1*b0 - a0*b1).
// The pair loop accumulates S1 = sum a0*b1 and S2 = sum a1*b0 for either axis
// (no branch on the axis inside the loop); the axis picks the combination.
template <int J, int T, typename CT>
__device__ __forceinline__ void prod_bit(int axis, const Regs<CT, T> &x, double &pr, double &pi) {
    double s1r = 0.0, s1i = 0.0, s2r = 0.0, s2i = 0.0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);
        cmac(s1r, s1i, x.ar[i], x.ai[i], x.br[k], x.bi[k]);
        cmac(s2r, s2i, x.ar[k], x.ai[k], x.br[i], x.bi[i]);
    }
    const bool ax = axis == 0;
    pr += sel(ax, s1r + s2r, s1i - s2i);
    pi += sel(ax, s1i + s2i, s2r - s1r);
}

// Adjoint rotation on the pairs of register bit J.  The matrices of RX and RY
// adjoints have exact zeros (RX: real diagonal, imaginary off-diagonal; RY:
// real), so each output is two products instead of four.
template <int J, int T, typename CT>
__device__ __forceinline__ void rot_bit(int axis, Regs<CT, T> &x, const M2<CT> m) {
    if (axis == 0) {
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i & (1 << J)) continue;
            const int k = i | (1 << J);
            CT ur = x.ar[i], ui = x.ai[i], vr = x.ar[k], vi = x.ai[k];
            x.ar[i] = m.ar * ur - m.bi * vi;
            x.ai[i] = m.ar * ui + m.bi * vr;
            x.ar[k] = m.dr * vr - m.ci * ui;
            x.ai[k] = m.dr * vi + m.ci * ur;
            ur = x.br[i]; ui = x.bi[i]; vr = x.br[k]; vi = x.bi[k];
            x.br[i] = m.ar * ur - m.bi * vi;
            x.bi[i] = m.ar * ui + m.bi * vr;
            x.br[k] = m.dr * vr - m.ci * ui;
            x.bi[k] = m.dr * vi + m.ci * ur;
        }
    } else {
#pragma unroll
        for (int i = 0; i < T; ++i) {
            if (i & (1 << J)) continue;
            const int k = i | (1 << J);
            CT ur = x.ar[i], ui = x.ai[i], vr = x.ar[k], vi = x.ai[k];
            x.ar[i] = m.ar * ur + m.br * vr;
            x.ai[i] = m.ar * ui + m.br * vi;
            x.ar[k] = m.cr * ur + m.dr * vr;
            x.ai[k] = m.cr * ui + m.dr * vi;
            ur = x.br[i]; ui = x.bi[i]; vr = x.br[k]; vi = x.bi[k];
            x.br[i] = m.ar * ur + m.br * vr;
            x.bi[i] = m.ar * ui + m.br * vi;
            x.br[k] = m.cr * ur + m.dr * vr;
            x.bi[k] = m.cr * ui + m.dr * vi;
        }
    }
}

// swap the pair of register bit J where the control holds; ctrl has bit i set
// when register i's control value is 1
template <int J, int T, typename CT>
__device__ __forceinline__ void cnot_bit(Regs<CT, T> &x, uint32_t ctrl) {
#pragma unroll
    for (int i = 0; i < T; ++i) {
        if (i & (1 << J)) continue;
        const int k = i | (1 << J);
        const bool c = (ctrl >> i) & 1u;
        const CT a0r = x.ar[i], a0i = x.ai[i], a1r = x.ar[k], a1i = x.ai[k];
        const CT b0r = x.br[i], b0i = x.bi[i], b1r = x.br[k], b1i = x.bi[k];
        x.ar[i] = sel(c, a1r, a0r); x.ar[k] = sel(c, a0r, a1r);
        x.ai[i] = sel(c, a1i, a0i); x.ai[k] = sel(c, a0i, a1i);
        x.br[i] = sel(c, b1r, b0r); x.br[k] = sel(c, b0r, b1r);
        x.bi[i] = sel(c, b1i, b0i); x.bi[k] = sel(c, b0i, b1i);
    }
}

template <int J, int T, typename CT>
__device__ __forceinline__ void rot_prod_bit(int type, int axis, Regs<CT, T> &x, const M2<CT> mm, double &pr,
                                             double &pi) {
    if (type != OP_ROT) prod_bit<J, T, CT>(axis, x, pr, pi);
    if (type != OP_PROD) rot_bit<J, T, CT>(axis, x, mm);
}

// Dispatch a runtime register position j to its template instance.
template <int RB, int T, typename CT>
__device__ __forceinline__ void rot_prod_at(int j, int type, int axis, Regs<CT, T> &x, const M2<CT> mm, double &pr,
                                            double &pi) {
    switch (j) {
    case 0: rot_prod_bit<0, T, CT>(type, axis, x, mm, pr, pi); break;
    case 1: if constexpr (RB > 1) rot_prod_bit<1, T, CT>(type, axis, x, mm, pr, pi); break;
    case 2: if constexpr (RB > 2) rot_prod_bit<2, T, CT>(type, axis, x, mm, pr, pi); break;
    case 3: if constexpr (RB > 3) rot_prod_bit<3, T, CT>(type, axis, x, mm, pr, pi); break;
    default: break;
    }
}

template <int RB, int T, typename CT>
__device__ __forceinline__ void cnot_at(int j, Regs<CT, T> &x, uint32_t ctrl) {
    switch (j) {
    case 0: cnot_bit<0, T, CT>(x, ctrl); break;
    case 1: if constexpr (RB > 1) cnot_bit<1, T, CT>(x, ctrl); break;
    case 2: if constexpr (RB > 2) cnot_bit<2, T, CT>(x, ctrl); break;
    case 3: if constexpr (RB > 3) cnot_bit<3, T, CT>(x, ctrl); break;
    default: break;
    }
}

// Global (element) offset of each of a thread's registers under a mapping.
template <int RB, int T>
__device__ __forceinline__ void global_offsets(const DevPass *pp, const DevMap *mp, int tbits, int tid, uint64_t base,
                                               uint64_t (&off)[T]) {
    uint64_t dth = base;
    for (int t = 0; t < tbits; ++t) dth |= (uint64_t)((tid >> t) & 1) << pp->tile_q[mp->pos[RB + t]];
    uint64_t u[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) u[j] = (uint64_t)1 << pp->tile_q[mp->pos[j]];
#pragma unroll
    for (int i = 0; i < T; ++i) {
        uint64_t d = dth;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if ((i >> j) & 1) d |= u[j];
        off[i] = d;
    }
}

// Local (in-tile) index of each of a thread's registers under a mapping.
template <int RB, int T>
__device__ __forceinline__ void local_offsets(const DevMap *mp, int tbits, int tid, uint32_t (&off)[T]) {
    uint32_t lth = 0;
    for (int t = 0; t < tbits; ++t) lth |= (uint32_t)((tid >> t) & 1) << mp->pos[RB + t];
    uint32_t u[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) u[j] = 1u << mp->pos[j];
#pragma unroll
    for (int i = 0; i < T; ++i) {
        uint32_t l = lth;
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if ((i >> j) & 1) l |= u[j];
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

template <typename R, typename CT, int RB>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(RB >= 4 ? 1 : 3, 8))) void k_sweep_reg(const LaunchItem *__restrict__ items, int n_items,
                                                        const DevPass *__restrict__ passes,
                                                        const DevOp *__restrict__ ops,
                                                        const DevMap *__restrict__ maps,
                                                        const double *__restrict__ mats,
                                                        double2 *__restrict__ partials) {
    constexpr int T = 1 << RB;
    using C = typename Amp<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];

    // ---- which item (one pass of one column) this work-group serves
    const uint32_t wg = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    const LaunchItem it = items[lo];
    const DevPass *pp = passes + it.pass;
    const uint32_t tile = wg - it.tile_begin;
    const int m = pp->m;
    const uint32_t dimT = 1u << m;
    const int tbits = m - RB;
    const int tid = threadIdx.x;
    const bool active = (tid >> tbits) == 0;

    using CX = typename Amp<CT>::T;
    CX *xbuf = (CX *)smem;                                // [2^m] exchange buffer
    double2 *red = (double2 *)(xbuf + dimT);              // [kMaxSlots][kRows]
    double2 *zs = red + kMaxSlots * kRows;                // [kRows]

    uint64_t base = 0;
    for (int k = 0; k < pp->nrest; ++k) base |= (uint64_t)((tile >> k) & 1u) << pp->rest_q[k];

    C *gA = (C *)it.regA;
    C *gB = (C *)it.regB;
    Regs<CT, T> x;

    // ---- load
    const DevMap *cur = maps + pp->map_load;
    {
        uint64_t off[T];
        global_offsets<RB, T>(pp, cur, tbits, tid, base, off);
        if (active) {
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const C v = gA[off[i]];
                x.ar[i] = v.x;
                x.ai[i] = v.y;
            }
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const C v = gB[off[i]];
                x.br[i] = v.x;
                x.bi[i] = v.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < T; ++i) x.ar[i] = x.ai[i] = x.br[i] = x.bi[i] = (CT)0;
        }
    }
    // plain tile sum <A|B>_tile for Z inner products on qubits outside the tile
    double Sr = 0.0, Si = 0.0;
    if (pp->has_zsum) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int i = 0; i < T; ++i) cmac(sr, si, x.ar[i], x.ai[i], x.br[i], x.bi[i]);
        row_store(zs, 0, tid, sr, si);
        __syncthreads();
        for (int w = 0; w < kRows; ++w) {
            Sr += zs[w].x;
            Si += zs[w].y;
        }
    }

    // ---- operations
    const int n_ops = (int)pp->n_ops;
    const DevOp *op_ptr = ops + pp->op_begin;
    for (int oi = 0; oi < n_ops; ++oi) {
        const DevOp op = op_ptr[oi];
        const int type = op.type;
        if (type == OP_ROT || type == OP_PRODROT || type == OP_PROD) {
            const M2<CT> mm = type != OP_PROD ? load_m2<CT>(mats + (size_t)op.gate * 8) : M2<CT>{};
            double pr = 0.0, pi = 0.0;
            rot_prod_at<RB, T, CT>(op.b0, type, op.axis, x, mm, pr, pi);
            if (type != OP_ROT) row_store(red, op.slot, tid, pr, pi);
        } else if (type == OP_DIAG || type == OP_PRODZ || type == OP_PRODDIAG) {
            const uint32_t ones = loc_mask<T>(op.b0, op.q0, tid, base);
            if (type != OP_DIAG) {
                double pr = 0.0, pi = 0.0;
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    double tr = 0.0, ti = 0.0;
                    cmac(tr, ti, x.ar[i], x.ai[i], x.br[i], x.bi[i]);
                    const double sg = ((ones >> i) & 1u) ? -1.0 : 1.0;
                    pr += sg * tr;
                    pi += sg * ti;
                }
                row_store(red, op.slot, tid, pr, pi);
            }
            if (type != OP_PRODZ) {
                const CT d0r = (CT)mats[(size_t)op.gate * 8 + 0], d0i = (CT)mats[(size_t)op.gate * 8 + 1];
                const CT d1r = (CT)mats[(size_t)op.gate * 8 + 6], d1i = (CT)mats[(size_t)op.gate * 8 + 7];
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const bool one = (ones >> i) & 1u;
                    const CT fr = sel(one, d1r, d0r), fi = sel(one, d1i, d0i);
                    cmul<CT>(x.ar[i], x.ai[i], fr, fi);
                    cmul<CT>(x.br[i], x.bi[i], fr, fi);
                }
            }
        } else if (type == OP_CNOT) {
            const uint32_t ctrl = loc_mask<T>(op.b1, op.q0, tid, base);
            if (ctrl) cnot_at<RB, T, CT>(op.b0, x, ctrl);
        } else if (type == OP_CZ) {
            const uint32_t neg = loc_mask<T>(op.b0, op.q0, tid, base) & loc_mask<T>(op.b1, op.q1, tid, base);
#pragma unroll
            for (int i = 0; i < T; ++i) {
                const CT sg = sel<CT>((neg >> i) & 1u, (CT)-1, (CT)1);
                x.ar[i] *= sg;
                x.ai[i] *= sg;
                x.br[i] *= sg;
                x.bi[i] *= sg;
            }
        } else if (type == OP_ZSUM) {
            if (tid == 0) {
                const double sg = ((base >> op.q0) & 1u) ? -1.0 : 1.0;
                red[op.slot * kRows] = make_double2(sg * Sr, sg * Si);
                for (int w = 1; w < kRows; ++w) red[op.slot * kRows + w] = make_double2(0.0, 0.0);
            }
        } else if (type == OP_XPOSE) {
            const DevMap *next = maps + op.aux;
            uint32_t lo_old[T], lo_new[T];
            local_offsets<RB, T>(cur, tbits, tid, lo_old);
            local_offsets<RB, T>(next, tbits, tid, lo_new);
            if (active) {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    CX v;
                    v.x = x.ar[i];
                    v.y = x.ai[i];
                    xbuf[lo_old[i]] = v;
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const CX v = xbuf[lo_new[i]];
                    x.ar[i] = v.x;
                    x.ai[i] = v.y;
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    CX v;
                    v.x = x.br[i];
                    v.y = x.bi[i];
                    xbuf[lo_old[i]] = v;
                }
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int i = 0; i < T; ++i) {
                    const CX v = xbuf[lo_new[i]];
                    x.br[i] = v.x;
                    x.bi[i] = v.y;
                }
            }
            __syncthreads();
            cur = next;
        }
    }

    // ---- store
    {
        uint64_t off[T];
        global_offsets<RB, T>(pp, cur, tbits, tid, base, off);
        if (active) {
#pragma unroll
            for (int i = 0; i < T; ++i) {
                C v;
                v.x = (R)x.ar[i];
                v.y = (R)x.ai[i];
                gA[off[i]] = v;
            }
#pragma unroll
            for (int i = 0; i < T; ++i) {
                C v;
                v.x = (R)x.br[i];
                v.y = (R)x.bi[i];
                gB[off[i]] = v;
            }
        }
    }
    // ---- per-tile partial sums
    __syncthreads();
    for (int k = tid; k < pp->n_slots; k += kThreads) {
        double xr = 0.0, xi = 0.0;
        for (int w = 0; w < kRows; ++w) {
            xr += red[k * kRows + w].x;
            xi += red[k * kRows + w].y;
        }
        partials[it.partial_off + (uint64_t)k * it.ntiles + tile] = make_double2(xr, xi);
    }
}

__global__ __launch_bounds__(kThreads) void k_reduce_tasks(const ReduceTask *__restrict__ tasks,
                                                           const double2 *__restrict__ partials,
                                                           double2 *__restrict__ results) {
    __shared__ double sr[kThreads], si[kThreads];
    const ReduceTask t = tasks[blockIdx.x];
    double a = 0.0, b = 0.0;
    for (uint32_t k = threadIdx.x; k < t.count; k += kThreads) {
        const double2 v = partials[t.off + k];
        a += v.x;
        b += v.y;
    }
    sr[threadIdx.x] = a;
    si[threadIdx.x] = b;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) results[t.dest] = make_double2(sr[0], si[0]);
}

template <typename CT> size_t smem_bytes(int m) {
    return ((size_t)1 << m) * sizeof(typename Amp<CT>::T) + (size_t)(kMaxSlots + 1) * kRows * sizeof(double2);
}

template <typename R, typename CT, int RB>
void launch_rb(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
               const DevMap *maps, const double *mats, double *partials, int m, hipStream_t st) {
    const size_t smem = smem_bytes<CT>(m);
    static size_t attr_set = 0;
    if (smem > attr_set) {
        (void)hipFuncSetAttribute((const void *)k_sweep_reg<R, CT, RB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem);
        (void)hipGetLastError();
        attr_set = smem;
    }
    hipLaunchKernelGGL((k_sweep_reg<R, CT, RB>), dim3(total_tiles), dim3(kThreads), smem, st, items, n_items, passes,
                       ops, maps, mats, (double2 *)partials);
}

template <typename R, typename CT>
void launch_ct(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes, const DevOp *ops,
               const DevMap *maps, const double *mats, double *partials, int m, int rb, hipStream_t st) {
    switch (rb) {
    case 1: launch_rb<R, CT, 1>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st); break;
    case 2: launch_rb<R, CT, 2>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st); break;
    case 3: launch_rb<R, CT, 3>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st); break;
    case 4:
        if constexpr (sizeof(CT) == 4) {
            launch_rb<R, CT, 4>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, st);
            break;
        }
        [[fallthrough]];
    default: throw hipErrorInvalidValue;
    }
}

}  // namespace

template <typename R>
void launch_sweep_pass(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                       const DevOp *ops, const DevMap *maps, const double *mats, double *partials, int m, int rb,
                       bool f64_registers, hipStream_t st) {
    if (n_items <= 0 || total_tiles == 0) return;
    if constexpr (sizeof(R) == 8) {
        (void)f64_registers;
        launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, rb, st);
    } else {
        if (f64_registers)
            launch_ct<R, double>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, rb, st);
        else
            launch_ct<R, float>(items, n_items, total_tiles, passes, ops, maps, mats, partials, m, rb, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

void launch_reduce_tasks(const ReduceTask *tasks, int n_tasks, const double *partials, double *results,
                         hipStream_t st) {
    if (n_tasks <= 0) return;
    hipLaunchKernelGGL(k_reduce_tasks, dim3(n_tasks), dim3(kThreads), 0, st, tasks, (const double2 *)partials,
                       (double2 *)results);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

template void launch_sweep_pass<double>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                        const DevMap *, const double *, double *, int, int, bool, hipStream_t);
template void launch_sweep_pass<float>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                       const DevMap *, const double *, double *, int, int, bool, hipStream_t);

}  // namespace qng
