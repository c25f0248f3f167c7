// sweep_kernels.hip -- the fused sweep-pass kernel for gfx950 (see sweep.hpp).
//
// One work-group (256 threads = 4 wave64) owns one tile: the 2^m amplitudes of
// lambda (A) and phi (B) whose indices agree outside the pass's m tile qubits.
// Load: local index l (bit b <-> qubit tile_q[b], tile qubits ascending, so the
// lowest local bits are the lowest qubits and consecutive threads read
// contiguous runs) -> LDS.  Execute: the pass's operations on LDS, one barrier
// after each; every pair/amplitude is owned by exactly one thread within an
// operation.  Inner products accumulate per thread in FP64, are summed across
// each wave with shuffles and stored per (slot, wave) in LDS.  Store: LDS ->
// the same global addresses (in place: the tile is read and written only by
// this work-group).  Finally one FP64 partial sum per (slot, tile) goes to
// global memory; k_reduce_tasks adds the partials of each slot over all tiles
// in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "sweep.hpp"

namespace qng {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename R> struct Amp;
template <> struct Amp<double> { using T = double2; };
template <> struct Amp<float>  { using T = float2; };

__device__ __forceinline__ uint32_t insert0(uint32_t p, int b) {
    return ((p >> b) << (b + 1)) | (p & ((1u << b) - 1u));
}

__device__ __forceinline__ void wave_sum(double &a, double &b) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
}

// conj(x) * y accumulated in FP64
template <typename C>
__device__ __forceinline__ void cmac(double &sr, double &si, const C &x, const C &y) {
    const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
    sr += xr * yr + xi * yi;
    si += xr * yi - xi * yr;
}

// <a|sigma|b> over the pair (i0, i1) of one qubit: Z: a0*b0 - a1*b1;
// X: a0*b1 + a1*b0; Y: i (a1*b0 - a0*b1)   (a* meaning conj(a))
template <typename C>
__device__ __forceinline__ void pair_prod(int axis, const C &a0, const C &a1, const C &b0, const C &b1, double &sr,
                                          double &si) {
    if (axis == 2) {
        cmac(sr, si, a0, b0);
        double tr = 0.0, ti = 0.0;
        cmac(tr, ti, a1, b1);
        sr -= tr;
        si -= ti;
    } else if (axis == 0) {
        cmac(sr, si, a0, b1);
        cmac(sr, si, a1, b0);
    } else {
        double tr = 0.0, ti = 0.0;
        cmac(tr, ti, a1, b0);
        double ur = 0.0, ui = 0.0;
        cmac(ur, ui, a0, b1);
        tr -= ur;
        ti -= ui;
        sr -= ti;
        si += tr;
    }
}

template <typename R, typename C>
__device__ __forceinline__ void mat_apply(const R *m, C &x0, C &x1) {
    const C u = x0, v = x1;
    x0.x = m[0] * u.x - m[1] * u.y + m[2] * v.x - m[3] * v.y;
    x0.y = m[0] * u.y + m[1] * u.x + m[2] * v.y + m[3] * v.x;
    x1.x = m[4] * u.x - m[5] * u.y + m[6] * v.x - m[7] * v.y;
    x1.y = m[4] * u.y + m[5] * u.x + m[6] * v.y + m[7] * v.x;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void k_sweep_pass(const LaunchItem *__restrict__ items, int n_items,
                                                         const DevPass *__restrict__ passes,
                                                         const DevOp *__restrict__ ops,
                                                         const double *__restrict__ mats,
                                                         double2 *__restrict__ partials) {
    using C = typename Amp<R>::T;
    extern __shared__ __align__(16) unsigned char smem[];

    // which item (pass of one column) this work-group belongs to
    const uint32_t wg = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    const LaunchItem it = items[lo];
    const DevPass *pp = passes + it.pass;      // uniform: read with scalar loads, never copied
    const uint32_t tile = wg - it.tile_begin;
    const int m = pp->m;
    const uint32_t dimT = 1u << m;
    C *A = (C *)smem;
    C *B = A + dimT;
    double2 *red = (double2 *)(B + dimT);          // [kMaxSlots][kWaves]
    double2 *zs = red + kMaxSlots * kWaves;        // [kWaves]
    uint64_t *dep_hi_tab = (uint64_t *)(zs + kWaves);   // [2^(m-8)]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nrest = pp->nrest;
    const int n_ops = (int)pp->n_ops, op_begin = (int)pp->op_begin, n_slots = pp->n_slots;
    const bool has_zsum = pp->has_zsum != 0;

    uint64_t base = 0;
    for (int k = 0; k < nrest; ++k) base |= (uint64_t)((tile >> k) & 1u) << pp->rest_q[k];
    uint64_t dep_lo = 0;
    const int mlo = m < 8 ? m : 8;
    for (int k = 0; k < mlo; ++k) dep_lo |= (uint64_t)((tid >> k) & 1) << pp->tile_q[k];
    const int nhi = m > 8 ? (1 << (m - 8)) : 1;
    if (tid < nhi) {
        uint64_t d = 0;
        for (int k = 8; k < m; ++k) d |= (uint64_t)((tid >> (k - 8)) & 1) << pp->tile_q[k];
        dep_hi_tab[tid] = d;
    }
    __syncthreads();

    C *gA = (C *)it.regA;
    C *gB = (C *)it.regB;

    // ---- load (and the plain tile sum <A|B>_tile if a Z product outside the tile needs it)
    double sr = 0.0, si = 0.0;
    for (uint32_t l = tid; l < dimT; l += kThreads) {
        const uint64_t g = base | dep_lo | dep_hi_tab[l >> 8];
        const C a = gA[g], b = gB[g];
        A[l] = a;
        B[l] = b;
        if (has_zsum) cmac(sr, si, a, b);
    }
    double Sr = 0.0, Si = 0.0;
    if (has_zsum) {
        wave_sum(sr, si);
        if (lane == 0) zs[wave] = make_double2(sr, si);
    }
    __syncthreads();
    if (has_zsum) {
        for (int w = 0; w < kWaves; ++w) { Sr += zs[w].x; Si += zs[w].y; }
    }

    // ---- operations
    const uint32_t npairs = dimT >> 1;
    for (int oi = 0; oi < n_ops; ++oi) {
        const DevOp op = ops[op_begin + oi];
        switch (op.type) {
        case OP_ROT:
        case OP_PRODROT:
        case OP_PROD: {
            const int b = op.b0;
            R mm[8];
            if (op.type != OP_PROD) {
#pragma unroll
                for (int k = 0; k < 8; ++k) mm[k] = (R)mats[(size_t)op.gate * 8 + k];
            }
            double pr = 0.0, pi = 0.0;
            // pairs owned by this thread, processed in batches of kBatch so that the
            // LDS loads of a batch are all in flight before the first is used
            constexpr int kBatch = 4;
            for (uint32_t p0 = tid; p0 < npairs; p0 += kThreads * kBatch) {
                uint32_t i0[kBatch];
                C a0[kBatch], a1[kBatch], b0[kBatch], b1[kBatch];
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    const uint32_t p = p0 + j * kThreads;
                    i0[j] = insert0(p < npairs ? p : 0u, b);
                    a0[j] = A[i0[j]]; a1[j] = A[i0[j] | (1u << b)];
                    b0[j] = B[i0[j]]; b1[j] = B[i0[j] | (1u << b)];
                }
#pragma unroll
                for (int j = 0; j < kBatch; ++j) {
                    if (p0 + j * kThreads >= npairs) continue;
                    if (op.type != OP_ROT) pair_prod(op.axis, a0[j], a1[j], b0[j], b1[j], pr, pi);
                    if (op.type != OP_PROD) {
                        mat_apply<R, C>(mm, a0[j], a1[j]);
                        mat_apply<R, C>(mm, b0[j], b1[j]);
                        A[i0[j]] = a0[j]; A[i0[j] | (1u << b)] = a1[j];
                        B[i0[j]] = b0[j]; B[i0[j] | (1u << b)] = b1[j];
                    }
                }
            }
            if (op.type != OP_ROT) {
                wave_sum(pr, pi);
                if (lane == 0) red[op.slot * kWaves + wave] = make_double2(pr, pi);
            }
            break;
        }
        case OP_CNOT: {
            const int bt = op.b1;
            if (op.b0 == kNoBit) {
                if (!((base >> op.q0) & 1u)) break;   // control fixed to 0 on this tile
                for (uint32_t p = tid; p < npairs; p += kThreads) {
                    const uint32_t i0 = insert0(p, bt), i1 = i0 | (1u << bt);
                    const C a0 = A[i0], b0 = B[i0];
                    A[i0] = A[i1]; A[i1] = a0;
                    B[i0] = B[i1]; B[i1] = b0;
                }
            } else {
                const uint32_t cb = 1u << op.b0;
                for (uint32_t p = tid; p < npairs; p += kThreads) {
                    const uint32_t i0 = insert0(p, bt), i1 = i0 | (1u << bt);
                    if (!(i0 & cb)) continue;
                    const C a0 = A[i0], b0 = B[i0];
                    A[i0] = A[i1]; A[i1] = a0;
                    B[i0] = B[i1]; B[i1] = b0;
                }
            }
            break;
        }
        case OP_CZ: {
            const bool la = op.b0 != kNoBit, lb = op.b1 != kNoBit;
            const uint32_t fa = la ? 0u : (uint32_t)((base >> op.q0) & 1u);
            const uint32_t fb = lb ? 0u : (uint32_t)((base >> op.q1) & 1u);
            for (uint32_t l = tid; l < dimT; l += kThreads) {
                const uint32_t xa = la ? (l >> op.b0) & 1u : fa;
                const uint32_t xb = lb ? (l >> op.b1) & 1u : fb;
                if (xa & xb) {
                    C a = A[l], b = B[l];
                    a.x = -a.x; a.y = -a.y; b.x = -b.x; b.y = -b.y;
                    A[l] = a; B[l] = b;
                }
            }
            break;
        }
        case OP_ZSUM: {
            if (tid == 0) {
                const double sg = ((base >> op.q0) & 1u) ? -1.0 : 1.0;
                red[op.slot * kWaves] = make_double2(sg * Sr, sg * Si);
                for (int w = 1; w < kWaves; ++w) red[op.slot * kWaves + w] = make_double2(0.0, 0.0);
            }
            break;
        }
        default: break;
        }
        __syncthreads();
    }

    // ---- store
    for (uint32_t l = tid; l < dimT; l += kThreads) {
        const uint64_t g = base | dep_lo | dep_hi_tab[l >> 8];
        gA[g] = A[l];
        gB[g] = B[l];
    }
    // ---- per-tile partial sums
    for (int k = tid; k < n_slots; k += kThreads) {
        double xr = 0.0, xi = 0.0;
        for (int w = 0; w < kWaves; ++w) { xr += red[k * kWaves + w].x; xi += red[k * kWaves + w].y; }
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

template <typename R> size_t smem_bytes(int m) {
    return 2 * ((size_t)1 << m) * sizeof(typename Amp<R>::T) + (size_t)(kMaxSlots + 1) * kWaves * sizeof(double2) +
           32 * sizeof(uint64_t);
}

}  // namespace

template <typename R>
void launch_sweep_pass(const LaunchItem *items, int n_items, uint32_t total_tiles, const DevPass *passes,
                       const DevOp *ops, const double *mats, double *partials, int max_m, hipStream_t st) {
    if (n_items <= 0 || total_tiles == 0) return;
    const size_t smem = smem_bytes<R>(max_m);
    static size_t attr_set = 0;
    if (smem > attr_set) {
        (void)hipFuncSetAttribute((const void *)k_sweep_pass<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)smem);
        (void)hipGetLastError();
        attr_set = smem;
    }
    hipLaunchKernelGGL(k_sweep_pass<R>, dim3(total_tiles), dim3(kThreads), smem, st, items, n_items, passes, ops, mats,
                       (double2 *)partials);
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
                                        const double *, double *, int, hipStream_t);
template void launch_sweep_pass<float>(const LaunchItem *, int, uint32_t, const DevPass *, const DevOp *,
                                       const double *, double *, int, hipStream_t);

}  // namespace qng
