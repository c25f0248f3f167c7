// kernels.hip -- per-primitive HIP kernels for gfx950 (clone, apply gate,
// inner product, Pauli-sum Hamiltonian).  See kernels.hpp.
//
// Layout: a register of n qubits is 2^n interleaved complex amplitudes of
// element type R; qubit q is bit q of the index.  A single-qubit gate on q
// pairs amplitudes i0 (bit q clear) and i1 = i0 | 2^q; consecutive threads
// take consecutive pair indices, so loads and stores are coalesced for every q
// (for q >= 1 both halves are contiguous runs; for q = 0 each thread touches one
// 2-amplitude run).
#include <hip/hip_runtime.h>

#include <utility>

#include "kernels.hpp"

namespace qng {

namespace {

constexpr int kBlock = 256;
constexpr int kReduceBlocksMax = 1024;

template <typename R> struct Cplx;
template <> struct Cplx<double> { using T = double2; };
template <> struct Cplx<float>  { using T = float2; };

__device__ __forceinline__ uint64_t insert_zero(uint64_t p, int q) {
    const uint64_t low = p & ((uint64_t(1) << q) - 1);
    return ((p >> q) << (q + 1)) | low;
}

__device__ __forceinline__ uint64_t insert_two_zeros(uint64_t p, int lo, int hi) {
    return insert_zero(insert_zero(p, lo), hi);   // lo < hi
}

// Loads and stores with the nontemporal hint: a state streamed once through a
// kernel is not kept in the caches.  Measured on a 2^26 complex64 state, an
// isolated rotation on a target qubit q >= 4 moves 5.8-6.7 TB/s with the hint
// against 5.1-6.2 TB/s without (the dip at q = 19-23 was the worst case); for
// q < 4 the two amplitudes of a pair share cache lines and the plain accesses
// are faster (5.9 against 5.6 TB/s), so the rotation launchers pick the hint by
// qubit.  CNOT and CZ, which rewrite only part of each line, and the clone
// were slower with it (CZ 4.6-5.5 against 6.5-7.0 TB/s) and keep plain
// accesses; so do the sweep passes, whose reverse tile order relies on the
// last pass's tiles still being in the caches (3.5 ms against 1.8 ms a pass).
template <typename V> struct NtVec;
template <> struct NtVec<double2> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct NtVec<float2> { typedef float T __attribute__((ext_vector_type(2))); };
template <bool NT, typename V> __device__ __forceinline__ V load_amp(const V *p) {
    if constexpr (NT) {
        const typename NtVec<V>::T v = __builtin_nontemporal_load((const typename NtVec<V>::T *)p);
        V o;
        o.x = v.x;
        o.y = v.y;
        return o;
    } else {
        return *p;
    }
}
template <bool NT, typename V> __device__ __forceinline__ void store_amp(V *p, V v) {
    if constexpr (NT) {
        typename NtVec<V>::T w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, (typename NtVec<V>::T *)p);
    } else {
        *p = v;
    }
}
constexpr int kNtMinQubit = 4;

inline unsigned grid_for(uint64_t work) {
    uint64_t g = (work + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > (uint64_t(1) << 20)) g = uint64_t(1) << 20;
    return (unsigned)g;
}

inline void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

// ------------------------------------------------------------------ state init

template <typename R>
__global__ void k_init_state(typename Cplx<R>::T *dst, uint64_t dim, const double2 *src) {
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        typename Cplx<R>::T v;
        if (src) { v.x = (R)src[x].x; v.y = (R)src[x].y; }
        else     { v.x = (R)(x == 0 ? 1.0 : 0.0); v.y = (R)0; }
        dst[x] = v;
    }
}

template <typename R>
__global__ void k_to_c128(const typename Cplx<R>::T *src, double2 *dst, uint64_t dim) {
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        const typename Cplx<R>::T v = src[x];
        dst[x] = make_double2((double)v.x, (double)v.y);
    }
}

template <typename R>
__global__ void k_copy(const typename Cplx<R>::T *src, typename Cplx<R>::T *dst, uint64_t dim) {
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock)
        dst[x] = src[x];
}

// ------------------------------------------------------------------ gates

template <typename R, bool NT = false>
__device__ __forceinline__ void mat_pair(typename Cplx<R>::T *s, uint64_t i0, uint64_t i1, R ar, R ai, R br, R bi,
                                         R cr, R ci, R dr, R di) {
    const typename Cplx<R>::T u = load_amp<NT>(s + i0), v = load_amp<NT>(s + i1);
    typename Cplx<R>::T o0, o1;
    o0.x = ar * u.x - ai * u.y + br * v.x - bi * v.y;
    o0.y = ar * u.y + ai * u.x + br * v.y + bi * v.x;
    o1.x = cr * u.x - ci * u.y + dr * v.x - di * v.y;
    o1.y = cr * u.y + ci * u.x + dr * v.y + di * v.x;
    store_amp<NT>(s + i0, o0);
    store_amp<NT>(s + i1, o1);
}

template <typename R, bool NT>
__global__ void k_apply_1q(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int q, DevMat2 m) {
    const uint64_t npairs = uint64_t(1) << (n - 1);
    const R ar = (R)m.ar, ai = (R)m.ai, br = (R)m.br, bi = (R)m.bi;
    const R cr = (R)m.cr, ci = (R)m.ci, dr = (R)m.dr, di = (R)m.di;
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_zero(p, q), i1 = i0 | (uint64_t(1) << q);
        mat_pair<R, NT>(s0, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
        if (s1) mat_pair<R, NT>(s1, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
    }
}

// Same, with the matrix read from device memory (8 doubles, row-major re/im):
// launches whose arguments do not depend on the angles can be captured once
// and replayed with new matrices.
template <typename R, bool NT>
__global__ void k_apply_1q_tab(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int q,
                               const double *__restrict__ mt) {
    const uint64_t npairs = uint64_t(1) << (n - 1);
    const R ar = (R)mt[0], ai = (R)mt[1], br = (R)mt[2], bi = (R)mt[3];
    const R cr = (R)mt[4], ci = (R)mt[5], dr = (R)mt[6], di = (R)mt[7];
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_zero(p, q), i1 = i0 | (uint64_t(1) << q);
        mat_pair<R, NT>(s0, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
        if (s1) mat_pair<R, NT>(s1, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
    }
}

// Controlled single-qubit gate: the matrix acts on the pairs (x, x | 2^q) whose
// control bit c is 1 (a quarter index p enumerates the pairs with bit c set and
// bit q clear); the other amplitudes keep their values.
template <typename R>
__global__ void k_apply_c1q(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int c, int q, DevMat2 m) {
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int lo = c < q ? c : q, hi = c < q ? q : c;
    const R ar = (R)m.ar, ai = (R)m.ai, br = (R)m.br, bi = (R)m.bi;
    const R cr = (R)m.cr, ci = (R)m.ci, dr = (R)m.dr, di = (R)m.di;
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_two_zeros(p, lo, hi) | (uint64_t(1) << c), i1 = i0 | (uint64_t(1) << q);
        mat_pair<R>(s0, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
        if (s1) mat_pair<R>(s1, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
    }
}

// Same, with the matrix read from device memory (as k_apply_1q_tab).
template <typename R>
__global__ void k_apply_c1q_tab(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int c, int q,
                                const double *__restrict__ mt) {
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int lo = c < q ? c : q, hi = c < q ? q : c;
    const R ar = (R)mt[0], ai = (R)mt[1], br = (R)mt[2], bi = (R)mt[3];
    const R cr = (R)mt[4], ci = (R)mt[5], dr = (R)mt[6], di = (R)mt[7];
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_two_zeros(p, lo, hi) | (uint64_t(1) << c), i1 = i0 | (uint64_t(1) << q);
        mat_pair<R>(s0, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
        if (s1) mat_pair<R>(s1, i0, i1, ar, ai, br, bi, cr, ci, dr, di);
    }
}

// Pauli string S in mask form: (S psi)[x] = w (-1)^{popcount(x & zy)} psi[x ^ flip],
// w = (-i)^{n_y}.  A rotation c + kappa S' with S' the string without w (the
// host folds w and i sin into kappa): out[x] = c psi[x] + kappa sgn(x) psi[x ^ flip].
// flip != 0: pairs (x0, x0 ^ flip) with the highest bit hb of flip clear in x0;
// flip == 0: a diagonal phase.
__device__ __forceinline__ double string_sign(uint64_t x, uint64_t zy) { return (__popcll(x & zy) & 1) ? -1.0 : 1.0; }

template <typename R>
__device__ __forceinline__ void string_pair(typename Cplx<R>::T *s, uint64_t x0, uint64_t x1, R c, R kr, R ki, R g0,
                                            R g1) {
    const typename Cplx<R>::T u = s[x0], v = s[x1];
    typename Cplx<R>::T o0, o1;
    o0.x = c * u.x + g0 * (kr * v.x - ki * v.y);
    o0.y = c * u.y + g0 * (kr * v.y + ki * v.x);
    o1.x = c * v.x + g1 * (kr * u.x - ki * u.y);
    o1.y = c * v.y + g1 * (kr * u.y + ki * u.x);
    s[x0] = o0;
    s[x1] = o1;
}

template <typename R>
__global__ void k_apply_string(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, uint64_t flip, uint64_t zy,
                               double c, double kr, double ki) {
    const R cc = (R)c, kkr = (R)kr, kki = (R)ki;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    if (flip) {
        const int hb = 63 - __clzll(flip);
        const uint64_t npairs = uint64_t(1) << (n - 1);
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += stride) {
            const uint64_t x0 = insert_zero(p, hb), x1 = x0 ^ flip;
            const R g0 = (R)string_sign(x0, zy), g1 = (R)string_sign(x1, zy);
            string_pair<R>(s0, x0, x1, cc, kkr, kki, g0, g1);
            if (s1) string_pair<R>(s1, x0, x1, cc, kkr, kki, g0, g1);
        }
    } else {
        const uint64_t dim = uint64_t(1) << n;
        for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += stride) {
            const R g = (R)string_sign(x, zy);
            const R fr = cc + g * kkr, fi = g * kki;
            typename Cplx<R>::T *regs[2] = {s0, s1};
            for (int k = 0; k < 2; ++k) {
                if (!regs[k]) continue;
                const typename Cplx<R>::T u = regs[k][x];
                typename Cplx<R>::T o;
                o.x = fr * u.x - fi * u.y;
                o.y = fr * u.y + fi * u.x;
                regs[k][x] = o;
            }
        }
    }
}

// lam = y; phi = S y with S = w S' (w = wr + i wi, a power of -i).
template <typename R>
__global__ void k_seed_string(const typename Cplx<R>::T *y, typename Cplx<R>::T *lam, typename Cplx<R>::T *phi, int n,
                              uint64_t flip, uint64_t zy, double wr, double wi) {
    const uint64_t dim = uint64_t(1) << n;
    const R ar = (R)wr, ai = (R)wi;
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        lam[x] = y[x];
        const typename Cplx<R>::T v = y[x ^ flip];
        const R g = (R)string_sign(x, zy);
        typename Cplx<R>::T o;
        o.x = g * (ar * v.x - ai * v.y);
        o.y = g * (ar * v.y + ai * v.x);
        phi[x] = o;
    }
}

// CNOT(control c, target t): swap amplitudes (x, x ^ 2^t) for x with bit c set and bit t clear.
template <typename R, bool NT>
__global__ void k_cnot(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int c, int t) {
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int lo = c < t ? c : t, hi = c < t ? t : c;
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_two_zeros(p, lo, hi) | (uint64_t(1) << c);
        const uint64_t i1 = i0 | (uint64_t(1) << t);
        typename Cplx<R>::T u = load_amp<NT>(s0 + i0), v = load_amp<NT>(s0 + i1);
        store_amp<NT>(s0 + i0, v);
        store_amp<NT>(s0 + i1, u);
        if (s1) {
            u = load_amp<NT>(s1 + i0);
            v = load_amp<NT>(s1 + i1);
            store_amp<NT>(s1 + i0, v);
            store_amp<NT>(s1 + i1, u);
        }
    }
}

// A run of CNOTs as one gather: undoing the run on the output index y (its
// CNOTs in reverse order, each its own inverse) gives the input index.
struct CnotRun {
    uint8_t c[kCnotRunMax], t[kCnotRunMax];
    int count;
};

template <typename R>
__global__ void k_cnot_run(const typename Cplx<R>::T *src, typename Cplx<R>::T *dst, int n, CnotRun run) {
    const uint64_t dim = uint64_t(1) << n;
    for (uint64_t y = blockIdx.x * (uint64_t)kBlock + threadIdx.x; y < dim; y += (uint64_t)gridDim.x * kBlock) {
        uint64_t x = y;
        for (int k = run.count - 1; k >= 0; --k) x ^= ((x >> run.c[k]) & 1) << run.t[k];
        dst[y] = src[x];
    }
}

// CZ(a, b): negate amplitudes with both bits set.
template <typename R, bool NT>
__global__ void k_cz(typename Cplx<R>::T *s0, typename Cplx<R>::T *s1, int n, int a, int b) {
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i = insert_two_zeros(p, lo, hi) | (uint64_t(1) << a) | (uint64_t(1) << b);
        typename Cplx<R>::T u = load_amp<NT>(s0 + i);
        u.x = -u.x; u.y = -u.y;
        store_amp<NT>(s0 + i, u);
        if (s1) {
            u = load_amp<NT>(s1 + i);
            u.x = -u.x; u.y = -u.y;
            store_amp<NT>(s1 + i, u);
        }
    }
}

// lam = y; phi = sigma_q y.   (X: swap; Y: phi0 = -i y1, phi1 = i y0; Z: phi1 = -y1)
// With a control qubit c >= 0 the generator is |1><1|_c (x) sigma_q: phi is
// zero on the amplitudes whose bit c is 0 (c != q).
template <typename R>
__global__ void k_seed(const typename Cplx<R>::T *y, typename Cplx<R>::T *lam, typename Cplx<R>::T *phi, int n, int q,
                       int axis, int c) {
    const uint64_t npairs = uint64_t(1) << (n - 1);
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t i0 = insert_zero(p, q), i1 = i0 | (uint64_t(1) << q);
        const typename Cplx<R>::T u = y[i0], v = y[i1];
        lam[i0] = u;
        lam[i1] = v;
        typename Cplx<R>::T o0, o1;
        if (axis == 0) { o0 = v; o1 = u; }
        else if (axis == 1) { o0.x = v.y; o0.y = -v.x; o1.x = -u.y; o1.y = u.x; }
        else { o0 = u; o1.x = -v.x; o1.y = -v.y; }
        if (c >= 0 && !((i0 >> c) & 1)) { o0.x = o0.y = o1.x = o1.y = (R)0; }
        phi[i0] = o0;
        phi[i1] = o1;
    }
}

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ void block_reduce_store(double sr, double si, double *out2) {
    __shared__ double sh[2 * kBlock];
    sh[threadIdx.x] = sr;
    sh[kBlock + threadIdx.x] = si;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[threadIdx.x] += sh[threadIdx.x + w];
            sh[kBlock + threadIdx.x] += sh[kBlock + threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { out2[0] = sh[0]; out2[1] = sh[kBlock]; }
}

// conj(a) * b accumulated in FP64
__device__ __forceinline__ void cmac(double &sr, double &si, double ar, double ai, double br, double bi) {
    sr += ar * br + ai * bi;
    si += ar * bi - ai * br;
}

// Block partials of <a| sigma_q |b> (axis 0/1/2; axis < 0: the identity).
// With a control qubit c >= 0 the operator is |1><1|_c (x) sigma_q: only the
// amplitudes whose bit c is 1 contribute (c != q; for axis < 0, q is ignored).
template <typename R>
__global__ void k_pauli_prod_partial(const typename Cplx<R>::T *a, const typename Cplx<R>::T *b, int n, int q,
                                     int axis, int c, double *partials) {
    double sr = 0.0, si = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    if (axis < 0) {
        const uint64_t dim = uint64_t(1) << (c >= 0 ? n - 1 : n);
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < dim; p += stride) {
            const uint64_t x = c >= 0 ? insert_zero(p, c) | (uint64_t(1) << c) : p;
            const typename Cplx<R>::T u = a[x], v = b[x];
            cmac(sr, si, u.x, u.y, v.x, v.y);
        }
    } else {
        const uint64_t npairs = uint64_t(1) << (c >= 0 ? n - 2 : n - 1);
        const int lo = c < q ? c : q, hi = c < q ? q : c;
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += stride) {
            const uint64_t i0 = c >= 0 ? insert_two_zeros(p, lo, hi) | (uint64_t(1) << c) : insert_zero(p, q);
            const uint64_t i1 = i0 | (uint64_t(1) << q);
            const typename Cplx<R>::T a0 = a[i0], a1 = a[i1], b0 = b[i0], b1 = b[i1];
            if (axis == 2) {            // conj(a0) b0 - conj(a1) b1
                cmac(sr, si, a0.x, a0.y, b0.x, b0.y);
                cmac(sr, si, -(double)a1.x, -(double)a1.y, b1.x, b1.y);
            } else if (axis == 0) {     // conj(a0) b1 + conj(a1) b0
                cmac(sr, si, a0.x, a0.y, b1.x, b1.y);
                cmac(sr, si, a1.x, a1.y, b0.x, b0.y);
            } else {                    // i (conj(a1) b0 - conj(a0) b1)
                double tr = 0.0, ti = 0.0;
                cmac(tr, ti, a1.x, a1.y, b0.x, b0.y);
                cmac(tr, ti, -(double)a0.x, -(double)a0.y, b1.x, b1.y);
                sr += -ti;
                si += tr;
            }
        }
    }
    block_reduce_store(sr, si, partials + 2 * blockIdx.x);
}

// Block partials of <a| S |b> = w sum_x conj(a[x]) sgn(x) b[x ^ flip] (w = wr + i wi).
template <typename R>
__global__ void k_string_prod_partial(const typename Cplx<R>::T *a, const typename Cplx<R>::T *b, int n,
                                      uint64_t flip, uint64_t zy, double wr, double wi, double *partials) {
    double sr = 0.0, si = 0.0;
    const uint64_t dim = uint64_t(1) << n;
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        const typename Cplx<R>::T u = a[x], v = b[x ^ flip];
        const double g = string_sign(x, zy);
        cmac(sr, si, g * (double)u.x, g * (double)u.y, v.x, v.y);
    }
    block_reduce_store(sr * wr - si * wi, sr * wi + si * wr, partials + 2 * blockIdx.x);
}

__global__ void k_reduce_final(const double *partials, int nb, double *dest) {
    double sr = 0.0, si = 0.0;
    for (int k = threadIdx.x; k < nb; k += kBlock) { sr += partials[2 * k]; si += partials[2 * k + 1]; }
    block_reduce_store(sr, si, dest);
}

// ------------------------------------------------------------------ column start

// sigma (axis 0/1/2 = X/Y/Z) on the pair (u, v): (o0, o1)
template <typename C>
__device__ __forceinline__ void pauli_pair(int axis, const C &u, const C &v, C &o0, C &o1) {
    if (axis == 0) { o0 = v; o1 = u; }
    else if (axis == 1) { o0.x = v.y; o0.y = -v.x; o1.x = -u.y; o1.y = u.x; }
    else { o0 = u; o1.x = -v.x; o1.y = -v.y; }
}

// One pass over the forward register for the start of a column s:
//   psi <- R psi (the rotation just before y_s, matrix mt; qr < 0: none),
//   lam = psi, phi = sigma_s psi, and the block partials of <psi|sigma_s|psi>.
// (Replaces apply + inner product + seed, which read psi three times.)
template <typename R>
__global__ void k_advance_seed(typename Cplx<R>::T *psi, typename Cplx<R>::T *lam, typename Cplx<R>::T *phi, int n,
                               int qr, const double *__restrict__ mt, int qs, int axis, double *partials) {
    using C = typename Cplx<R>::T;
    R ar = 0, ai = 0, br = 0, bi = 0, cr = 0, ci = 0, dr = 0, di = 0;
    if (qr >= 0) {
        ar = (R)mt[0]; ai = (R)mt[1]; br = (R)mt[2]; bi = (R)mt[3];
        cr = (R)mt[4]; ci = (R)mt[5]; dr = (R)mt[6]; di = (R)mt[7];
    }
    auto rot = [&](C &u, C &v) {
        const C a = u, b = v;
        u.x = ar * a.x - ai * a.y + br * b.x - bi * b.y;
        u.y = ar * a.y + ai * a.x + br * b.y + bi * b.x;
        v.x = cr * a.x - ci * a.y + dr * b.x - di * b.y;
        v.y = cr * a.y + ci * a.x + dr * b.y + di * b.x;
    };
    double sr = 0.0, si = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t ms = uint64_t(1) << qs;
    if (qr < 0 || qr == qs) {
        const uint64_t npairs = uint64_t(1) << (n - 1);
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += stride) {
            const uint64_t i0 = insert_zero(p, qs), i1 = i0 | ms;
            C u = psi[i0], v = psi[i1];
            if (qr >= 0) {
                rot(u, v);
                psi[i0] = u;
                psi[i1] = v;
            }
            C o0, o1;
            pauli_pair(axis, u, v, o0, o1);
            lam[i0] = u; lam[i1] = v;
            phi[i0] = o0; phi[i1] = o1;
            cmac(sr, si, u.x, u.y, o0.x, o0.y);
            cmac(sr, si, v.x, v.y, o1.x, o1.y);
        }
    } else {
        const uint64_t mr = uint64_t(1) << qr;
        const int lo = qr < qs ? qr : qs, hi = qr < qs ? qs : qr;
        const uint64_t nq = uint64_t(1) << (n - 2);
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += stride) {
            const uint64_t b = insert_two_zeros(p, lo, hi);
            C y00 = psi[b], y10 = psi[b | mr], y01 = psi[b | ms], y11 = psi[b | mr | ms];
            rot(y00, y10);
            rot(y01, y11);
            psi[b] = y00; psi[b | mr] = y10; psi[b | ms] = y01; psi[b | mr | ms] = y11;
            lam[b] = y00; lam[b | mr] = y10; lam[b | ms] = y01; lam[b | mr | ms] = y11;
            C o00, o01, o10, o11;
            pauli_pair(axis, y00, y01, o00, o01);
            pauli_pair(axis, y10, y11, o10, o11);
            phi[b] = o00; phi[b | ms] = o01; phi[b | mr] = o10; phi[b | mr | ms] = o11;
            cmac(sr, si, y00.x, y00.y, o00.x, o00.y);
            cmac(sr, si, y01.x, y01.y, o01.x, o01.y);
            cmac(sr, si, y10.x, y10.y, o10.x, o10.y);
            cmac(sr, si, y11.x, y11.y, o11.x, o11.y);
        }
    }
    block_reduce_store(sr, si, partials + 2 * blockIdx.x);
}

// Column seeds of many registers in one launch (the batched metric): item k
// applies up to two forward rotations (qa then qb; -1: none) to its register
// psi, then writes lam = psi, phi = sigma_qs psi and its work-groups' partial
// sums of <psi|sigma_qs|psi>.  A thread walks groups of eight amplitudes over
// three distinct bits in fixed slots -- slot 0 the seeded qubit qs, slot 1 qa
// (unless it is qs), slot 2 qb, the lowest other qubits where those are fewer
// (registers of at least 3 qubits) -- so that every amplitude index within a
// group is a constant and the group stays in registers.  The work-groups of
// item k are block_begin .. block_begin + nblocks - 1; each writes one partial
// at its own index.
// (the matrix entries in the register's precision, as in k_advance_seed)
template <typename R, typename C>
__device__ __forceinline__ void rot_pair(const double *m, C &u, C &v) {
    const C a = u, b = v;
    const R m0 = (R)m[0], m1 = (R)m[1], m2 = (R)m[2], m3 = (R)m[3];
    const R m4 = (R)m[4], m5 = (R)m[5], m6 = (R)m[6], m7 = (R)m[7];
    u.x = m0 * a.x - m1 * a.y + m2 * b.x - m3 * b.y;
    u.y = m0 * a.y + m1 * a.x + m2 * b.y + m3 * b.x;
    v.x = m4 * a.x - m5 * a.y + m6 * b.x - m7 * b.y;
    v.y = m4 * a.y + m5 * a.x + m6 * b.y + m7 * b.x;
}
// the rotation m on slot J of a group of eight
template <int J, typename R, typename C>
__device__ __forceinline__ void rot_slot(const double *m, C (&v)[8]) {
#pragma unroll
    for (int g = 0; g < 8; ++g)
        if (!(g & (1 << J))) rot_pair<R>(m, v[g], v[g | (1 << J)]);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_seed_multi(const SeedItem *__restrict__ items, int n_items, double *partials) {
    using C = typename Cplx<R>::T;
    const uint32_t wg = blockIdx.x;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].block_begin <= wg) lo = mid;
        else hi = mid - 1;
    }
    const SeedItem it = items[lo];
    C *psi = (C *)it.psi, *lam = (C *)it.lam, *phi = (C *)it.phi;
    // the qubits of the three slots (qb, when given, differs from qs and qa)
    const int s0 = it.qs;
    int s1 = (it.qa >= 0 && it.qa != s0) ? it.qa : -1;
    int s2 = it.qb;
    int f = 0;   // lowest qubit not taken yet
    if (s1 < 0) {
        while (f == s0 || f == s2) ++f;
        s1 = f++;
    }
    if (s2 < 0) {
        while (f == s0 || f == s1) ++f;
        s2 = f;
    }
    const int ja = it.qa < 0 ? -1 : (it.qa == s0 ? 0 : 1);   // slot of rotation a
    // ascending for the zero insertions
    const int b0 = min(s0, min(s1, s2)), b2 = max(s0, max(s1, s2)), b1 = s0 + s1 + s2 - b0 - b2;
    const uint64_t m0 = uint64_t(1) << s0, m1 = uint64_t(1) << s1, m2 = uint64_t(1) << s2;
    double sr = 0.0, si = 0.0;
    const uint64_t ngroups = uint64_t(1) << (it.n - 3);
    const uint64_t stride = (uint64_t)it.nblocks * kBlock;
    for (uint64_t p = (uint64_t)(wg - it.block_begin) * kBlock + threadIdx.x; p < ngroups; p += stride) {
        const uint64_t b = insert_zero(insert_zero(insert_zero(p, b0), b1), b2);
        C v[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) v[g] = psi[b | ((g & 1) ? m0 : 0) | ((g & 2) ? m1 : 0) | ((g & 4) ? m2 : 0)];
        if (ja == 0) rot_slot<0, R>(it.ma, v);
        else if (ja == 1) rot_slot<1, R>(it.ma, v);
        if (it.qb >= 0) rot_slot<2, R>(it.mb, v);
        C o[8];
#pragma unroll
        for (int g = 0; g < 8; g += 2) pauli_pair(it.axis, v[g], v[g + 1], o[g], o[g + 1]);
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const uint64_t x = b | ((g & 1) ? m0 : 0) | ((g & 2) ? m1 : 0) | ((g & 4) ? m2 : 0);
            if (ja >= 0) psi[x] = v[g];
            lam[x] = v[g];
            phi[x] = o[g];
            cmac(sr, si, v[g].x, v[g].y, o[g].x, o[g].y);
        }
    }
    block_reduce_store(sr, si, partials + 2 * wg);
}

// ------------------------------------------------------------------ sweep steps
//
// One step of the recurrence's back sweep over lambda and several phi
// registers at once (columns of one block): for the rotation r at this step,
// <lambda|K_r|phi_k> for every phi register from the values before the step,
// then the adjoint of r on lambda and every phi (K_r commutes with r, so the
// product is the same before or after).  The threads walk the index groups of
// the rotation's own structure, which is also the structure of K_r:
//   STEP_1Q     pairs (i0, i0 | 2^q), K = sigma on the pair;
//   STEP_C1Q    the pairs with control bit c set, K = sigma there (zero elsewhere,
//               where the gate also acts as the identity);
//   STEP_STRING pairs (x0, x0 ^ flip) with the highest flip bit clear in x0, or
//               single amplitudes when flip = 0; K = S.

template <typename C>
__device__ __forceinline__ C cmul(C a, double br, double bi) {   // a * (br + i bi)
    C o;
    o.x = a.x * br - a.y * bi;
    o.y = a.x * bi + a.y * br;
    return o;
}

// 2x2 adjoint matrix (row-major a, b, c, d; re, im) on the pair (u, v)
template <typename C, typename RR>
__device__ __forceinline__ void mat2(const RR (&m)[8], C &u, C &v) {
    const C a = u, b = v;
    u.x = m[0] * a.x - m[1] * a.y + m[2] * b.x - m[3] * b.y;
    u.y = m[0] * a.y + m[1] * a.x + m[2] * b.y + m[3] * b.x;
    v.x = m[4] * a.x - m[5] * a.y + m[6] * b.x - m[7] * b.y;
    v.y = m[4] * a.y + m[5] * a.x + m[6] * b.y + m[7] * b.x;
}

template <int KIND, typename R>
__global__ void k_sweep_step(StepRegs regs, StepGate g, double *partials) {
    using C = typename Cplx<R>::T;
    constexpr int M = kStepMaxPhi;
    const int nphi = regs.n_phi;
    const int n = g.n;
    R m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) m[k] = (R)g.m[k];
    double sr[M], si[M];
#pragma unroll
    for (int k = 0; k < M; ++k) sr[k] = si[k] = 0.0;
    C *lam = (C *)regs.lam;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    // K on a pair of values (w0, w1) at indices (x0, x1): (o0, o1)
    auto apply_k = [&](const C &w0, const C &w1, uint64_t x0, uint64_t x1, C &o0, C &o1) {
        if constexpr (KIND == STEP_STRING) {
            const double g0 = string_sign(x0, g.zy), g1 = string_sign(x1, g.zy);
            o0 = cmul(w1, g0 * g.wr, g0 * g.wi);
            o1 = cmul(w0, g1 * g.wr, g1 * g.wi);
        } else {
            pauli_pair(g.axis, w0, w1, o0, o1);
        }
    };
    if (KIND == STEP_STRING && g.flip == 0) {
        // diagonal string: K = sgn(x) (no Y letter), the adjoint is c + kappa sgn(x)
        const uint64_t dim = uint64_t(1) << n;
        for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += stride) {
            const double gx = string_sign(x, g.zy);
            const R fr = m[0] + (R)gx * m[2], fi = (R)gx * m[3];
            const C l = lam[x];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                if (k >= nphi) break;
                C *ph = (C *)regs.phi[k];
                C f = ph[x];
                cmac(sr[k], si[k], l.x, l.y, gx * (double)f.x, gx * (double)f.y);
                const C t = f;
                f.x = fr * t.x - fi * t.y;
                f.y = fr * t.y + fi * t.x;
                ph[x] = f;
            }
            C o;
            o.x = fr * l.x - fi * l.y;
            o.y = fr * l.y + fi * l.x;
            lam[x] = o;
        }
    } else {
        const uint64_t npairs = uint64_t(1) << (KIND == STEP_C1Q ? n - 2 : n - 1);
        const int lo = g.c < g.q ? g.c : g.q, hi = g.c < g.q ? g.q : g.c;
        const int hb = KIND == STEP_STRING ? 63 - __clzll(g.flip) : 0;
        for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < npairs; p += stride) {
            uint64_t x0, x1;
            if constexpr (KIND == STEP_1Q) {
                x0 = insert_zero(p, g.q);
                x1 = x0 | (uint64_t(1) << g.q);
            } else if constexpr (KIND == STEP_C1Q) {
                x0 = insert_two_zeros(p, lo, hi) | (uint64_t(1) << g.c);
                x1 = x0 | (uint64_t(1) << g.q);
            } else {
                x0 = insert_zero(p, hb);
                x1 = x0 ^ g.flip;
            }
            C l0 = lam[x0], l1 = lam[x1];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                if (k >= nphi) break;
                C *ph = (C *)regs.phi[k];
                C f0 = ph[x0], f1 = ph[x1], k0, k1;
                apply_k(f0, f1, x0, x1, k0, k1);
                cmac(sr[k], si[k], l0.x, l0.y, k0.x, k0.y);
                cmac(sr[k], si[k], l1.x, l1.y, k1.x, k1.y);
                if constexpr (KIND == STEP_STRING) {
                    // c + kappa S' on the pair: S' maps x1 -> x0 with sgn(x0), x0 -> x1 with sgn(x1)
                    const double g0 = string_sign(x0, g.zy), g1 = string_sign(x1, g.zy);
                    const C a = f0, b = f1;
                    f0.x = m[0] * a.x + (R)g0 * (m[2] * b.x - m[3] * b.y);
                    f0.y = m[0] * a.y + (R)g0 * (m[2] * b.y + m[3] * b.x);
                    f1.x = m[0] * b.x + (R)g1 * (m[2] * a.x - m[3] * a.y);
                    f1.y = m[0] * b.y + (R)g1 * (m[2] * a.y + m[3] * a.x);
                } else {
                    mat2(m, f0, f1);
                }
                ph[x0] = f0;
                ph[x1] = f1;
            }
            if constexpr (KIND == STEP_STRING) {
                const double g0 = string_sign(x0, g.zy), g1 = string_sign(x1, g.zy);
                const C a = l0, b = l1;
                l0.x = m[0] * a.x + (R)g0 * (m[2] * b.x - m[3] * b.y);
                l0.y = m[0] * a.y + (R)g0 * (m[2] * b.y + m[3] * b.x);
                l1.x = m[0] * b.x + (R)g1 * (m[2] * a.x - m[3] * a.y);
                l1.y = m[0] * b.y + (R)g1 * (m[2] * a.y + m[3] * a.x);
            } else {
                mat2(m, l0, l1);
            }
            lam[x0] = l0;
            lam[x1] = l1;
        }
    }
    if (nphi == 0) return;
    // block sums of every product, one after the other through one LDS array
    __shared__ double sh[2 * kBlock];
    for (int k = 0; k < nphi; ++k) {
        double vr = 0.0, vi = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j == k) { vr = sr[j]; vi = si[j]; }
        __syncthreads();
        sh[threadIdx.x] = vr;
        sh[kBlock + threadIdx.x] = vi;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                sh[threadIdx.x] += sh[threadIdx.x + w];
                sh[kBlock + threadIdx.x] += sh[kBlock + threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            partials[2 * ((size_t)blockIdx.x * M + k)] = sh[0];
            partials[2 * ((size_t)blockIdx.x * M + k) + 1] = sh[kBlock];
        }
    }
}

// dest[k] (complex128 at base + 2 * off[k]) = sum over blocks of partials[block][k]
__global__ void k_reduce_steps(const double *partials, int nb, StepDests d) {
    const int k = blockIdx.x;
    double sr = 0.0, si = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
        sr += partials[2 * ((size_t)b * kStepMaxPhi + k)];
        si += partials[2 * ((size_t)b * kStepMaxPhi + k) + 1];
    }
    block_reduce_store(sr, si, d.base + 2 * d.off[k]);
}

// A fixed gate on lambda and every phi register: CNOT (swap the target pair
// where the control is 1) or CZ (negate where both bits are 1).
template <bool IS_CNOT, typename R>
__global__ void k_fixed_multi(StepRegs regs, int n, int a, int b) {
    using C = typename Cplx<R>::T;
    const uint64_t nq = uint64_t(1) << (n - 2);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < nq; p += (uint64_t)gridDim.x * kBlock) {
        const uint64_t base = insert_two_zeros(p, lo, hi) | (uint64_t(1) << a);
        for (int k = -1; k < regs.n_phi; ++k) {
            C *s = (C *)(k < 0 ? regs.lam : regs.phi[k]);
            if constexpr (IS_CNOT) {
                const uint64_t i1 = base | (uint64_t(1) << b);
                const C u = s[base], v = s[i1];
                s[base] = v;
                s[i1] = u;
            } else {
                const uint64_t i = base | (uint64_t(1) << b);
                C u = s[i];
                u.x = -u.x;
                u.y = -u.y;
                s[i] = u;
            }
        }
    }
}

// The same with two rotations before y_s: psi <- R_b R_a psi (matrices ma on
// qubit qa, then mb on qubit qb), lam = psi, phi = sigma_c psi and the block
// partials of <psi|sigma_c|psi>, for three distinct qubits.  A thread takes
// the 8 amplitudes of one (qa, qb, qc) octet; LA, LB, LC are the positions of
// qa, qb, qc among the three in increasing order (bits of the local index), so
// every register index is a compile-time constant.
template <typename R, int LA, int LB, int LC>
__global__ void k_advance2_seed(typename Cplx<R>::T *psi, typename Cplx<R>::T *lam, typename Cplx<R>::T *phi, int n,
                                int p0, int p1, int p2, const double *__restrict__ ma, const double *__restrict__ mb,
                                int axis, double *partials) {
    using C = typename Cplx<R>::T;
    R a[8], b[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) { a[k] = (R)ma[k]; b[k] = (R)mb[k]; }
    double sr = 0.0, si = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t no = uint64_t(1) << (n - 3);
    const uint64_t bit[3] = {uint64_t(1) << p0, uint64_t(1) << p1, uint64_t(1) << p2};
    for (uint64_t p = blockIdx.x * (uint64_t)kBlock + threadIdx.x; p < no; p += stride) {
        const uint64_t base = insert_zero(insert_zero(insert_zero(p, p0), p1), p2);
        uint64_t off[8];
        C v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            off[k] = base | ((k & 1) ? bit[0] : 0) | ((k & 2) ? bit[1] : 0) | ((k & 4) ? bit[2] : 0);
            v[k] = psi[off[k]];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (!(k & (1 << LA))) mat2(a, v[k], v[k | (1 << LA)]);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (!(k & (1 << LB))) mat2(b, v[k], v[k | (1 << LB)]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            psi[off[k]] = v[k];
            lam[off[k]] = v[k];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k & (1 << LC)) continue;
            const int k1 = k | (1 << LC);
            C o0, o1;
            pauli_pair(axis, v[k], v[k1], o0, o1);
            phi[off[k]] = o0;
            phi[off[k1]] = o1;
            cmac(sr, si, v[k].x, v[k].y, o0.x, o0.y);
            cmac(sr, si, v[k1].x, v[k1].y, o1.x, o1.y);
        }
    }
    block_reduce_store(sr, si, partials + 2 * blockIdx.x);
}

// ------------------------------------------------------------------ Hamiltonian

template <typename R>
__global__ void k_pauli_term(const typename Cplx<R>::T *psi, typename Cplx<R>::T *out, int n, uint64_t flip,
                             uint64_t zy, double fr, double fi, int first) {
    const uint64_t dim = uint64_t(1) << n;
    const R cr = (R)fr, ci = (R)fi;
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        const typename Cplx<R>::T v = psi[x ^ flip];
        const R sgn = (__popcll(x & zy) & 1) ? (R)-1 : (R)1;
        typename Cplx<R>::T o;
        o.x = sgn * (cr * v.x - ci * v.y);
        o.y = sgn * (cr * v.y + ci * v.x);
        if (!first) { const typename Cplx<R>::T w = out[x]; o.x += w.x; o.y += w.y; }
        out[x] = o;
    }
}

// All terms of a chunk in one pass: out[x] = (first ? 0 : out[x]) +
// sum_t c_t (-1)^{popcount(x & zy_t)} psi[x ^ flip_t], summed in the storage
// precision as the one-term kernel does; with partials, the block sums of
// conj(psi[x]) out[x] in FP64.
struct HamChunk {
    HamTerm t[kHamChunk];
    int n_terms, first;
};

template <typename R>
__global__ void k_pauli_sum(const typename Cplx<R>::T *psi, typename Cplx<R>::T *out, int n, HamChunk h,
                            double *partials) {
    using C = typename Cplx<R>::T;
    const uint64_t dim = uint64_t(1) << n;
    double er = 0.0, ei = 0.0;
    for (uint64_t x = blockIdx.x * (uint64_t)kBlock + threadIdx.x; x < dim; x += (uint64_t)gridDim.x * kBlock) {
        C acc;
        if (h.first) { acc.x = (R)0; acc.y = (R)0; }
        else acc = out[x];
        for (int t = 0; t < h.n_terms; ++t) {
            const HamTerm &term = h.t[t];
            const C v = psi[x ^ term.flip];
            const R sgn = (__popcll(x & term.zy) & 1) ? (R)-1 : (R)1;
            const R cr = (R)term.cr, ci = (R)term.ci;
            acc.x += sgn * (cr * v.x - ci * v.y);
            acc.y += sgn * (cr * v.y + ci * v.x);
        }
        out[x] = acc;
        if (partials) {
            const C p = psi[x];
            cmac(er, ei, p.x, p.y, acc.x, acc.y);
        }
    }
    if (partials) block_reduce_store(er, ei, partials + 2 * blockIdx.x);
}

// ------------------------------------------------------------------ unpack

__global__ void k_unpack_metric(const double *Lraw, const double *Traw, const int *param_of, int P, double *G,
                                double *Tout, const int *rot_block, const int *rot_ctrl, int l_only) {
    const int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (idx >= (int64_t)P * P) return;
    const int r = (int)(idx / P), s = (int)(idx % P);
    // T_k = (i/2) <y_k|sigma_k|y_k>
    const double trr = -0.5 * Traw[2 * r + 1], tri = 0.5 * Traw[2 * r];
    const double tsr = -0.5 * Traw[2 * s + 1], tsi = 0.5 * Traw[2 * s];
    double lr, li;
    if (r < s)      { lr = 0.25 * Lraw[2 * ((int64_t)r * P + s)]; li = 0.25 * Lraw[2 * ((int64_t)r * P + s) + 1]; }
    else if (r > s) { lr = 0.25 * Lraw[2 * ((int64_t)s * P + r)]; li = -0.25 * Lraw[2 * ((int64_t)s * P + r) + 1]; }
    else            { lr = (rot_ctrl && rot_ctrl[s] >= 0) ? 0.25 * Lraw[2 * ((int64_t)s * P + s)] : 0.25; li = 0.0; }
    // G = L - conj(T_r) T_s (or L alone); zero between different blocks
    double pr = trr * tsr + tri * tsi, pi = trr * tsi - tri * tsr;
    if (l_only) pr = pi = 0.0;
    const int pr_ = param_of ? param_of[r] : r, ps_ = param_of ? param_of[s] : s;
    const int64_t o = (int64_t)pr_ * P + ps_;
    const bool off_block = rot_block && rot_block[r] != rot_block[s];
    G[2 * o] = off_block ? 0.0 : lr - pr;
    G[2 * o + 1] = off_block ? 0.0 : li - pi;
    if (Tout && r == s) { Tout[2 * pr_] = trr; Tout[2 * pr_ + 1] = tri; }
}

__global__ void k_grad_from_raw(const double *graw, const int *param_of, int P, double *grad) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r < P) grad[param_of[r]] = -graw[2 * r + 1];
}

// Shared parameters: G'[a][b] = sum over rotations r of a and s of b of
// G[r][s], T'[a] = sum over r of a of T[r] (the rotations of parameter a are
// rot[off[a] .. off[a+1]); G, T in rotation order, P rotations).
__global__ void k_contract_metric(const double *G, const double *T, int P, const int *off, const int *rot, int NP,
                                  double *Gp, double *Tp) {
    const int64_t idx = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (idx >= (int64_t)NP * NP) return;
    const int a = (int)(idx / NP), b = (int)(idx % NP);
    double gr = 0.0, gi = 0.0;
    for (int i = off[a]; i < off[a + 1]; ++i)
        for (int j = off[b]; j < off[b + 1]; ++j) {
            const int64_t o = (int64_t)rot[i] * P + rot[j];
            gr += G[2 * o];
            gi += G[2 * o + 1];
        }
    Gp[2 * idx] = gr;
    Gp[2 * idx + 1] = gi;
    if (Tp && b == 0) {
        double tr = 0.0, ti = 0.0;
        for (int i = off[a]; i < off[a + 1]; ++i) {
            tr += T[2 * rot[i]];
            ti += T[2 * rot[i] + 1];
        }
        Tp[2 * a] = tr;
        Tp[2 * a + 1] = ti;
    }
}

__global__ void k_grad_contract(const double *graw, const int *off, const int *rot, int NP, double *grad) {
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= NP) return;
    double g = 0.0;
    for (int i = off[a]; i < off[a + 1]; ++i) g -= graw[2 * rot[i] + 1];
    grad[a] = g;
}

}  // namespace

// ====================================================================== launchers

int reduce_blocks(int n) {
    const int64_t work = (int64_t(1) << n) / (kBlock * 8);
    if (work < 1) return 1;
    return work > kReduceBlocksMax ? kReduceBlocksMax : (int)work;
}

template <typename R> void launch_init_state(void *dst, int n, const void *src, hipStream_t st) {
    const uint64_t dim = uint64_t(1) << n;
    hipLaunchKernelGGL(k_init_state<R>, dim3(grid_for(dim)), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)dst, dim, (const double2 *)src);
    check_launch();
}

template <typename R> void launch_to_c128(const void *src, void *dst, int n, hipStream_t st) {
    const uint64_t dim = uint64_t(1) << n;
    hipLaunchKernelGGL(k_to_c128<R>, dim3(grid_for(dim)), dim3(kBlock), 0, st,
                       (const typename Cplx<R>::T *)src, (double2 *)dst, dim);
    check_launch();
}

template <typename R> void launch_copy(const void *src, void *dst, int n, hipStream_t st) {
    const uint64_t dim = uint64_t(1) << n;
    hipLaunchKernelGGL(k_copy<R>, dim3(grid_for(dim)), dim3(kBlock), 0, st,
                       (const typename Cplx<R>::T *)src, (typename Cplx<R>::T *)dst, dim);
    check_launch();
}

template <typename R> void launch_apply_1q(void *s0, void *s1, int n, int q, const DevMat2 &m, hipStream_t st) {
    hipLaunchKernelGGL((q >= kNtMinQubit ? k_apply_1q<R, true> : k_apply_1q<R, false>),
                       dim3(grid_for(uint64_t(1) << (n - 1))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, q, m);
    check_launch();
}

template <typename R> void launch_apply_1q_tab(void *s0, void *s1, int n, int q, const double *m_dev, hipStream_t st) {
    hipLaunchKernelGGL((q >= kNtMinQubit ? k_apply_1q_tab<R, true> : k_apply_1q_tab<R, false>),
                       dim3(grid_for(uint64_t(1) << (n - 1))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, q, m_dev);
    check_launch();
}

template <typename R>
void launch_apply_c1q(void *s0, void *s1, int n, int c, int q, const DevMat2 &m, hipStream_t st) {
    hipLaunchKernelGGL(k_apply_c1q<R>, dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, c, q, m);
    check_launch();
}

template <typename R>
void launch_apply_c1q_tab(void *s0, void *s1, int n, int c, int q, const double *m_dev, hipStream_t st) {
    hipLaunchKernelGGL(k_apply_c1q_tab<R>, dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, c, q, m_dev);
    check_launch();
}

// w = (-i)^{n_y}
inline void string_phase(int n_y, double &wr, double &wi) {
    wr = 1.0;
    wi = 0.0;
    for (int k = 0; k < (n_y & 3); ++k) { const double t = wr; wr = wi; wi = -t; }
}

template <typename R>
void launch_apply_string(void *s0, void *s1, int n, uint64_t flip, uint64_t zy, int n_y, double c, double sr,
                         double si, hipStream_t st) {
    // kappa = (sr + i si) w
    double wr, wi;
    string_phase(n_y, wr, wi);
    const double kr = sr * wr - si * wi, ki = sr * wi + si * wr;
    const uint64_t work = flip ? uint64_t(1) << (n - 1) : uint64_t(1) << n;
    hipLaunchKernelGGL(k_apply_string<R>, dim3(grid_for(work)), dim3(kBlock), 0, st, (typename Cplx<R>::T *)s0,
                       (typename Cplx<R>::T *)s1, n, flip, zy, c, kr, ki);
    check_launch();
}

template <typename R>
void launch_seed_string(const void *y, void *lam, void *phi, int n, uint64_t flip, uint64_t zy, int n_y,
                        hipStream_t st) {
    double wr, wi;
    string_phase(n_y, wr, wi);
    hipLaunchKernelGGL(k_seed_string<R>, dim3(grid_for(uint64_t(1) << n)), dim3(kBlock), 0, st,
                       (const typename Cplx<R>::T *)y, (typename Cplx<R>::T *)lam, (typename Cplx<R>::T *)phi, n, flip,
                       zy, wr, wi);
    check_launch();
}

template <typename R>
void launch_string_prod(const void *a, const void *b, int n, uint64_t flip, uint64_t zy, int n_y, double *partials,
                        double *dest, hipStream_t st) {
    double wr, wi;
    string_phase(n_y, wr, wi);
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_string_prod_partial<R>, dim3(nb), dim3(kBlock), 0, st, (const typename Cplx<R>::T *)a,
                       (const typename Cplx<R>::T *)b, n, flip, zy, wr, wi, partials);
    check_launch();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, (const double *)partials, nb, dest);
    check_launch();
}

template <typename R>
void launch_sweep_step(const StepRegs &regs, const StepGate &g, double *partials, const StepDests *dests,
                       hipStream_t st) {
    if (regs.n_phi < 0 || regs.n_phi > kStepMaxPhi) throw hipErrorInvalidValue;
    const int nb = reduce_blocks(g.n);
    switch (g.kind) {
    case STEP_1Q:
        hipLaunchKernelGGL((k_sweep_step<STEP_1Q, R>), dim3(nb), dim3(kBlock), 0, st, regs, g, partials);
        break;
    case STEP_C1Q:
        hipLaunchKernelGGL((k_sweep_step<STEP_C1Q, R>), dim3(nb), dim3(kBlock), 0, st, regs, g, partials);
        break;
    case STEP_STRING:
        hipLaunchKernelGGL((k_sweep_step<STEP_STRING, R>), dim3(nb), dim3(kBlock), 0, st, regs, g, partials);
        break;
    default: throw hipErrorInvalidValue;
    }
    check_launch();
    if (regs.n_phi > 0 && dests) {
        hipLaunchKernelGGL(k_reduce_steps, dim3(regs.n_phi), dim3(kBlock), 0, st, (const double *)partials, nb, *dests);
        check_launch();
    }
}

template <typename R> void launch_fixed_multi(const StepRegs &regs, int n, bool cnot, int a, int b, hipStream_t st) {
    if (regs.n_phi < 0 || regs.n_phi > kStepMaxPhi) throw hipErrorInvalidValue;
    if (cnot)
        hipLaunchKernelGGL((k_fixed_multi<true, R>), dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st, regs,
                           n, a, b);
    else
        hipLaunchKernelGGL((k_fixed_multi<false, R>), dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st, regs,
                           n, a, b);
    check_launch();
}

template <typename R>
void launch_cnot_run(const void *src, void *dst, int n, const int *control, const int *target, int count,
                     hipStream_t st) {
    if (count < 0 || count > kCnotRunMax) throw hipErrorInvalidValue;
    CnotRun run;
    run.count = count;
    for (int k = 0; k < count; ++k) {
        if (control[k] < 0 || control[k] >= n || target[k] < 0 || target[k] >= n) throw hipErrorInvalidValue;
        run.c[k] = (uint8_t)control[k];
        run.t[k] = (uint8_t)target[k];
    }
    const uint64_t dim = uint64_t(1) << n;
    hipLaunchKernelGGL(k_cnot_run<R>, dim3(grid_for(dim)), dim3(kBlock), 0, st, (const typename Cplx<R>::T *)src,
                       (typename Cplx<R>::T *)dst, n, run);
    check_launch();
}

template <typename R> void launch_cnot(void *s0, void *s1, int n, int c, int t, hipStream_t st) {
    hipLaunchKernelGGL((k_cnot<R, false>),
                       dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, c, t);
    check_launch();
}

template <typename R> void launch_cz(void *s0, void *s1, int n, int a, int b, hipStream_t st) {
    hipLaunchKernelGGL((k_cz<R, false>),
                       dim3(grid_for(uint64_t(1) << (n - 2))), dim3(kBlock), 0, st,
                       (typename Cplx<R>::T *)s0, (typename Cplx<R>::T *)s1, n, a, b);
    check_launch();
}

template <typename R>
void launch_seed(const void *y, void *lam, void *phi, int n, int q, int axis, hipStream_t st, int ctrl) {
    hipLaunchKernelGGL(k_seed<R>, dim3(grid_for(uint64_t(1) << (n - 1))), dim3(kBlock), 0, st,
                       (const typename Cplx<R>::T *)y, (typename Cplx<R>::T *)lam, (typename Cplx<R>::T *)phi, n, q,
                       axis, ctrl);
    check_launch();
}

template <typename R>
void launch_pauli_prod(const void *a, const void *b, int n, int q, int axis, double *partials, double *dest,
                       hipStream_t st, int ctrl) {
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_pauli_prod_partial<R>, dim3(nb), dim3(kBlock), 0, st, (const typename Cplx<R>::T *)a,
                       (const typename Cplx<R>::T *)b, n, q, axis, ctrl, partials);
    check_launch();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, (const double *)partials, nb, dest);
    check_launch();
}

template <typename R>
void launch_advance_seed(void *psi, void *lam, void *phi, int n, int qr, const double *m_dev, int qs, int axis,
                         double *partials, double *dest, hipStream_t st) {
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_advance_seed<R>, dim3(nb), dim3(kBlock), 0, st, (typename Cplx<R>::T *)psi,
                       (typename Cplx<R>::T *)lam, (typename Cplx<R>::T *)phi, n, qr, m_dev, qs, axis, partials);
    check_launch();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, (const double *)partials, nb, dest);
    check_launch();
}

template <typename R>
void launch_seed_multi(const SeedItem *items, int n_items, uint32_t total_blocks, double *partials, hipStream_t st) {
    if (n_items <= 0 || total_blocks == 0) return;
    hipLaunchKernelGGL(k_seed_multi<R>, dim3(total_blocks), dim3(kBlock), 0, st, items, n_items, partials);
    check_launch();
}

template <typename R>
void launch_advance2_seed(void *psi, void *lam, void *phi, int n, int qa, const double *ma, int qb, const double *mb,
                          int qc, int axis, double *partials, double *dest, hipStream_t st) {
    if (n < 3 || qa == qb || qa == qc || qb == qc) throw hipErrorInvalidValue;
    int q[3] = {qa, qb, qc};
    int s[3] = {qa, qb, qc};
    if (s[0] > s[1]) std::swap(s[0], s[1]);
    if (s[1] > s[2]) std::swap(s[1], s[2]);
    if (s[0] > s[1]) std::swap(s[0], s[1]);
    int l[3];
    for (int k = 0; k < 3; ++k) l[k] = q[k] == s[0] ? 0 : q[k] == s[1] ? 1 : 2;
    const int nb = reduce_blocks(n);
    using C = typename Cplx<R>::T;
    const int code = l[0] * 9 + l[1] * 3 + l[2];
#define QNG_ADV2(LA, LB, LC)                                                                                       \
    case LA * 9 + LB * 3 + LC:                                                                                     \
        hipLaunchKernelGGL((k_advance2_seed<R, LA, LB, LC>), dim3(nb), dim3(kBlock), 0, st, (C *)psi, (C *)lam,     \
                           (C *)phi, n, s[0], s[1], s[2], ma, mb, axis, partials);                                  \
        break;
    switch (code) {
        QNG_ADV2(0, 1, 2)
        QNG_ADV2(0, 2, 1)
        QNG_ADV2(1, 0, 2)
        QNG_ADV2(1, 2, 0)
        QNG_ADV2(2, 0, 1)
        QNG_ADV2(2, 1, 0)
    default: throw hipErrorInvalidValue;
    }
#undef QNG_ADV2
    check_launch();
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, (const double *)partials, nb, dest);
    check_launch();
}

template <typename R>
void launch_pauli_sum(const void *psi, void *out, int n, const HamTerm *terms, int n_terms, double *partials,
                      double *dest, hipStream_t st) {
    const int nb = reduce_blocks(n);
    for (int t0 = 0; t0 < n_terms || t0 == 0; t0 += kHamChunk) {
        HamChunk h;
        h.n_terms = n_terms - t0 < kHamChunk ? n_terms - t0 : kHamChunk;
        h.first = t0 == 0;
        for (int k = 0; k < h.n_terms; ++k) h.t[k] = terms[t0 + k];
        const bool last = t0 + kHamChunk >= n_terms;
        hipLaunchKernelGGL(k_pauli_sum<R>, dim3(nb), dim3(kBlock), 0, st, (const typename Cplx<R>::T *)psi,
                           (typename Cplx<R>::T *)out, n, h, (last && dest) ? partials : nullptr);
        check_launch();
        if (n_terms == 0) break;
    }
    if (dest) {
        hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, st, (const double *)partials, nb, dest);
        check_launch();
    }
}

template <typename R>
void launch_pauli_term(const void *psi, void *out, int n, uint64_t flip, uint64_t zy, int n_y, double coeff, int first,
                       hipStream_t st) {
    // coeff * (-i)^{n_y}
    double fr = coeff, fi = 0.0;
    for (int k = 0; k < (n_y & 3); ++k) { const double t = fr; fr = fi; fi = -t; }
    const uint64_t dim = uint64_t(1) << n;
    hipLaunchKernelGGL(k_pauli_term<R>, dim3(grid_for(dim)), dim3(kBlock), 0, st, (const typename Cplx<R>::T *)psi,
                       (typename Cplx<R>::T *)out, n, flip, zy, fr, fi, first);
    check_launch();
}

void launch_unpack_metric(const double *Lraw, const double *Traw, const int *param_of, int P, double *G_out,
                          double *T_out, const int *rot_block, const int *rot_ctrl, bool l_only, hipStream_t st) {
    const int64_t work = (int64_t)P * P;
    if (work == 0) return;
    hipLaunchKernelGGL(k_unpack_metric, dim3((unsigned)((work + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, Lraw,
                       Traw, param_of, P, G_out, T_out, rot_block, rot_ctrl, l_only ? 1 : 0);
    check_launch();
}

void launch_contract_metric(const double *G, const double *T, int P, const int *off, const int *rot, int NP,
                            double *Gp, double *Tp, hipStream_t st) {
    const int64_t work = (int64_t)NP * NP;
    if (work == 0) return;
    hipLaunchKernelGGL(k_contract_metric, dim3((unsigned)((work + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, G, T,
                       P, off, rot, NP, Gp, Tp);
    check_launch();
}

void launch_grad_contract(const double *graw, const int *off, const int *rot, int NP, double *grad, hipStream_t st) {
    if (NP == 0) return;
    hipLaunchKernelGGL(k_grad_contract, dim3((unsigned)((NP + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, graw, off,
                       rot, NP, grad);
    check_launch();
}

void launch_grad_from_raw(const double *graw, const int *param_of, int P, double *grad, hipStream_t st) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_grad_from_raw, dim3((P + kBlock - 1) / kBlock), dim3(kBlock), 0, st, graw, param_of, P, grad);
    check_launch();
}

#define QNG_INSTANTIATE(R)                                                                                        \
    template void launch_init_state<R>(void *, int, const void *, hipStream_t);                                  \
    template void launch_to_c128<R>(const void *, void *, int, hipStream_t);                                      \
    template void launch_copy<R>(const void *, void *, int, hipStream_t);                                         \
    template void launch_apply_1q<R>(void *, void *, int, int, const DevMat2 &, hipStream_t);                     \
    template void launch_apply_1q_tab<R>(void *, void *, int, int, const double *, hipStream_t);                  \
    template void launch_apply_c1q<R>(void *, void *, int, int, int, const DevMat2 &, hipStream_t);               \
    template void launch_apply_c1q_tab<R>(void *, void *, int, int, int, const double *, hipStream_t);            \
    template void launch_apply_string<R>(void *, void *, int, uint64_t, uint64_t, int, double, double, double,      \
                                         hipStream_t);                                                            \
    template void launch_seed_string<R>(const void *, void *, void *, int, uint64_t, uint64_t, int, hipStream_t);  \
    template void launch_string_prod<R>(const void *, const void *, int, uint64_t, uint64_t, int, double *,        \
                                        double *, hipStream_t);                                                   \
    template void launch_sweep_step<R>(const StepRegs &, const StepGate &, double *, const StepDests *,           \
                                       hipStream_t);                                                              \
    template void launch_fixed_multi<R>(const StepRegs &, int, bool, int, int, hipStream_t);                      \
    template void launch_cnot<R>(void *, void *, int, int, int, hipStream_t);                                     \
    template void launch_cnot_run<R>(const void *, void *, int, const int *, const int *, int, hipStream_t);       \
    template void launch_cz<R>(void *, void *, int, int, int, hipStream_t);                                       \
    template void launch_seed<R>(const void *, void *, void *, int, int, int, hipStream_t, int);                 \
    template void launch_pauli_prod<R>(const void *, const void *, int, int, int, double *, double *, hipStream_t, \
                                       int);                                                                      \
    template void launch_advance_seed<R>(void *, void *, void *, int, int, const double *, int, int, double *,       \
                                         double *, hipStream_t);                                                  \
    template void launch_seed_multi<R>(const SeedItem *, int, uint32_t, double *, hipStream_t);                      \
    template void launch_pauli_term<R>(const void *, void *, int, uint64_t, uint64_t, int, double, int, hipStream_t); \
    template void launch_pauli_sum<R>(const void *, void *, int, const HamTerm *, int, double *, double *, hipStream_t); \
    template void launch_advance2_seed<R>(void *, void *, void *, int, int, const double *, int, const double *, int, \
                                          int, double *, double *, hipStream_t);

QNG_INSTANTIATE(double)
QNG_INSTANTIATE(float)

}  // namespace qng
