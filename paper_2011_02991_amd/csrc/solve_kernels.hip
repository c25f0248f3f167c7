// solve_kernels.hip -- the natural-gradient step's shifted solve on the device.
//
// The step of Sec. 1 is g dtheta = -dt grad E with g = Re G, solved with a
// Tikhonov shift: (Re G + eps I) dtheta = -dt grad E.  The device entry point
// of the step keeps G and grad E on the device, so the solve runs there too:
// one work-group factors the shifted matrix by Cholesky (right-looking, in
// FP64, in a workspace copy of the lower triangle), then does the forward and
// backward substitutions.  P is a few hundred, so the O(P^3 / 3) factorisation
// is a few million multiply-adds: latency, not throughput, sets its time, and
// one work-group with a barrier per column is enough.
//
// A non-positive or non-finite pivot stops the factorisation and sets the
// status word to QNG_E_NOT_SPD; the solution is written only when it is
// QNG_OK, and k_copy_if_ok lets every other output follow the same rule.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "solve_kernels.hpp"

namespace qng {

namespace {

constexpr int kSolveThreads = 1024;

// G: P x P complex row-major (Re G used); grad: P; A: P x P scratch (lower
// triangle used); y: P scratch; x: P output; status: one int32.
__global__ __launch_bounds__(kSolveThreads) void k_shifted_solve(const double *__restrict__ G, int P, double eps,
                                                                 const double *__restrict__ grad, double dt,
                                                                 double *__restrict__ A, double *__restrict__ y,
                                                                 double *__restrict__ x, int32_t *status) {
    const int tid = threadIdx.x;
    __shared__ int bad;
    __shared__ double piv;
    for (int64_t idx = tid; idx < (int64_t)P * P; idx += kSolveThreads) {
        const int i = (int)(idx / P), j = (int)(idx % P);
        if (j <= i) A[idx] = G[2 * idx] + (i == j ? eps : 0.0);
    }
    for (int i = tid; i < P; i += kSolveThreads) y[i] = -dt * grad[i];
    if (tid == 0) bad = 0;
    __syncthreads();
    // A = L L^T, L overwriting the lower triangle column by column
    for (int k = 0; k < P; ++k) {
        if (tid == 0) {
            const double d = A[(int64_t)k * P + k];
            bad = !(d > 0.0) || !isfinite(d);
            piv = bad ? 1.0 : sqrt(d);
            A[(int64_t)k * P + k] = piv;
        }
        __syncthreads();
        if (bad) break;
        for (int i = k + 1 + tid; i < P; i += kSolveThreads) A[(int64_t)i * P + k] /= piv;
        __syncthreads();
        // trailing lower triangle: rows and columns k+1 .. P-1
        const int m = P - 1 - k;
        for (int64_t t = tid; t < (int64_t)m * m; t += kSolveThreads) {
            const int i = k + 1 + (int)(t / m), j = k + 1 + (int)(t % m);
            if (j <= i) A[(int64_t)i * P + j] -= A[(int64_t)i * P + k] * A[(int64_t)j * P + k];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) *status = -7;   // QNG_E_NOT_SPD
        return;
    }
    // L z = b (z in y), column by column
    for (int k = 0; k < P; ++k) {
        if (tid == 0) y[k] /= A[(int64_t)k * P + k];
        __syncthreads();
        const double zk = y[k];
        for (int i = k + 1 + tid; i < P; i += kSolveThreads) y[i] -= A[(int64_t)i * P + k] * zk;
        __syncthreads();
    }
    // L^T x = z, from the last unknown up (row k of L is column k of L^T)
    for (int k = P - 1; k >= 0; --k) {
        if (tid == 0) y[k] /= A[(int64_t)k * P + k];
        __syncthreads();
        const double xk = y[k];
        for (int i = tid; i < k; i += kSolveThreads) y[i] -= A[(int64_t)k * P + i] * xk;
        __syncthreads();
    }
    for (int i = tid; i < P; i += kSolveThreads) x[i] = y[i];
    if (tid == 0) *status = 0;
}

__global__ void k_copy_if_ok(const int32_t *status, const double *__restrict__ src, double *__restrict__ dst,
                             int64_t count) {
    if (*status != 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

inline void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw e;
}

}  // namespace

void launch_shifted_solve(const double *G, int P, double eps, const double *grad, double dt, double *A, double *y,
                          double *x, int32_t *status, hipStream_t st) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_shifted_solve, dim3(1), dim3(kSolveThreads), 0, st, G, P, eps, grad, dt, A, y, x, status);
    check_launch();
}

void launch_copy_if_ok(const int32_t *status, const double *src, double *dst, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_copy_if_ok, dim3((unsigned)blocks), dim3(256), 0, st, status, src, dst, count);
    check_launch();
}

}  // namespace qng
