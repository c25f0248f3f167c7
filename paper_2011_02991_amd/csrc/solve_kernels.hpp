// solve_kernels.hpp -- device launchers of the step's shifted solve (Sec. 1:
// (Re G + eps I) dtheta = -dt grad E).  All pointers are device pointers;
// launches are asynchronous on `st`.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace qng {

// x solves (Re G + eps I) x = -dt grad by Cholesky in FP64 (one work-group).
// G: P x P complex row-major; grad, x: P doubles; A: P*P doubles and y: P
// doubles of scratch.  *status <- 0, or QNG_E_NOT_SPD (-7) with x untouched.
void launch_shifted_solve(const double *G, int P, double eps, const double *grad, double dt, double *A, double *y,
                          double *x, int32_t *status, hipStream_t st);

// dst[0 .. count) <- src[0 .. count) if *status == 0, else nothing.
void launch_copy_if_ok(const int32_t *status, const double *src, double *dst, int64_t count, hipStream_t st);

}  // namespace qng
