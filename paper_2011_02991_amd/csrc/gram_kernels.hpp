// gram_kernels.hpp -- Gram matrix of the explicit derivative states on the
// matrix cores (see gram_kernels.hip).  Device pointers; asynchronous on `st`.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace qng {

// Bytes of the partial-sum buffer launch_gram needs for Q states of n qubits.
size_t gram_partial_bytes(int n, int Q);

// X: Q states of 2^n complex amplitudes one after another (complex64 or
// complex128), X_0 the forward state lambda* and X_{1+s} the derivative state
// of column s, all in one frame, each up to the sign sign[q] (+-1, device).
// mode 0 writes Re and mode 1 Im of sign[a] sign[b] <X_a|X_b> for a < b: a = 0
// into traw[b-1] (complex, that part only), a >= 1 into lraw[(a-1)*P + (b-1)]
// (complex, that part only).
void launch_gram(const void *X, bool complex64, int n, int Q, int P, int mode, const int8_t *sign, double *partials,
                 double *lraw, double *traw, hipStream_t st);

// Multiply-add flops (2 per term) of one launch_gram mode, tiles included.
double gram_flops(int n, int Q);

}  // namespace qng
