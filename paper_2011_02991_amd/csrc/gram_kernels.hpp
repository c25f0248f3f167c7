// gram_kernels.hpp -- Gram matrix of the explicit derivative states on the
// matrix cores (see gram_kernels.hip).  Device pointers; asynchronous on `st`.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace qng {

// One operand of launch_gram: positions 0 .. n1-1 are the states at p1 (one
// after another, 2^n complex amplitudes each), positions n1 .. n-1 those at
// p2; position q holds the state of column col1 + q (q < n1) or of column
// col2 + q - n1, where column -1 stands for the forward state lambda*.
struct GramSet {
    const void *p1 = nullptr, *p2 = nullptr;
    int n1 = 0, n = 0;
    int col1 = 0, col2 = 0;
};

// Bytes of the partial-sum buffer launch_gram needs for QA x QB states of n
// qubits (QB = 0: the symmetric product of QA states).
size_t gram_partial_bytes(int n, int QA, int QB);

// The inner products of kept states (complex64 or complex128, each up to the
// sign sign[column + 1] = +-1, device).  B == nullptr: every pair of positions
// a < b of A, whose columns ascend with the position; else every pair of a
// position of A and one of B, every column of B above every column of A.  For
// each pair, columns ca < cb, mode 0 writes Re and mode 1 Im of sign[ca + 1]
// sign[cb + 1] <X_a|X_b>: ca = -1 into traw[cb] (complex, that part only),
// else into lraw[ca * P + cb] (complex, that part only).
void launch_gram(const GramSet &A, const GramSet *B, bool complex64, int n, int P, int mode, const int8_t *sign,
                 double *partials, double *lraw, double *traw, hipStream_t st);

// Multiply-add flops (2 per term) of one launch_gram mode, tiles included.
double gram_flops(int n, int QA, int QB);

}  // namespace qng
