// sweep_kernels_real_exact.hip -- the sweep-pass kernels for complex64 storage
// in FP32 registers with every inner-product term formed and accumulated in
// FP64, keeping the real parts of the metric's inner products only (the
// natural-gradient step solves with Re G): the same source as
// sweep_kernels.hip, built with both switches.  Exports
// launch_sweep_pass_real_exact.
#define QNG_REAL_PRODUCTS 1
#define QNG_EXACT_PRODUCTS 1
#include "sweep_kernels.hip"
