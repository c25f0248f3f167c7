// sweep_kernels_exact.hip -- the sweep-pass kernels for complex64 storage in
// FP32 registers with every inner-product term formed and accumulated in FP64
// (QNG_OPT_EXACT_PRODUCTS): the same source as sweep_kernels.hip, built with
// the product precision switched to FP64.  Exports launch_sweep_pass_exact.
#define QNG_EXACT_PRODUCTS 1
#include "sweep_kernels.hip"
