// sweep_kernels_real.hip -- the sweep-pass kernels with the metric's inner
// products reduced to their real parts (the natural-gradient step solves with
// Re G only): the same source as sweep_kernels.hip, built with
// QNG_REAL_PRODUCTS = 1.  Exports launch_sweep_pass_real.
#define QNG_REAL_PRODUCTS 1
#include "sweep_kernels.hip"
