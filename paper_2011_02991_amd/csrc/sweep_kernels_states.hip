// sweep_kernels_states.hip -- the sweep-pass kernels without inner products:
// the passes carry lambda and the phi registers of a column block through the
// adjoint gates and the in-pass seeds only, so that each phi register ends as
// an explicit derivative state (the derivative-state variant of the metric,
// whose inner products are then one Gram matrix).  The same source as
// sweep_kernels.hip, built with QNG_NO_PRODUCTS = 1.  Exports
// launch_sweep_pass_states.
#define QNG_NO_PRODUCTS 1
#include "sweep_kernels.hip"
