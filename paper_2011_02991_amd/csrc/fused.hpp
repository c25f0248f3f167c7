// fused.hpp -- host executor of the fused, tiled metric (see sweep.hpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <vector>

#include "circuit.hpp"
#include "kernels.hpp"
#include "sweep.hpp"

namespace qng {

struct FusedBuffers {
    char *states = nullptr;        // state 0 = psi; column b of a group uses states 1+2b (lambda), 2+2b (phi)
    size_t state_bytes = 0;
    char *scratch = nullptr;       // matrix table, plan images, launch items, reduce tasks, partial sums
    size_t scratch_bytes = 0;
    double *traw = nullptr;        // P complex: <y_s|sigma_s|y_s>
    double *lraw = nullptr;        // P*P complex: <lambda|sigma_r|phi> at (r, s)
    double *reduce_partials = nullptr;  // scratch of the per-primitive reductions
    // Derivative-state variant (xi != nullptr): P + 1 states at xi, one after
    // another -- the forward state lambda* in the sweeps' final frame, then the
    // swept phi register of every column s (its derivative state, up to the
    // factor i/2 and a unitary common to all columns) -- the passes take no
    // inner product, and L and T come from the Gram matrix of those states
    // (gram_partials: gram_partial_bytes of scratch).  dummy: one state for
    // the unused phi register of the lowest block.
    char *xi = nullptr;
    char *dummy = nullptr;
    double *gram_partials = nullptr;
};

size_t fused_scratch_bytes(const SweepPlan &plan, const FusedRun &fr, int M);

// Runs T for every rotation and L_rs for every r < s.  psi (state 0) must hold
// |in> on entry; on return it holds y_{P-1} and the gate position of the last
// rotation is returned.
// real_products: the inner products of L keep their real parts only (what a
// natural-gradient step needs); T stays complex.
template <typename R>
int run_fused_metric(const SweepPlan &plan, const FusedRun &fr, const Circuit &c, const std::vector<Mat2> &fwd,
                     const std::vector<Mat2> &adj, const FusedBuffers &buf, hipStream_t st, qng_stats *stats,
                     bool profile, int reg_mode, bool real_products = false);

size_t fused_gradient_scratch_bytes(const SweepPlan &g, int M);

// Reverse sweep of the energy gradient through the fused passes of the
// gradient plan g (build_gradient_plan): lam holds H psi and psi the final
// state on entry (both are swept back in place); <lam|sigma_r|psi> of every
// rotation r is written to graw[r] (complex).
template <typename R>
void run_fused_gradient(const SweepPlan &g, const Circuit &c, const std::vector<Mat2> &adj, void *lam, void *psi,
                        double *graw, char *scratch, size_t scratch_bytes, hipStream_t st, qng_stats *stats,
                        bool profile, int reg_mode);

}  // namespace qng
