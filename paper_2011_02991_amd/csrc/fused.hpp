// fused.hpp -- host executor of the fused, tiled metric (see sweep.hpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <functional>
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
    // Derivative-state variant (xi != nullptr): the forward state lambda* in
    // the sweeps' final frame and column 0's derivative state at xi, one after
    // the other, and the swept phi register of every column s >= 1 (its
    // derivative state, up to the factor i/2 and a unitary common to all
    // columns) at xi_chunk + (s - chunk_col0) states (xi_chunk nullptr: xi + 2
    // states, chunk_col0 = 1); the passes take no inner product, and L and T
    // come from the Gram matrix of those states (run_states_metric;
    // gram_partials: the Gram kernel's partial sums, gram_signs: P + 1 bytes).
    // dummy: one state for the unused phi registers of the lowest block.
    // blk_begin .. blk_end - 1: the column blocks run (blk_end < 0: all).
    char *xi = nullptr;
    char *dummy = nullptr;
    double *gram_partials = nullptr;
    int8_t *gram_signs = nullptr;
    char *xi_chunk = nullptr;
    int chunk_col0 = 1;
    int blk_begin = 0, blk_end = -1;
};

// Column blocks of the derivative-state variant taken a chunk at a time: whole
// blocks of the plan, in its order, columns col_lo .. col_hi (column 0 is kept
// apart with lambda*).
struct StateChunk {
    int blk_begin, blk_end, col_lo, col_hi;
};
// Chunks of at most max_cols columns each (QNG_E_OUT_OF_MEMORY when a block
// alone has more).
std::vector<StateChunk> state_chunks(const SweepPlan &plan, int max_cols);
// Kept states of the derivative-state variant with chunks of at most max_cols
// columns: the dummy, lambda*, column 0 and one chunk (all P - 1 columns) or
// two chunks.
size_t kept_states(int P, int max_cols);
// Bytes of the Gram kernel's partial sums and the signs for those chunks.
size_t states_gram_bytes(int n, int P, int max_cols);

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

// The derivative-state variant (buf.xi != nullptr) in chunks of at most
// max_cols columns: the derivative states of one chunk are prepared at a time
// (the forward state restarted from |in> by `restart` for every chunk after the
// first) and the Gram matrix is taken chunk by chunk, so that two chunks are
// kept at once; one chunk when every column fits.  Returns as
// run_fused_metric does.
template <typename R>
int run_states_metric(const SweepPlan &plan, const FusedRun &fr, const Circuit &c, const std::vector<Mat2> &fwd,
                      const std::vector<Mat2> &adj, const FusedBuffers &buf, int max_cols,
                      const std::function<void()> &restart, hipStream_t st, qng_stats *stats, bool profile,
                      bool real_products);

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
