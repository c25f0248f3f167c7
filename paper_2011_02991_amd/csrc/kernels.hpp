// kernels.hpp -- host-side launchers of the per-primitive HIP kernels.
//
// The paper builds everything from three primitives on 2^n-amplitude state
// vectors: clone a state, apply a gate, take an inner product (abstract;
// appendix introduction).  These launchers are those primitives (plus the
// Pauli-sum Hamiltonian) as one kernel each, on interleaved complex states of
// element type R (double: complex128, float: complex64).  Inner products are
// always accumulated in FP64 through a deterministic two-stage reduction.
//
// All pointers are device pointers; every launch is asynchronous on `st`.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace qng {

struct DevMat2 {   // 2x2 complex matrix, FP64, row-major
    double ar, ai, br, bi, cr, ci, dr, di;
};

// Number of first-stage blocks used by the reductions for a register of n qubits.
int reduce_blocks(int n);

// One step of the back sweep over lambda and up to kStepMaxPhi phi registers
// (the columns of a block share lambda): launch_sweep_step takes
// <lambda|K|phi_k> for every phi register, K the generator of the step's
// rotation, then applies the rotation's adjoint to lambda and every phi.
constexpr int kStepMaxPhi = 8;
enum StepKind : int { STEP_1Q = 0, STEP_C1Q = 1, STEP_STRING = 2 };
struct StepRegs {
    void *lam;
    void *phi[kStepMaxPhi];
    int n_phi;
};
struct StepGate {
    int kind, n;
    int q, c, axis;          // STEP_1Q: target q, generator axis; STEP_C1Q: also control c
    uint64_t flip, zy;       // STEP_STRING: the string in mask form (w = wr + i wi = (-i)^{n_y})
    double wr, wi;
    double m[8];             // the adjoint: 2x2 matrix (row-major, re/im), or for a string
                             // m[0] = c and (m[2], m[3]) = kappa of c + kappa S' (S = w S')
};
struct StepDests {            // product k goes to the complex128 at base + 2 * off[k]
    double *base;
    int64_t off[kStepMaxPhi];
};
// partials: reduce_blocks(n) * kStepMaxPhi complex128.  dests == nullptr: no products kept.
template <typename R>
void launch_sweep_step(const StepRegs &regs, const StepGate &g, double *partials, const StepDests *dests,
                       hipStream_t st);
// CNOT (cnot = true; control a, target b) or CZ on lambda and every phi register.
template <typename R> void launch_fixed_multi(const StepRegs &regs, int n, bool cnot, int a, int b, hipStream_t st);

template <typename R> void launch_init_state(void *dst, int n, const void *src_c128, hipStream_t st);
template <typename R> void launch_to_c128(const void *src, void *dst, int n, hipStream_t st);
template <typename R> void launch_copy(const void *src, void *dst, int n, hipStream_t st);

// Apply a 2x2 matrix on qubit q to one register (s1 == nullptr) or to two.
template <typename R> void launch_apply_1q(void *s0, void *s1, int n, int q, const DevMat2 &m, hipStream_t st);
// As launch_apply_1q, the matrix read from device memory (8 doubles: a, b, c, d as re, im).
template <typename R> void launch_apply_1q_tab(void *s0, void *s1, int n, int q, const double *m_dev, hipStream_t st);
// Controlled: the matrix acts on qubit q where qubit c (!= q) is 1.
template <typename R>
void launch_apply_c1q(void *s0, void *s1, int n, int c, int q, const DevMat2 &m, hipStream_t st);
// The same with the matrix in device memory (8 doubles), for captured graphs.
template <typename R>
void launch_apply_c1q_tab(void *s0, void *s1, int n, int c, int q, const double *m_dev, hipStream_t st);
template <typename R> void launch_cnot(void *s0, void *s1, int n, int control, int target, hipStream_t st);

// A run of CNOTs (control[k], target[k], k = 0 .. count-1, applied in that
// order) as one permutation of the amplitudes, out of place: dst[y] =
// src[x] with x the index the run maps to y.  count <= kCnotRunMax.
constexpr int kCnotRunMax = 64;
template <typename R>
void launch_cnot_run(const void *src, void *dst, int n, const int *control, const int *target, int count,
                     hipStream_t st);

// Pauli-string gates, S in mask form (S psi)[x] = (-i)^{n_y} (-1)^{popcount(x & zy)} psi[x ^ flip]:
// apply c + (sr + i si) S to one register (s1 == nullptr) or two; lam = y, phi = S y;
// dest (one complex128) = <a| S |b> (partials: reduce_blocks(n) complex128).
template <typename R>
void launch_apply_string(void *s0, void *s1, int n, uint64_t flip, uint64_t zy, int n_y, double c, double sr,
                         double si, hipStream_t st);
template <typename R>
void launch_seed_string(const void *y, void *lam, void *phi, int n, uint64_t flip, uint64_t zy, int n_y,
                        hipStream_t st);
template <typename R>
void launch_string_prod(const void *a, const void *b, int n, uint64_t flip, uint64_t zy, int n_y, double *partials,
                        double *dest, hipStream_t st);
template <typename R> void launch_cz(void *s0, void *s1, int n, int a, int b, hipStream_t st);

// lam = y; phi = sigma_q y  (axis 0/1/2 = X/Y/Z).  ctrl >= 0: phi = (|1><1|_ctrl (x) sigma_q) y,
// the generator of a controlled rotation.
template <typename R>
void launch_seed(const void *y, void *lam, void *phi, int n, int q, int axis, hipStream_t st, int ctrl = -1);

// Start of a metric column in one pass over the forward register:
// psi <- R psi (R: the rotation on qubit qr whose matrix is m_dev, 8 doubles;
// qr < 0: no gate), lam = psi, phi = sigma_qs psi (axis 0/1/2 = X/Y/Z) and
// dest (one complex128) = <psi| sigma_qs |psi>.  partials: reduce_blocks(n) complex128.
template <typename R>
void launch_advance_seed(void *psi, void *lam, void *phi, int n, int qr, const double *m_dev, int qs, int axis,
                         double *partials, double *dest, hipStream_t st);

// Column seeds of several registers in one launch (the batched metric): item
// k applies its forward rotations qa (matrix ma) then qb (mb) (-1: none) to
// psi, then lam = psi, phi = sigma_qs psi, and its work-groups write partial
// sums of <psi|sigma_qs|psi> at partials[2 * (block_begin .. block_begin +
// nblocks - 1)] (sum them with launch_reduce_tasks).  Registers of >= 3 qubits;
// block_begin ascending, total_blocks = the last item's end.
struct SeedItem {
    void *psi, *lam, *phi;
    const double *ma, *mb;   // 8 doubles each (a, b, c, d as re, im), device
    int32_t qa, qb, qs, axis, n;
    uint32_t block_begin, nblocks;
    int32_t pad;
};
template <typename R>
void launch_seed_multi(const SeedItem *items, int n_items, uint32_t total_blocks, double *partials, hipStream_t st);
// The same with two rotations before y_s (qa, ma first, then qb, mb; three
// distinct qubits qa, qb, qc = the seeded column's qubit, n >= 3): one pass.
template <typename R>
void launch_advance2_seed(void *psi, void *lam, void *phi, int n, int qa, const double *ma, int qb, const double *mb,
                          int qc, int axis, double *partials, double *dest, hipStream_t st);

// dest (one complex128) = <a| sigma_q |b>; axis -1 means the identity (plain inner product).
// ctrl >= 0: <a| |1><1|_ctrl (x) sigma_q |b> (only amplitudes with bit ctrl = 1).
// partials: reduce_blocks(n) complex128 scratch.
template <typename R>
void launch_pauli_prod(const void *a, const void *b, int n, int q, int axis, double *partials, double *dest,
                       hipStream_t st, int ctrl = -1);

// out = H psi for H = sum_t c_t S_t in one pass per chunk of kHamChunk terms
// (each amplitude of out gathers psi[x ^ flip_t] of every term), and
// dest (one complex128, nullable) = <psi|out> from the stored values.
// c_t holds coeff_t (-i)^{n_y} of term t.  partials: reduce_blocks(n) complex128.
constexpr int kHamChunk = 96;
struct HamTerm {
    uint64_t flip, zy;
    double cr, ci;
};
template <typename R>
void launch_pauli_sum(const void *psi, void *out, int n, const HamTerm *terms, int n_terms, double *partials,
                      double *dest, hipStream_t st);

// out (+)= coeff * (-i)^{n_y} (-1)^{popcount(x & zy)} psi[x ^ flip]; first != 0 overwrites.
template <typename R>
void launch_pauli_term(const void *psi, void *out, int n, uint64_t flip, uint64_t zy, int n_y, double coeff,
                       int first, hipStream_t st);

// Device-side unpack of G = L - T^* T into parameter order (Alg. 1 unpack):
// Lraw[r*P+s] (r<s, rotation order) holds <lam|sigma_r|phi>, Traw[s] holds <y_s|sigma_s|y_s>;
// param_of[r] maps rotation r to its parameter index.  G_out: P*P complex, T_out: P complex (nullable).
// param_of = NULL: rotation order.  rot_block (nullable): block id per
// rotation; entries between rotations of different blocks are set to zero
// (block-diagonal approximation).  rot_ctrl (nullable): control qubit per
// rotation (-1: plain); a controlled rotation s takes L_ss = Lraw[s*P+s] / 4,
// where the caller stored <y_s|(|1><1| on the control)|y_s> (Sec. 2); plain
// rotations take 1/4.  l_only: G = L (the conj(T_r) T_s term left out).
void launch_unpack_metric(const double *Lraw, const double *Traw, const int *param_of, int P, double *G_out,
                          double *T_out, const int *rot_block, const int *rot_ctrl, bool l_only, hipStream_t st);

// grad[param_of[r]] = -Im graw[r]   (d_r E = 2 Re[(i/2) <lambda|sigma_r|phi>]).
void launch_grad_from_raw(const double *graw, const int *param_of, int P, double *grad, hipStream_t st);

// Shared parameters (rotations rot[off[a] .. off[a+1]) carry parameter a):
// Gp = J^T G J, Tp = J^T T from G (P x P, rotation order) and T (P), and
// grad[a] = sum over those rotations of -Im graw[r].
void launch_contract_metric(const double *G, const double *T, int P, const int *off, const int *rot, int NP,
                            double *Gp, double *Tp, hipStream_t st);
void launch_grad_contract(const double *graw, const int *off, const int *rot, int NP, double *grad, hipStream_t st);

}  // namespace qng
