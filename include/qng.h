/*
 * qng.h -- C ABI of the MI355X (gfx950) quantum-natural-gradient library.
 *
 * The library evaluates, for a unitary ansatz U = U_P ... U_1 with one unique
 * parameter per parameterised gate acting on an input state |in>
 * (Jones, "Efficient classical calculation of the Quantum Natural Gradient",
 * Sec. 2 problem statement) -- or with parameters shared by several gates, whose
 * results are the contractions G' = J^T G J, T' = J^T T, grad' = J^T grad of
 * the one-parameter-per-gate results (J: gate parameter -> shared parameter;
 * the derivative of a shared angle is the sum over its gates):
 *
 *   - the quantum geometric tensor G_ij = L_ij - T_i^* T_j (Sec. 2, assembly
 *     equation; Sec. 1 definition), with L_ij = <d_i psi, d_j psi> and
 *     T_i = <psi, d_i psi>, by the recurrent O(P^2)-gate, O(1)-state-vector
 *     method of Sec. 3 (Alg. 1);
 *   - the energy <E> = <psi|H|psi> of a Pauli-sum Hamiltonian and its gradient
 *     vector (Sec. 1) by an O(P)-gate reverse sweep;
 *   - the natural-gradient step g dtheta = -dt grad E with g = Re G
 *     (Sec. 1), regularised as (Re G + eps I) dtheta = -dt grad E.
 *
 * Conventions (fixed for every entry point):
 *   - Qubit q is bit q of the amplitude index (qubit 0 = least significant bit).
 *   - A state of n qubits is 2^n complex amplitudes stored contiguously as
 *     interleaved (re, im) pairs: FP64 pairs for complex128 inputs/outputs.
 *   - Rotations use the paper's sign: R_sigma(theta) = exp(+i theta sigma / 2)
 *     (Sec. 2, rotation example).  The common exp(-i theta sigma/2) convention
 *     maps onto this one by theta -> -theta.
 *   - Row/column i of G, entry i of T, grad and dtheta refer to PARAMETER
 *     index i, not to gate position.
 *   - Matrices are row-major; a complex P x P matrix is 2*P*P doubles.
 *
 * Ownership and errors:
 *   - Every input pointer is borrowed for the duration of the call only.
 *   - Host outputs are caller-allocated; on error they are not written.
 *   - Host-pointer entry points are synchronous.  "_dev" entry points take
 *     device pointers, enqueue their work on the context's stream and return
 *     without waiting; their device outputs are valid once that stream has
 *     reached the end of the call.
 *   - A context owns its device workspace (grown on demand, freed by
 *     qng_destroy) and, unless one was supplied, its HIP stream.  A context
 *     must not be used from two threads at once.
 *   - No C++ exception crosses this boundary.  Every call returns a
 *     qng_status; on failure qng_last_error() describes the cause.
 *   - All validation happens before any device work, so invalid inputs never
 *     reach a kernel.
 */
#ifndef QNG_H
#define QNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QNG_OK = 0,
    QNG_E_INVALID_ARG = -1,     /* null pointer, bad size, unknown option/precision */
    QNG_E_BAD_CIRCUIT = -2,     /* qubit out of range, q0 == q1, unknown gate kind */
    QNG_E_BAD_PARAMS = -3,      /* a parameter index outside 0..n_params-1, or a parameter no rotation carries */
    QNG_E_NOT_NORMALIZED = -4,  /* | <in|in> - 1 | > 1e-12 */
    QNG_E_NONFINITE = -5,       /* NaN/Inf in theta, dt, eps, coefficients or the input state */
    QNG_E_OUT_OF_MEMORY = -6,   /* workspace above the device memory or the context's limit */
    QNG_E_NOT_SPD = -7,         /* Re G + eps I is not positive definite (e.g. eps = 0, singular G) */
    QNG_E_DEVICE = -8,          /* a HIP runtime call failed */
    QNG_E_UNSUPPORTED = -9      /* valid request this build does not implement */
} qng_status;

typedef enum {
    QNG_RX = 0, QNG_RY = 1, QNG_RZ = 2, QNG_CNOT = 3, QNG_CZ = 4,
    QNG_CRX = 5, QNG_CRY = 6, QNG_CRZ = 7,  /* controlled rotations (Sec. 2, the controlled-rotation diagonal) */
    QNG_RPAULI = 8                          /* Pauli-string rotation (Sec. 2, single-Pauli-string gates) */
} qng_gate_kind;

/* Storage precision of the state vectors.  QNG_C64 keeps states and gate
 * matrices in complex64 (rounded from FP64) while every product of an inner
 * product is formed from the stored FP32 values in FP64 and accumulated in
 * FP64, and the assembly of G and the solve stay in FP64.  With
 * QNG_OPT_EXACT_PRODUCTS = 0 the fused passes form each thread's share of an
 * inner product (at most 16 amplitudes) in FP32 instead, before the FP64 sums
 * (faster, a narrower arithmetic). */
typedef enum { QNG_C128 = 0, QNG_C64 = 1 } qng_precision;

/* One gate.  Rotations (RX/RY/RZ): q0 = target, q1 = -1, param = its parameter
 * index (>= 0).  CNOT: q0 = control, q1 = target, param = -1.  CZ: q0, q1 the
 * two qubits, param = -1.  Controlled rotations (CRX/CRY/CRZ): q0 = control,
 * q1 = target (q0 != q1), param >= 0; the gate is |0><0| (x) 1 + |1><1| (x)
 * exp(i theta sigma/2), so its column of G has the generator |1><1| (x) sigma
 * and the diagonal L_ii = 1/4 Prob(control = 1) instead of 1/4 (Sec. 2).
 * Pauli-string rotations (RPAULI): q0 = index of the string in the circuit's
 * table (0 <= q0 < n_strings), q1 = -1, param >= 0; the gate is
 * exp(i theta S/2) = cos(theta/2) + i sin(theta/2) S for the tensor product S
 * of the string's letters, so its column has the generator S and, as S^2 = 1,
 * the diagonal L_ii = 1/4.
 * With fusion on (QNG_OPT_FUSION = 1), controlled rotations run on the fused
 * sweep passes like the others (their control may be any qubit, their target
 * is brought into the pass's tile), and every Pauli-string rotation is
 * rewritten as the same unitary made of fixed basis rotations, CNOTs onto its
 * lowest qubit and an RZ there that carries its parameter (the state, and so
 * G, T, E and the gradient, are the same functions of theta), which the fused
 * passes take too; a string with no letter (a global phase) keeps the circuit
 * on one kernel per sweep step.  With fusion off, one kernel per primitive
 * with the string kernels.  qng_step_batched and the derivative-state
 * variant (QNG_OPT_METHOD = 1) take controlled rotations on the fused passes
 * and rewrite the strings the same way; with QNG_E_UNSUPPORTED both reject a
 * string with no letter, and qng_plan_export circuits with strings.
 * Gates act in array order: gates[0] first. */
typedef struct { int32_t kind, q0, q1, param; } qng_gate;

/* An ansatz: parameterised rotations whose param fields lie in
 * 0..n_params-1, each parameter carried by at least one rotation (one unique
 * parameter per gate, Sec. 2, when they form a permutation; otherwise shared
 * parameters, see above), plus any number of fixed CNOT/CZ gates.
 * strings: n_strings Pauli strings for RPAULI gates, n_qubits letters each,
 * strings[k*n_qubits + q] in {0=I, 1=X, 2=Y, 3=Z} acting on qubit q (host
 * pointer; may be NULL when n_strings = 0, which zero-initialised structs give). */
typedef struct {
    int32_t n_qubits;
    int32_t n_gates;
    int32_t n_params;
    const qng_gate *gates;
    int32_t n_strings;
    const uint8_t *strings;
} qng_circuit;

/* H = sum_t coeff[t] * (Pauli string t); pauli[t*n_qubits + q] in
 * {0=I, 1=X, 2=Y, 3=Z} acts on qubit q.  Host pointers. */
typedef struct {
    int32_t n_terms;
    const double *coeff;
    const uint8_t *pauli;
} qng_pauli_sum;

typedef struct qng_ctx qng_ctx;

/* Options for qng_set_option. */
typedef enum {
    QNG_OPT_FUSION = 0,          /* 1 (default): tiled fused sweep passes; 0: one kernel per primitive */
    QNG_OPT_TILE_QUBITS = 1,     /* qubits per on-chip tile of a fused pass (0 = automatic) */
    QNG_OPT_COLUMN_STREAMS = 2,  /* columns swept concurrently, each with its own 2 states (0 = automatic) */
    QNG_OPT_PROFILE = 3,         /* 1: time every sweep-pass launch with HIP events (see qng_stats) */
    QNG_OPT_SMALL_N_KERNEL = 4,  /* 1 (default): whole-column on-chip kernel for small registers */
    QNG_OPT_F64_REGISTERS = 5,   /* complex64 storage: 1 = sweep tiles computed in FP64 registers, 0 = FP32 */
    QNG_OPT_GRAPH = 6,           /* qng_step_batched: 1 (default) = capture the metric phase of a batch into a
                                    hipGraph on first use and replay it (needs a non-null stream) */
    QNG_OPT_AUTOTUNE = 7,        /* qng_step_batched: 1 = time candidate tile widths and launch sizes on the
                                    first call for a batch structure and keep the fastest; 0 (default) = fixed */
    QNG_OPT_BATCH_TILES = 8,     /* qng_step_batched: work-groups per sweep launch to aim for (0 = 4096) */
    QNG_OPT_BLOCK_COLUMNS = 9,   /* fused metric: columns sharing one lambda sweep, 1, 2 or 4 (0 = default: 4
                                    where it applies, else 2, else 1).  4 needs complex64 storage in FP32
                                    registers, tiles of 11 qubits (registers of >= 11 qubits) and no
                                    controlled rotation (in qng_step_batched, per member); 2 needs tiles of
                                    >= 11 qubits; where the choice does not apply the next smaller one is
                                    used */
    QNG_OPT_METRIC_KIND = 10,    /* 0 (default): G = L - T^* T; 1: L alone, L_ij = <d_i psi, d_j psi> (the
                                    coefficient matrix of imaginary-time evolution when psi's global phase does
                                    not depend on theta); T is still returned.  Metric and step entry points. */
    QNG_OPT_EXACT_PRODUCTS = 11  /* complex64 with FP32 registers: 1 (default) = every product formed and
                                    accumulated in FP64 (exact products of the stored FP32 values); 0 = each
                                    thread forms its share of an inner product (16 or fewer amplitudes) in FP32
                                    and converts it to FP64, all further sums FP64 (faster, narrower) */,
    QNG_OPT_METHOD = 12          /* how the metric's inner products are taken: 0 (default) = the recurrence of
                                    Sec. 3 (Alg. 1) with a constant number of states, each inner product formed
                                    in the sweep; 1 = the appendix's derivative-state strategy (its last
                                    algorithm: every derivative state prepared from a rolling prefix and kept):
                                    the same tiled sweeps carry every column's derivative state to one common
                                    frame without forming any product, the P + 1 states are kept (P + 2 states of
                                    device memory in all) and all inner products are one Gram matrix on the
                                    matrix cores (FP64 products and sums).  Where they do not fit (free device
                                    memory, qng_set_mem_limit) or QNG_OPT_STATE_CHUNK asks for it, the columns
                                    are prepared in chunks (see there).  Method 1 takes the fused passes'
                                    gate set (no string without a letter) and the full metric
                                    (QNG_E_UNSUPPORTED otherwise); qng_step_batched uses method 0. */,
    QNG_OPT_STATE_CHUNK = 13     /* method 1: at most this many derivative states per chunk, but at least one
                                    column block (0 = automatic: all P when they fit, else the most that
                                    fit).  With K > 1 chunks (whole column
                                    blocks, two chunks kept at once: 2 x chunk + 3 states) chunk i's states are
                                    paired with every chunk above it, which is prepared again each time:
                                    1 + K (K - 1) / 2 preparations of a chunk's states in place of K, and the
                                    same products.  QNG_E_OUT_OF_MEMORY when not even a chunk of one column
                                    block fits.  Results agree with the unchunked run to rounding (the Gram
                                    sums run in another order). */
} qng_option;

/* Counters of the last metric/energy/step call on a context. */
typedef struct {
    int64_t sweep_launches;      /* launches of the fused sweep-pass kernel */
    int64_t sweep_tiles;         /* tiles processed by those launches */
    double  sweep_ms;            /* summed HIP-event duration of those launches (QNG_OPT_PROFILE) */
    double  sweep_bytes;         /* algorithmic HBM bytes of those launches: read+write of lambda and of the phi
                                    states of each pass (2 states; 3 for a block of two columns) */
    double  sweep_flops;         /* algorithmic FLOPs of those launches, per amplitude per element: 8 for
                                    <lambda|sigma|phi> (4 for its real part, taken when qng_step has no G
                                    output), 6 for the rotation adjoint on phi, 6 on lambda shared by the
                                    columns of a block (20 for one column per sweep, 17 for two; 13 for two
                                    with real parts) */
    int64_t elements;            /* L_ij (i<j) elements evaluated */
    int64_t other_launches;      /* every other kernel launch */
    double  metric_ms;           /* wall-clock of the metric part (G) */
    double  grad_ms;             /* wall-clock of energy + gradient */
    double  solve_ms;            /* wall-clock of the FP64 solve */
    int32_t tile_qubits;         /* qng_step_batched: tile width used (0 = library default) */
    int32_t target_tiles;        /* qng_step_batched: work-groups per launch aimed for */
    double  tune_ms;             /* qng_step_batched: wall-clock spent autotuning in this call */
    int64_t graph_replays;       /* qng_step_batched: register classes run as a replay of a captured graph */
    int32_t block_columns;       /* fused metric: columns per lambda sweep of the last call (0: none ran) */
    int32_t state_chunks;        /* derivative-state variant: chunks its columns were prepared in (1: every
                                    state kept at once; 0: the variant did not run) */
} qng_stats;

/* Plan of a circuit under the current options (host only, no device work). */
typedef struct {
    int64_t passes;              /* fused sweep passes over all columns */
    int64_t elements;            /* P(P-1)/2 */
    int64_t ops;                 /* gate applications + inner products inside those passes */
    int64_t transposes;          /* LDS exchanges between register phases inside those passes */
    int32_t tile_qubits;         /* qubits per tile used by the plan */
    int32_t small_n;             /* 1 if the whole-column on-chip kernel is used */
} qng_plan_info;

/* ----------------------------------------------------------- context */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run
 * on, or NULL for a context-owned stream.  QNG_E_DEVICE if the device is absent. */
qng_status qng_create(qng_ctx **out, int device, void *hip_stream);
void qng_destroy(qng_ctx *ctx);
/* Message for the last failing call on ctx (or for the last failing qng_create
 * / host-only call when ctx is NULL).  Never NULL. */
const char *qng_last_error(const qng_ctx *ctx);
/* Run the context's work on hip_stream from now on.  NULL selects the HIP null
 * stream (ordered with all null-stream work, e.g. PyTorch's default stream);
 * a stream the context created itself is released. */
qng_status qng_set_stream(qng_ctx *ctx, void *hip_stream);
/* Cap on the workspace the context may allocate; 0 = device memory only.
 * A call whose workspace exceeds it fails with QNG_E_OUT_OF_MEMORY. */
qng_status qng_set_mem_limit(qng_ctx *ctx, size_t bytes);
qng_status qng_set_option(qng_ctx *ctx, int option, int value);
qng_status qng_get_stats(const qng_ctx *ctx, qng_stats *out);
/* Block-diagonal approximation of the metric (a cheaper variant: only the
 * entries between parameters of one block are formed).  block_of_param[a] is
 * the block id of parameter a (any int32 values; equal ids = one block).  The
 * metric and step entry points then return G (or L) with zeros between
 * different blocks and T in full; each column's sweep stops at the lowest
 * rotation of its block (no work for the entries left out).  The setting
 * applies to circuits with exactly n_params parameters (others fail with
 * QNG_E_INVALID_ARG) until n_params = 0 clears it; qng_step_batched rejects it.
 * The array is copied. */
qng_status qng_set_metric_blocks(qng_ctx *ctx, int32_t n_params, const int32_t *block_of_param);
/* Synchronise the context's stream. */
qng_status qng_synchronize(qng_ctx *ctx);

/* ---------------------------------------------- host-only (no GPU needed) */

/* Validate a circuit, parameters and (nullable) Hamiltonian without touching
 * a device.  Same rules and status codes as the compute entry points.  msg
 * (nullable) receives a description of the first problem found. */
qng_status qng_validate(const qng_circuit *circ, const double *theta, const qng_pauli_sum *ham,
                        char *msg, size_t msg_len);
/* Compile the sweep plan of a circuit for the given fusion mode and tile width
 * (0 = automatic) and report its size.  Host only. */
qng_status qng_plan(const qng_circuit *circ, int fusion, int tile_qubits, qng_plan_info *out);
/* Export a fused sweep plan (host only): one row of 10 int32 per operation,
 * in execution order (in-register exchanges omitted): {column s, pass index
 * within the column, kind (0 gate adjoint, 1 inner product then the adjoint of
 * its rotation, 2 inner product, 3 seed of a column's phi register), qubit q0
 * (CNOT: control), qubit q1 (CNOT target / CZ second qubit, else -1), gate
 * position of the adjoint (or -1), destination of an inner product (or -1),
 * Pauli axis of the inner product or seed (0 X, 1 Y, 2 Z; or -1), tile-qubit
 * mask bits 0..30, bits 31..61}.  A controlled rotation's adjoint row holds
 * its control in q0 and its target in q1 (as in the gate list); its inner
 * product and seed rows hold the target in q0 and the control in q1 (the
 * generator |1><1| on q1 times the axis's Pauli on q0; q1 = -1 for a plain one).
 * sweep = 0: the metric's columns s = 1..P-1 (Sec. 3, Alg. 1 inner loops),
 * destination r*P + s of <lambda|sigma_r|phi>; sweep = 2 (or 4): the same
 * metric with blocks of two (four) columns s-1, s (s-3 .. s) sharing one
 * lambda sweep (rows keyed by the top column s; an inner product for several
 * columns gives one row per destination, the adjoint on the last; a seed row
 * sets phi of column s_b to sigma lambda, sigma on qubit q0 with the row's
 * axis, and carries destination P*P + s_b of <lambda|phi>, i.e.
 * <y_{s_b}|sigma|y_{s_b}>); sweep = 1: the reverse sweep of the energy gradient
 * from the last gate (one column, s = P), destination r.
 * amp_bytes: 16 for complex128 plans, 8 for complex64.  With rows = NULL only
 * *n_rows is set. */
qng_status qng_plan_export(const qng_circuit *circ, int tile_qubits, int amp_bytes, int32_t sweep, int32_t *rows,
                           int64_t cap, int64_t *n_rows);
/* Solve (Re G + eps I) x = b in FP64 by Cholesky (host).  G: 2*P*P doubles
 * (complex, row-major), b, x: P doubles.  QNG_E_NOT_SPD if not positive definite. */
qng_status qng_solve_shifted(int32_t P, const double *G, double eps, const double *b, double *x);

/* ------------------------------------------------- host-pointer entry points */

/* Quantum geometric tensor by the recurrent method (Sec. 3, Alg. 1).
 * in_state: 2*2^n doubles (complex128) or NULL for |0...0>.  theta: P doubles.
 * G_out: 2*P*P doubles.  T_out: 2*P doubles or NULL. */
qng_status qng_metric(qng_ctx *ctx, const qng_circuit *circ, const double *in_state,
                      const double *theta, qng_precision prec, double *G_out, double *T_out);

/* Energy E = Re <psi|H|psi> and its gradient dE/dtheta (P doubles) by the
 * reverse sweep (Sec. 1 definitions; O(P) gates, O(1) states). */
qng_status qng_energy_grad(qng_ctx *ctx, const qng_circuit *circ, const double *in_state,
                           const qng_pauli_sum *ham, const double *theta, qng_precision prec,
                           double *E_out, double *grad_out);

/* One natural-gradient step (Sec. 1): dtheta solving (Re G + eps I) dtheta = -dt grad E.
 * G_out (2*P*P), grad_out (P), E_out (1) are optional (NULL = not returned).
 * The solve reads Re G only; with G_out = NULL the fused passes form only the
 * real parts of the metric's inner products (half their multiply-adds), with
 * G_out the full complex G is computed and returned. */
qng_status qng_step(qng_ctx *ctx, const qng_circuit *circ, const double *in_state,
                    const qng_pauli_sum *ham, const double *theta, double dt, double tikhonov,
                    qng_precision prec, double *dtheta_out, double *G_out, double *grad_out,
                    double *E_out);

/* B independent steps, one per ansatz (each its own circuit, input state,
 * Hamiltonian and theta; n and P may differ).  Array-of-pointer arguments have
 * B entries; in_states[b] may be NULL (|0...0>); G_out/grad_out/E_out may be
 * NULL as a whole.  The ansaetze are swept together: every launch carries
 * tiles of several ansaetze.  Without any G output the sweeps form only the
 * real parts of the metric's inner products, as qng_step does. */
qng_status qng_step_batched(qng_ctx *ctx, int32_t B, const qng_circuit *circs,
                            const double *const *in_states, const qng_pauli_sum *hams,
                            const double *const *thetas, double dt, double tikhonov,
                            qng_precision prec, double *const *dtheta_out, double *const *G_out,
                            double *const *grad_out, double *E_out);

/* ------------------------------------------------- device-pointer entry points
 * Device buffers: in_state_dev is complex128 (2*2^n doubles) or NULL;
 * outputs are FP64 device buffers of the sizes given above.  theta stays a
 * host pointer (the gate matrices are built on the host). */

qng_status qng_metric_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                          const double *theta, qng_precision prec, void *G_dev, void *T_dev);

/* Energy only: writes E (1 double) to E_dev and the final ansatz state psi
 * (complex128, 2*2^n doubles) to psi_dev, for a later qng_energy_grad_from_state_dev. */
qng_status qng_energy_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                          const qng_pauli_sum *ham, const double *theta, qng_precision prec,
                          void *E_dev, void *psi_dev);

/* Gradient by the reverse sweep, starting from a final state psi_dev produced by
 * qng_energy_dev for the same circuit/theta (it is read, not modified). */
qng_status qng_energy_grad_from_state_dev(qng_ctx *ctx, const qng_circuit *circ,
                                          const qng_pauli_sum *ham, const double *theta,
                                          qng_precision prec, const void *psi_dev, void *grad_dev);

/* Energy E = Re <psi|H|psi> and its gradient dE/dtheta (Sec. 1 definitions)
 * with device outputs: the arguments of qng_energy_grad, in_state_dev a
 * complex128 device state (NULL: |0...0>), E_dev one double and grad_dev P
 * doubles (parameter order) in device memory.  O(P) gates by the reverse
 * sweep; asynchronous on the context's stream. */
qng_status qng_energy_grad_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                               const qng_pauli_sum *ham, const double *theta, qng_precision prec, void *E_dev,
                               void *grad_dev);

/* qng_energy_grad_dev for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and results, but the call allocates
 * nothing.  Its whole workspace is a fixed device scratch of 64 MiB that the
 * library holds on every GPU it runs on until the process ends (looked up by
 * qng_create on that device); the context's own workspace is not used.
 * Fits complex128 registers up to n = 20 and complex64 up to n = 21 (two
 * registers plus the gradient's plan and partial sums); a call that needs
 * more fails with QNG_E_OUT_OF_MEMORY before any device work.  All calls on
 * one GPU share that scratch: calls that overlap on one GPU (two contexts,
 * two streams, two threads) race and must be ordered by the caller.  Kept
 * state: none -- every buffer is written before it is read in each call. */
qng_status qng_energy_grad_dev_noalloc(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                                       const qng_pauli_sum *ham, const double *theta, qng_precision prec,
                                       void *E_dev, void *grad_dev);

/* One natural-gradient step (Sec. 1: (Re G + eps I) dtheta = -dt grad E) with
 * device outputs: the arguments of qng_step, in_state_dev a complex128 device
 * state (NULL: |0...0>), dtheta_dev P doubles, G_dev 2*P*P doubles (NULL = not
 * returned; then the metric's inner products keep their real parts, as in
 * qng_step), grad_dev P doubles (nullable), E_dev one double (nullable), all
 * in device memory.  The shifted system is solved on the device (FP64
 * Cholesky), so nothing leaves the device.  status_dev (nullable) receives the
 * solve's status as one int32 in device memory: QNG_OK, or QNG_E_NOT_SPD when
 * Re G + eps I is not positive definite -- then none of the outputs is
 * written.  With status_dev the call is asynchronous on the context's stream
 * and returns QNG_OK once the work is enqueued; with status_dev = NULL it
 * waits for its stream and returns QNG_E_NOT_SPD itself in that case. */
qng_status qng_step_dev(qng_ctx *ctx, const qng_circuit *circ, const void *in_state_dev,
                        const qng_pauli_sum *ham, const double *theta, double dt, double tikhonov,
                        qng_precision prec, void *dtheta_dev, void *G_dev, void *grad_dev, void *E_dev,
                        int32_t *status_dev);

/* The clone primitive of the paper (appendix introduction: clone a state,
 * apply a gate, take an inner product): dst_dev <- src_dev, 2^n_qubits
 * amplitudes of the storage type of prec (complex128 or complex64), distinct
 * device buffers.  Asynchronous on the context's stream; no workspace. */
qng_status qng_clone_state_dev(qng_ctx *ctx, int32_t n_qubits, qng_precision prec, const void *src_dev,
                               void *dst_dev);

/* Apply the ansatz (every gate, in order) to a device state in place:
 * state_dev <- U(theta) state_dev (Sec. 2, psi = U|in>).  The state has the
 * storage type of prec: complex128 (QNG_C128) or complex64 (QNG_C64), 2^n
 * amplitudes.  Asynchronous on the context's stream; no workspace. */
qng_status qng_apply_circuit_dev(qng_ctx *ctx, const qng_circuit *circ, const double *theta, qng_precision prec,
                                 void *state_dev);

#ifdef __cplusplus
}
#endif

#endif /* QNG_H */
