/*
 * oracle.c -- plain FP64 CPU state-vector oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
 * load this file; only tests/, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the HIP
 * path (it keeps its own gate encoding constants, its own matrices and its own
 * loops).
 *
 * What it computes, and where in the paper each step is defined
 * (Jones, "Efficient classical calculation of the Quantum Natural Gradient"):
 *
 *  - The ansatz state psi = U_P ... U_1 |in>, one unique parameter per
 *    parameterised gate (Sec. 2, problem statement).  Non-parameterised
 *    gates (CNOT, CZ) are applied in list order like any other gate.
 *  - Rotations follow the paper's convention R_sigma(theta) =
 *    exp(+i theta sigma / 2) = cos(theta/2) I + i sin(theta/2) sigma
 *    (Sec. 2, the Pauli-generator discussion and the rotation example).
 *  - The derivative state d psi / d theta_p: every gate applied in order, with
 *    the gate that carries parameter p replaced by the entrywise derivative of
 *    its matrix, -1/2 sin(theta/2) I + i/2 cos(theta/2) sigma.  This is the
 *    plain definition of the partial derivative of U|in> (Sec. 1, definition
 *    of the geometric tensor), evaluated one derivative state per parameter
 *    with a rolling prefix state as in the appendix algorithm that prepares
 *    every derivative state from a cached prefix.
 *  - A Pauli-sum Hamiltonian applied term by term, each Pauli string acting
 *    letter by letter on a computational basis state.
 *
 * The Gram matrix <d_i psi | d_j psi>, T, G, E, the gradient and the linear
 * solve are assembled from these states by the Python wrapper with numpy
 * (library matrix products and a library solver).
 *
 * Conventions: qubit q is bit q of the amplitude index; amplitudes are C99
 * double complex, contiguous.  Gate rows are (kind, q0, q1, param) with
 * kind 0/1/2 = RX/RY/RZ on q0, 3 = CNOT (control q0, target q1), 4 = CZ,
 * 5/6/7 = controlled RX/RY/RZ (control q0, target q1): the rotation acts on the
 * target where the control is 1, the identity where it is 0, so its derivative
 * is the rotation's derivative where the control is 1 and zero where it is 0,
 * 8 = Pauli-string rotation exp(i theta S/2) with S the tensor product of the
 * letters strings[q0*n + q] (0..3 = I, X, Y, Z on qubit q), q1 = -1; since
 * S^2 = 1 it equals cos(theta/2) + i sin(theta/2) S and its derivative is
 * (i/2) S exp(i theta S/2) (Sec. 2, Pauli-string generators).
 *
 * Loops over amplitudes may run on several OpenMP threads; every amplitude is
 * written by exactly one iteration, so the result does not depend on the
 * thread count.  There are no sums across amplitudes in this file.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { OR_KIND_RX = 0, OR_KIND_RY = 1, OR_KIND_RZ = 2, OR_KIND_CNOT = 3, OR_KIND_CZ = 4,
       OR_KIND_CRX = 5, OR_KIND_CRY = 6, OR_KIND_CRZ = 7, OR_KIND_RPAULI = 8 };

/* Pauli matrix of a rotation kind, row-major [[s0, s1], [s2, s3]]. */
static void or_pauli_of_kind(int kind, cplx s[4])
{
    switch (kind) {
    case OR_KIND_RX: s[0] = 0; s[1] = 1;  s[2] = 1; s[3] = 0;  break;
    case OR_KIND_RY: s[0] = 0; s[1] = -I; s[2] = I; s[3] = 0;  break;
    default:         s[0] = 1; s[1] = 0;  s[2] = 0; s[3] = -1; break;
    }
}

/* R(theta) = cos(theta/2) I + i sin(theta/2) sigma. */
static void or_rotation(int kind, double theta, cplx m[4])
{
    cplx s[4];
    or_pauli_of_kind(kind, s);
    double c = cos(0.5 * theta), sn = sin(0.5 * theta);
    m[0] = c + I * sn * s[0];
    m[1] = I * sn * s[1];
    m[2] = I * sn * s[2];
    m[3] = c + I * sn * s[3];
}

/* dR/dtheta, entry by entry: -1/2 sin(theta/2) I + i/2 cos(theta/2) sigma. */
static void or_rotation_derivative(int kind, double theta, cplx m[4])
{
    cplx s[4];
    or_pauli_of_kind(kind, s);
    double c = cos(0.5 * theta), sn = sin(0.5 * theta);
    m[0] = -0.5 * sn + I * 0.5 * c * s[0];
    m[1] = I * 0.5 * c * s[1];
    m[2] = I * 0.5 * c * s[2];
    m[3] = -0.5 * sn + I * 0.5 * c * s[3];
}

/* psi <- (m on qubit q) psi */
static void or_apply_1q(cplx *psi, int n, int q, const cplx m[4])
{
    const int64_t dim = (int64_t)1 << n, bit = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if (i & bit) continue;
        const int64_t j = i | bit;
        const cplx a = psi[i], b = psi[j];
        psi[i] = m[0] * a + m[1] * b;
        psi[j] = m[2] * a + m[3] * b;
    }
}

/* (m on qubit t) where qubit c is 1; where c is 0 the amplitudes are kept, or
 * set to zero if zero_off (the derivative of a controlled rotation). */
static void or_apply_controlled_1q(cplx *psi, int n, int c, int t, const cplx m[4], int zero_off)
{
    const int64_t dim = (int64_t)1 << n, cb = (int64_t)1 << c, tb = (int64_t)1 << t;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if (i & tb) continue;
        const int64_t j = i | tb;
        if (!(i & cb)) {
            if (zero_off) { psi[i] = 0; psi[j] = 0; }
            continue;
        }
        const cplx a = psi[i], b = psi[j];
        psi[i] = m[0] * a + m[1] * b;
        psi[j] = m[2] * a + m[3] * b;
    }
}

/* CNOT: |c t> -> |c, t xor c> */
static void or_apply_cnot(cplx *psi, int n, int control, int target)
{
    const int64_t dim = (int64_t)1 << n, cb = (int64_t)1 << control, tb = (int64_t)1 << target;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i) {
        if ((i & cb) && !(i & tb)) {
            const cplx tmp = psi[i];
            psi[i] = psi[i | tb];
            psi[i | tb] = tmp;
        }
    }
}

/* CZ: |11> picks up a factor -1 */
static void or_apply_cz(cplx *psi, int n, int a, int b)
{
    const int64_t dim = (int64_t)1 << n, ab = (int64_t)1 << a, bb = (int64_t)1 << b;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < dim; ++i)
        if ((i & ab) && (i & bb)) psi[i] = -psi[i];
}

/*
 * out (+)= factor * S psi for the Pauli string S with letters p[0..n) (p[q]
 * acts on qubit q, 0..3 = I, X, Y, Z).  A Pauli string has one nonzero entry
 * per row: row y picks column x (X and Y flip bit q, I and Z keep it) with a
 * factor that is the product over qubits of the letter's matrix entry
 * <y_q|letter|x_q>: X gives 1, Y gives -i for y_q = 0 and +i for y_q = 1
 * (Y|0> = i|1>, Y|1> = -i|0>), Z gives (-1)^{y_q}.
 */
static void or_add_string(int n, const uint8_t *p, cplx factor0, const cplx *psi, cplx *out)
{
    const int64_t dim = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t y = 0; y < dim; ++y) {
        int64_t x = y;
        cplx factor = factor0;
        for (int q = 0; q < n; ++q) {
            const int64_t bit = (int64_t)1 << q;
            switch (p[q]) {
            case 1: x ^= bit; break;                              /* X|b> = |1-b> */
            case 2: x ^= bit; factor *= (x & bit) ? -I : I; break; /* Y|0>=i|1>, Y|1>=-i|0> */
            case 3: if (y & bit) factor = -factor; break;         /* Z|1> = -|1> */
            default: break;
            }
        }
        out[y] += factor * psi[x];
    }
}

/* Pauli-string rotation: psi <- cos(t/2) psi + i sin(t/2) S psi; derivative:
 * then psi <- (i/2) S psi. */
static void or_apply_string_rotation(cplx *psi, int n, const uint8_t *p, double t, int derivative)
{
    const int64_t dim = (int64_t)1 << n;
    cplx *tmp = (cplx *)malloc((size_t)dim * sizeof(cplx));
    memcpy(tmp, psi, (size_t)dim * sizeof(cplx));
    for (int64_t x = 0; x < dim; ++x) psi[x] *= cos(0.5 * t);
    or_add_string(n, p, I * sin(0.5 * t), tmp, psi);
    if (derivative) {
        memset(tmp, 0, (size_t)dim * sizeof(cplx));
        or_add_string(n, p, 0.5 * I, psi, tmp);
        memcpy(psi, tmp, (size_t)dim * sizeof(cplx));
    }
    free(tmp);
}

/* Apply gate row g; if derivative != 0 the rotation is replaced by dR/dtheta.
 * strings: the Pauli-string table of kind-8 gates (n letters per string). */
static void or_apply_gate(cplx *psi, int n, const int32_t *g, const double *theta, int derivative,
                          const uint8_t *strings)
{
    const int kind = g[0];
    if (kind == OR_KIND_RPAULI) {
        or_apply_string_rotation(psi, n, strings + (int64_t)g[1] * n, theta[g[3]], derivative);
        return;
    }
    if (kind == OR_KIND_CNOT) { or_apply_cnot(psi, n, g[1], g[2]); return; }
    if (kind == OR_KIND_CZ)   { or_apply_cz(psi, n, g[1], g[2]); return; }
    const int controlled = kind >= OR_KIND_CRX;
    const int axis = controlled ? kind - OR_KIND_CRX : kind;
    cplx m[4];
    if (derivative) or_rotation_derivative(axis, theta[g[3]], m);
    else            or_rotation(axis, theta[g[3]], m);
    if (controlled) or_apply_controlled_1q(psi, n, g[1], g[2], m, derivative);
    else            or_apply_1q(psi, n, g[1], m);
}

static void or_load_input(cplx *psi, int n, const cplx *in_state)
{
    const int64_t dim = (int64_t)1 << n;
    if (in_state) memcpy(psi, in_state, (size_t)dim * sizeof(cplx));
    else { memset(psi, 0, (size_t)dim * sizeof(cplx)); psi[0] = 1.0; }
}

/* ---------------------------------------------------------------- exports */

/* Ansatz state: every gate applied to |in> in list order.  Returns 0. */
int oracle_forward(int n, int n_gates, const int32_t *gates, const double *theta,
                   const cplx *in_state, cplx *out, const uint8_t *strings)
{
    or_load_input(out, n, in_state);
    for (int k = 0; k < n_gates; ++k) or_apply_gate(out, n, gates + 4 * k, theta, 0, strings);
    return 0;
}

/*
 * Derivative states d psi / d theta_p for the parameters listed in sel[0..n_sel).
 * out holds n_sel states back to back (n_sel * 2^n amplitudes).  A rolling prefix
 * state is advanced gate by gate; at a gate carrying a selected parameter, the
 * prefix is cloned, the derivative matrix applied and the remaining gates applied
 * to the clone.  A parameter carried by several gates gets the sum of those
 * terms (the product rule: U depends on theta_p through each of them).
 * psi_out (nullable) receives the ansatz state.
 * Returns 0, or -1 if a selected parameter carries no gate.
 */
int oracle_derivative_states(int n, int n_gates, const int32_t *gates, const double *theta,
                             const cplx *in_state, int n_sel, const int32_t *sel,
                             cplx *out, cplx *psi_out, const uint8_t *strings)
{
    const int64_t dim = (int64_t)1 << n;
    cplx *prefix = (cplx *)malloc((size_t)dim * sizeof(cplx));
    cplx *term = (cplx *)malloc((size_t)dim * sizeof(cplx));
    char *seen = (char *)calloc((size_t)(n_sel > 0 ? n_sel : 1), 1);
    if (!prefix || !term || !seen) { free(prefix); free(term); free(seen); return -2; }
    or_load_input(prefix, n, in_state);
    for (int k = 0; k < n_gates; ++k) {
        const int32_t *g = gates + 4 * k;
        if (g[3] >= 0) {
            for (int a = 0; a < n_sel; ++a) {
                if (sel[a] != g[3]) continue;
                cplx *d = out + (int64_t)a * dim;
                cplx *t = seen[a] ? term : d;
                memcpy(t, prefix, (size_t)dim * sizeof(cplx));
                or_apply_gate(t, n, g, theta, 1, strings);
                for (int k2 = k + 1; k2 < n_gates; ++k2) or_apply_gate(t, n, gates + 4 * k2, theta, 0, strings);
                if (seen[a])
                    for (int64_t x = 0; x < dim; ++x) d[x] += term[x];
                seen[a] = 1;
            }
        }
        or_apply_gate(prefix, n, g, theta, 0, strings);
    }
    if (psi_out) memcpy(psi_out, prefix, (size_t)dim * sizeof(cplx));
    int missing = 0;
    for (int a = 0; a < n_sel; ++a) missing += !seen[a];
    free(prefix);
    free(term);
    free(seen);
    return missing ? -1 : 0;
}

/*
 * out = H psi with H = sum_t coeff[t] * (Pauli string t); pauli[t*n + q] in
 * {0=I, 1=X, 2=Y, 3=Z} acts on qubit q.
 */
int oracle_apply_pauli_sum(int n, int n_terms, const uint8_t *pauli, const double *coeff,
                           const cplx *psi, cplx *out)
{
    const int64_t dim = (int64_t)1 << n;
    memset(out, 0, (size_t)dim * sizeof(cplx));
    for (int t = 0; t < n_terms; ++t) or_add_string(n, pauli + (int64_t)t * n, coeff[t], psi, out);
    return 0;
}

/* Single-qubit Pauli on a state, used by tests of the letter conventions. */
int oracle_apply_pauli_letter(int n, int q, int letter, cplx *psi)
{
    cplx s[4];
    if (letter == 0) return 0;
    or_pauli_of_kind(letter == 1 ? OR_KIND_RX : letter == 2 ? OR_KIND_RY : OR_KIND_RZ, s);
    or_apply_1q(psi, n, q, s);
    return 0;
}

/* Apply one gate row (rotation, or its derivative if derivative != 0). */
int oracle_apply_gate(int n, const int32_t *gate, const double *theta, int derivative, cplx *psi,
                      const uint8_t *strings)
{
    or_apply_gate(psi, n, gate, theta, derivative, strings);
    return 0;
}
