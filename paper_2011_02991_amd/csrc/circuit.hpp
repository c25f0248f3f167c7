// circuit.hpp -- host-side validation and compilation of an ansatz.
//
// The ansatz is U = U_P ... U_1 acting on |in>, one unique parameter per
// parameterised gate (Sec. 2, problem statement).  Fixed gates (CNOT, CZ) are
// allowed anywhere; they carry no parameter.  Rotations follow the paper's
// sign, R_sigma(theta) = exp(+i theta sigma / 2) (Sec. 2, rotation example).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/qng.h"

namespace qng {

using cd = std::complex<double>;

// Thrown by host code; converted to a qng_status at the C ABI boundary.
struct Error {
    qng_status status;
    std::string msg;
};

[[noreturn]] inline void fail(qng_status s, const std::string &m) { throw Error{s, m}; }

enum Axis : int { AX_X = 0, AX_Y = 1, AX_Z = 2 };

struct Mat2 {  // row-major 2x2 complex, [[a, b], [c, d]]
    cd a, b, c, d;
};

// One rotation of the ansatz, in gate-list order.  A controlled rotation
// (ctrl >= 0) rotates `qubit` where qubit `ctrl` is 1; its generator is
// |1><1|_ctrl (x) sigma, which replaces sigma in every product of its column.
// A Pauli-string rotation (string >= 0) has the generator S given by its masks
// (S psi)[x] = (-i)^{n_y} (-1)^{popcount(x & zy)} psi[x ^ flip]; axis and qubit
// are unused for it.
struct Rot {
    int axis;    // generator sigma: X, Y or Z
    int qubit;
    int param;   // parameter index (row/column of G)
    int pos;     // position in the gate list
    int ctrl = -1;
    int string = -1;
    uint64_t flip = 0, zy = 0;
    int n_y = 0;
};

struct Circuit {
    int n = 0;              // qubits
    int M = 0;              // gates
    int P = 0;              // rotations (one recurrence column each)
    int NP = 0;             // parameters; NP < P when rotations share parameters
    bool shared = false;    // some parameter is carried by several rotations
    bool controlled = false;  // some rotation is a controlled rotation
    bool has_strings = false; // some rotation is a Pauli-string rotation
    bool lowered = false;     // Pauli-string rotations rewritten (lower_strings)
    std::vector<qng_gate> gates;
    std::vector<int> rot_at;   // gate position -> rotation index (list order) or -1
    std::vector<Rot> rots;     // rotations in list order
    // Fixed single-qubit rotations exist in lowered circuits only: an RX/RY/RZ
    // gate with param = -1 turns by fixed_angle[pos] (0 at every other position;
    // empty when there are none).
    std::vector<double> fixed_angle;
    bool is_fixed_rotation(int pos) const { return gates[pos].kind <= QNG_RZ && gates[pos].param < 0; }
};

// Validation rules shared by every entry point (all before any device work).
void validate_circuit(const qng_circuit *c, int max_qubits);
void validate_theta(const qng_circuit *c, const double *theta);
void validate_hamiltonian(const qng_circuit *c, const qng_pauli_sum *h);
void validate_scalar(double v, const char *name);

Circuit compile_circuit(const qng_circuit *c);

// A Pauli-string rotation exp(i theta S/2) is U^dagger exp(i theta Z_p/2) U
// for U = C B: B turns each X letter into Z with RY(pi/2) and each Y letter
// with RX(-pi/2) (so B S B^dagger is Z on the whole support), and C, CNOTs from
// every other support qubit onto the pivot p (the lowest one), leaves Z_p
// alone.  lower_strings rewrites every string rotation as that gate sequence
// (B, C, RZ_p(theta), C, B^dagger): the state is the same function of the
// parameters, so are G, T, E and its gradient, and the rotation keeps its
// place in the rotation order with Z_p as its generator in the rewritten frame.
// Strings with no letter (a global phase) cannot be rewritten this way.
bool strings_lowerable(const Circuit &c);
Circuit lower_strings(const Circuit &c);

// R(theta) and R(theta)^dagger for a rotation axis.
Mat2 rotation(int axis, double theta);
Mat2 adjoint(const Mat2 &m);

// On pairs of real numbers, every adjoint rotation is the plane rotation
// [[c, s], [-s, c]]: RX on (re x0, im x1) and (re x1, im x0), RY on (re x0,
// re x1) and (im x0, im x1), RZ on (re x, im x) of the |0> amplitude and with s
// negated for the |1> amplitude.  The sweep applies it in place as three shears
//   a += u b;  b += w a;  a += u b,   u = s / (1 + c), w = -s.
// A rotation with c < 0 is applied as its negative (the same sign on both
// registers of a sweep cancels in every <lambda|sigma|phi>), so |u| <= 1.
struct Shear {
    double u, w;
};
Shear adjoint_shear(int axis, const Mat2 &adj);
// The same plane rotation as (c, s) without the negation: a controlled rotation
// acts on half of the amplitudes only, so a sign on it would not be global.
struct PlaneRot {
    double c, s;
};
PlaneRot adjoint_plane(int axis, const Mat2 &adj);

// Pauli string in bit-mask form: (sigma psi)[x] = (-i)^{nY} (-1)^{popcount(x & zy)} psi[x ^ flip],
// with flip = positions of X and Y letters, zy = positions of Z and Y letters
// (Y = -i (-1)^{x_q} on the flipped bit: Y|0> = i|1>, Y|1> = -i|0>).
struct PauliTerm {
    uint64_t flip = 0, zy = 0;
    int n_y = 0;
    double coeff = 0;
};
std::vector<PauliTerm> compile_hamiltonian(const qng_circuit *c, const qng_pauli_sum *h);

}  // namespace qng
