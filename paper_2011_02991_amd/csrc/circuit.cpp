// circuit.cpp -- validation and compilation of an ansatz (host only).
#include "circuit.hpp"

#include <cmath>
#include <cstdio>

namespace qng {

void validate_scalar(double v, const char *name) {
    if (!std::isfinite(v)) fail(QNG_E_NONFINITE, std::string(name) + " is not finite");
}

void validate_circuit(const qng_circuit *c, int max_qubits) {
    if (!c) fail(QNG_E_INVALID_ARG, "circuit is NULL");
    if (c->n_qubits < 1 || c->n_qubits > max_qubits)
        fail(QNG_E_BAD_CIRCUIT, "n_qubits=" + std::to_string(c->n_qubits) + " outside [1, " +
                                    std::to_string(max_qubits) + "]");
    if (c->n_gates < 0) fail(QNG_E_BAD_CIRCUIT, "n_gates < 0");
    if (c->n_params < 0) fail(QNG_E_BAD_PARAMS, "n_params < 0");
    if (c->n_gates > 0 && !c->gates) fail(QNG_E_INVALID_ARG, "gates is NULL");
    if (c->n_strings < 0) fail(QNG_E_BAD_CIRCUIT, "n_strings < 0");
    if (c->n_strings > 0 && !c->strings) fail(QNG_E_INVALID_ARG, "strings is NULL");
    const int n = c->n_qubits;
    for (int64_t k = 0; k < (int64_t)c->n_strings * n; ++k)
        if (c->strings[k] > 3)
            fail(QNG_E_BAD_CIRCUIT, "Pauli letter outside {0,1,2,3} in string " + std::to_string(k / n));
    std::vector<int> seen(c->n_params, 0);
    int n_rot = 0;
    for (int k = 0; k < c->n_gates; ++k) {
        const qng_gate &g = c->gates[k];
        const std::string where = "gate " + std::to_string(k) + ": ";
        switch (g.kind) {
        case QNG_RX:
        case QNG_RY:
        case QNG_RZ:
            if (g.q0 < 0 || g.q0 >= n) fail(QNG_E_BAD_CIRCUIT, where + "qubit out of range");
            if (g.q1 != -1) fail(QNG_E_BAD_CIRCUIT, where + "rotation must have q1 = -1");
            if (g.param < 0) fail(QNG_E_BAD_PARAMS, where + "rotation needs a parameter index >= 0");
            if (g.param >= c->n_params) fail(QNG_E_BAD_PARAMS, where + "parameter index >= n_params");
            ++seen[g.param];
            ++n_rot;
            break;
        case QNG_CRX:
        case QNG_CRY:
        case QNG_CRZ:
            if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n)
                fail(QNG_E_BAD_CIRCUIT, where + "qubit out of range");
            if (g.q0 == g.q1) fail(QNG_E_BAD_CIRCUIT, where + "control and target are the same qubit");
            if (g.param < 0) fail(QNG_E_BAD_PARAMS, where + "rotation needs a parameter index >= 0");
            if (g.param >= c->n_params) fail(QNG_E_BAD_PARAMS, where + "parameter index >= n_params");
            ++seen[g.param];
            ++n_rot;
            break;
        case QNG_RPAULI:
            if (g.q0 < 0 || g.q0 >= c->n_strings) fail(QNG_E_BAD_CIRCUIT, where + "string index out of range");
            if (g.q1 != -1) fail(QNG_E_BAD_CIRCUIT, where + "Pauli-string rotation must have q1 = -1");
            if (g.param < 0) fail(QNG_E_BAD_PARAMS, where + "rotation needs a parameter index >= 0");
            if (g.param >= c->n_params) fail(QNG_E_BAD_PARAMS, where + "parameter index >= n_params");
            ++seen[g.param];
            ++n_rot;
            break;
        case QNG_CNOT:
        case QNG_CZ:
            if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n)
                fail(QNG_E_BAD_CIRCUIT, where + "qubit out of range");
            if (g.q0 == g.q1) fail(QNG_E_BAD_CIRCUIT, where + "two-qubit gate on a single qubit");
            if (g.param != -1) fail(QNG_E_BAD_PARAMS, where + "fixed gate must have param = -1");
            break;
        default:
            fail(QNG_E_BAD_CIRCUIT, where + "unknown gate kind " + std::to_string(g.kind));
        }
    }
    // a parameter may be carried by several rotations (its derivative is the
    // sum of theirs), but every parameter must be carried by one
    for (int p = 0; p < c->n_params; ++p)
        if (!seen[p])
            fail(QNG_E_BAD_PARAMS, "parameter " + std::to_string(p) + " is carried by no rotation (n_params=" +
                                       std::to_string(c->n_params) + ", " + std::to_string(n_rot) + " rotations)");
}

void validate_theta(const qng_circuit *c, const double *theta) {
    if (c->n_params > 0 && !theta) fail(QNG_E_INVALID_ARG, "theta is NULL");
    for (int p = 0; p < c->n_params; ++p)
        if (!std::isfinite(theta[p])) fail(QNG_E_NONFINITE, "theta[" + std::to_string(p) + "] is not finite");
}

void validate_hamiltonian(const qng_circuit *c, const qng_pauli_sum *h) {
    if (!h) fail(QNG_E_INVALID_ARG, "Hamiltonian is NULL");
    if (h->n_terms < 0) fail(QNG_E_INVALID_ARG, "n_terms < 0");
    if (h->n_terms > 0 && (!h->coeff || !h->pauli)) fail(QNG_E_INVALID_ARG, "Hamiltonian arrays are NULL");
    for (int t = 0; t < h->n_terms; ++t) {
        if (!std::isfinite(h->coeff[t])) fail(QNG_E_NONFINITE, "coeff[" + std::to_string(t) + "] is not finite");
        for (int q = 0; q < c->n_qubits; ++q)
            if (h->pauli[(size_t)t * c->n_qubits + q] > 3)
                fail(QNG_E_INVALID_ARG, "Pauli letter outside {0,1,2,3} in term " + std::to_string(t));
    }
}

Circuit compile_circuit(const qng_circuit *c) {
    Circuit k;
    k.n = c->n_qubits;
    k.M = c->n_gates;
    k.NP = c->n_params;
    k.gates.assign(c->gates, c->gates + c->n_gates);
    k.rot_at.assign(k.M, -1);
    for (int pos = 0; pos < k.M; ++pos) {
        const qng_gate &g = k.gates[pos];
        if (g.kind <= QNG_RZ) {
            k.rot_at[pos] = (int)k.rots.size();
            k.rots.push_back(Rot{g.kind == QNG_RX ? AX_X : g.kind == QNG_RY ? AX_Y : AX_Z, g.q0, g.param, pos});
        } else if (g.kind >= QNG_CRX && g.kind <= QNG_CRZ) {
            k.rot_at[pos] = (int)k.rots.size();
            k.rots.push_back(Rot{g.kind - QNG_CRX, g.q1, g.param, pos, g.q0});
            k.controlled = true;
        } else if (g.kind == QNG_RPAULI) {
            Rot r{AX_X, 0, g.param, pos};
            r.string = g.q0;
            for (int q = 0; q < k.n; ++q) {
                const uint8_t l = c->strings[(int64_t)g.q0 * k.n + q];
                if (l == 1 || l == 2) r.flip |= uint64_t(1) << q;
                if (l == 2 || l == 3) r.zy |= uint64_t(1) << q;
                r.n_y += l == 2;
            }
            k.rot_at[pos] = (int)k.rots.size();
            k.rots.push_back(r);
            k.has_strings = true;
        }
    }
    k.P = (int)k.rots.size();
    k.shared = k.P != k.NP;
    return k;
}

bool strings_lowerable(const Circuit &c) {
    for (const Rot &r : c.rots)
        if (r.string >= 0 && (r.flip | r.zy) == 0) return false;
    return true;
}

Circuit lower_strings(const Circuit &c) {
    Circuit k;
    k.n = c.n;
    k.NP = c.NP;
    k.shared = c.shared;
    k.controlled = c.controlled;
    k.lowered = true;
    const double half_pi = 2.0 * std::atan(1.0);
    auto push = [&](int kind, int q0, int q1, int param, double angle) {
        k.gates.push_back(qng_gate{kind, q0, q1, param});
        k.fixed_angle.push_back(angle);
    };
    for (int pos = 0; pos < c.M; ++pos) {
        const qng_gate &g = c.gates[pos];
        const int r = c.rot_at[pos];
        if (g.kind != QNG_RPAULI) {
            if (r >= 0) {
                Rot rr = c.rots[r];
                rr.pos = (int)k.gates.size();
                k.rots.push_back(rr);
            }
            push(g.kind, g.q0, g.q1, g.param, 0.0);
            continue;
        }
        const Rot &rs = c.rots[r];
        const uint64_t supp = rs.flip | rs.zy;
        if (!supp) fail(QNG_E_DEVICE, "lower_strings: string without letters (internal)");
        int pivot = 0;
        while (!((supp >> pivot) & 1)) ++pivot;
        auto basis = [&](bool inverse) {
            for (int q = 0; q < c.n; ++q) {
                const bool x = (rs.flip >> q) & 1, z = (rs.zy >> q) & 1;
                if (x && !z) push(QNG_RY, q, -1, -1, inverse ? -half_pi : half_pi);   // X letter
                if (x && z) push(QNG_RX, q, -1, -1, inverse ? half_pi : -half_pi);   // Y letter
            }
        };
        basis(false);
        for (int q = 0; q < c.n; ++q)
            if (((supp >> q) & 1) && q != pivot) push(QNG_CNOT, q, pivot, -1, 0.0);
        Rot z{AX_Z, pivot, rs.param, (int)k.gates.size()};
        k.rots.push_back(z);
        push(QNG_RZ, pivot, -1, rs.param, 0.0);
        for (int q = c.n - 1; q >= 0; --q)
            if (((supp >> q) & 1) && q != pivot) push(QNG_CNOT, q, pivot, -1, 0.0);
        basis(true);
    }
    k.M = (int)k.gates.size();
    k.P = (int)k.rots.size();
    k.rot_at.assign(k.M, -1);
    for (int r = 0; r < k.P; ++r) k.rot_at[k.rots[r].pos] = r;
    if (k.P != c.P) fail(QNG_E_DEVICE, "lower_strings: rotation count changed (internal)");
    return k;
}

// R_sigma(theta) = cos(theta/2) I + i sin(theta/2) sigma.
Mat2 rotation(int axis, double theta) {
    const double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
    const cd I(0, 1);
    switch (axis) {
    case AX_X: return Mat2{c, I * s, I * s, c};
    case AX_Y: return Mat2{c, s, -s, c};          // i s * [[0,-i],[i,0]] = [[0, s], [-s, 0]]
    default:   return Mat2{cd(c, s), 0, 0, cd(c, -s)};
    }
}

Mat2 adjoint(const Mat2 &m) { return Mat2{std::conj(m.a), std::conj(m.c), std::conj(m.b), std::conj(m.d)}; }

Shear adjoint_shear(int axis, const Mat2 &adj) {
    double c = adj.a.real(), s;
    switch (axis) {
    case AX_X: s = -adj.b.imag(); break;   // adjoint b = -i sin
    case AX_Y: s = adj.b.real(); break;    // adjoint b = -sin
    default: s = -adj.a.imag(); break;     // adjoint a = cos - i sin
    }
    if (c < 0) {
        c = -c;
        s = -s;
    }
    return Shear{s / (1.0 + c), -s};
}

PlaneRot adjoint_plane(int axis, const Mat2 &adj) {
    double s;
    switch (axis) {
    case AX_X: s = -adj.b.imag(); break;
    case AX_Y: s = adj.b.real(); break;
    default: s = -adj.a.imag(); break;
    }
    return PlaneRot{adj.a.real(), s};
}

std::vector<PauliTerm> compile_hamiltonian(const qng_circuit *c, const qng_pauli_sum *h) {
    std::vector<PauliTerm> out(h->n_terms);
    for (int t = 0; t < h->n_terms; ++t) {
        PauliTerm &p = out[t];
        p.coeff = h->coeff[t];
        for (int q = 0; q < c->n_qubits; ++q) {
            const uint64_t bit = uint64_t(1) << q;
            switch (h->pauli[(size_t)t * c->n_qubits + q]) {
            case 1: p.flip |= bit; break;
            case 2: p.flip |= bit; p.zy |= bit; ++p.n_y; break;
            case 3: p.zy |= bit; break;
            default: break;
            }
        }
    }
    return out;
}

}  // namespace qng
