// solve.cpp -- FP64 shifted Cholesky solve for the natural-gradient step.
//
// The step of Sec. 1 is g dtheta = -dt grad E with g = Re G.  G is positive
// semidefinite but may be singular (e.g. a rotation that only changes the
// global phase), so the library solves (Re G + eps I) x = b with a Tikhonov
// shift eps >= 0 and reports QNG_E_NOT_SPD when the shifted matrix has a
// non-positive pivot.
#include <cmath>
#include <vector>

#include "circuit.hpp"

namespace qng {

// G: 2*P*P doubles (complex, row-major); only Re G is used.
void solve_shifted(int P, const double *G, double eps, const double *b, double *x) {
    std::vector<double> Lm((size_t)P * P, 0.0);
    for (int i = 0; i < P; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = G[2 * ((size_t)i * P + j)] + (i == j ? eps : 0.0);
            for (int k = 0; k < j; ++k) s -= Lm[(size_t)i * P + k] * Lm[(size_t)j * P + k];
            if (i == j) {
                if (!(s > 0.0) || !std::isfinite(s))
                    fail(QNG_E_NOT_SPD, "Re G + eps I is not positive definite (pivot " + std::to_string(i) + ")");
                Lm[(size_t)i * P + i] = std::sqrt(s);
            } else {
                Lm[(size_t)i * P + j] = s / Lm[(size_t)j * P + j];
            }
        }
    }
    std::vector<double> y(P);
    for (int i = 0; i < P; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= Lm[(size_t)i * P + k] * y[k];
        y[i] = s / Lm[(size_t)i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < P; ++k) s -= Lm[(size_t)k * P + i] * x[k];
        x[i] = s / Lm[(size_t)i * P + i];
    }
}

}  // namespace qng
