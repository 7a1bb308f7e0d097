// smalleig.cpp -- host linear algebra on the b x b blocks of the block Krylov
// method: Cholesky factor of a Gram matrix and the inverse of that factor
// (the Cholesky-QR orthonormalisation of each new block, GvL section 5.5.9).
#include "smalleig.hpp"

#include <algorithm>
#include <cmath>

namespace mbl {

bool cholesky_upper(int b, const double *G, std::vector<double> &R, double rel_tiny) {
    R.assign((size_t)b * b, 0.0);
    double dmax = 0.0;
    for (int i = 0; i < b; i++) dmax = std::max(dmax, G[(size_t)i * b + i]);
    bool ok = true;
    for (int j = 0; j < b; j++) {
        for (int i = 0; i <= j; i++) {
            double s = G[(size_t)j * b + i];
            for (int k = 0; k < i; k++) s -= R[(size_t)i * b + k] * R[(size_t)j * b + k];
            if (i == j) {
                if (s <= rel_tiny * dmax) { ok = false; s = std::max(s, rel_tiny * dmax + 1e-300); }
                R[(size_t)j * b + j] = std::sqrt(s);
            } else {
                R[(size_t)j * b + i] = s / R[(size_t)i * b + i];
            }
        }
    }
    return ok;
}

void upper_inverse(int b, const std::vector<double> &R, std::vector<double> &Ri) {
    Ri.assign((size_t)b * b, 0.0);
    for (int j = 0; j < b; j++) {
        Ri[(size_t)j * b + j] = 1.0 / R[(size_t)j * b + j];
        for (int i = j - 1; i >= 0; i--) {
            double s = 0.0;
            for (int k = i + 1; k <= j; k++) s += R[(size_t)k * b + i] * Ri[(size_t)j * b + k];
            Ri[(size_t)j * b + i] = -s / R[(size_t)i * b + i];
        }
    }
}

}  // namespace mbl
