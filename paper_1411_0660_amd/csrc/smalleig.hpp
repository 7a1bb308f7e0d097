// smalleig.hpp -- host linear algebra on the small projected matrices.
#pragma once

#include <cstdint>
#include <vector>

namespace mbl {

// A: m x m symmetric (column-major).  w: all eigenvalues ascending.  Y: m x
// sel.size() unit eigenvectors for the eigenvalues w[sel[j]].
void sym_eig_select(int m, const double *A, std::vector<double> &w, const std::vector<int> &sel,
                    std::vector<double> &Y);

// G = R^T R, R upper (column-major b x b).  Returns false if a pivot fell below
// rel_tiny * max diag (R is then completed with that floor).
bool cholesky_upper(int b, const double *G, std::vector<double> &R, double rel_tiny);
void upper_inverse(int b, const std::vector<double> &R, std::vector<double> &Ri);

}  // namespace mbl
