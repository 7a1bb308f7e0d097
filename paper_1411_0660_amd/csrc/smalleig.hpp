// smalleig.hpp -- host linear algebra on the small projected matrices.
#pragma once

#include <cstdint>
#include <vector>

namespace mbl {

// Householder tridiagonal form of a small symmetric matrix, kept between the
// eigenvalue and eigenvector stages.
struct SymEigWork {
    int m = 0;
    std::vector<double> a, d, e, tau;   // reflectors (in a), diagonal, off-diagonal
    double tmax = 0.0;                  // Gershgorin bound of |T|
};
// A: m x m symmetric (column-major).  w: all eigenvalues ascending (implicit
// QR with Wilkinson shifts on the tridiagonal form).
void sym_eig_values(int m, const double *A, SymEigWork &wk, std::vector<double> &w);
// Y: m x sel.size() unit eigenvectors for the eigenvalues w[sel[j]] (inverse
// iteration on the tridiagonal with Gram-Schmidt inside clusters, then
// back-transformation).
void sym_eig_vectors(const SymEigWork &wk, const std::vector<double> &w,
                     const std::vector<int> &sel, std::vector<double> &Y);
// both stages
void sym_eig_select(int m, const double *A, std::vector<double> &w, const std::vector<int> &sel,
                    std::vector<double> &Y);

// G = R^T R, R upper (column-major b x b).  Returns false if a pivot fell below
// rel_tiny * max diag (R is then completed with that floor).
bool cholesky_upper(int b, const double *G, std::vector<double> &R, double rel_tiny);
void upper_inverse(int b, const std::vector<double> &R, std::vector<double> &Ri);

}  // namespace mbl
