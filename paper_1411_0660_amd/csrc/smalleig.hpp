// smalleig.hpp -- host linear algebra on the small b x b blocks of the block
// Krylov method.  (The projected matrices' eigenproblems run on the device:
// launch_jacobi_eig in kernels.hpp.)
#pragma once

#include <cstdint>
#include <vector>

namespace mbl {

// G = R^T R, R upper (column-major b x b).  Returns false if a pivot fell below
// rel_tiny * max diag (R is then completed with that floor).
bool cholesky_upper(int b, const double *G, std::vector<double> &R, double rel_tiny);
void upper_inverse(int b, const std::vector<double> &R, std::vector<double> &Ri);

}  // namespace mbl
