// Host FP64 dense linear algebra (basis construction).
#pragma once

#include <complex>
#include <vector>

namespace rbmf {

// Eigen-decomposition of an n x n complex Hermitian matrix A (row-major; the
// lower triangle is read).  w: eigenvalues in descending order; V: row-major
// n x n with column j the unit eigenvector of w[j].  Returns false if the QL
// iteration fails to converge.
bool herm_eig_desc(int n, const std::vector<std::complex<double>>& A, std::vector<double>& w,
                   std::vector<std::complex<double>>& V);

}  // namespace rbmf
