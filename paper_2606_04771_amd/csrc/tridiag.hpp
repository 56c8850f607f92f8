// Small dense helpers on the host: the exponential of the Lanczos
// tridiagonal matrix.
#pragma once

#include <complex>
#include <vector>

namespace tdvp {

// Eigen-decomposition of the real symmetric tridiagonal matrix with diagonal
// d[0..n) and off-diagonal e[0..n-1) by the implicit QL method with
// Wilkinson shifts.  On return d holds the eigenvalues and z (n x n,
// column-major, z[i + n k]) the orthonormal eigenvectors.  Returns false if
// an eigenvalue needs more than 60 sweeps.
bool tridiag_eig(std::vector<double>& d, std::vector<double> e, std::vector<double>& z, int n);

// y = nrm * exp(tau T) e_1 for the tridiagonal T (alpha, beta).
bool tridiag_expm_e1(const std::vector<double>& alpha, const std::vector<double>& beta,
                     std::complex<double> tau, double nrm, std::vector<std::complex<double>>& y);

}  // namespace tdvp
