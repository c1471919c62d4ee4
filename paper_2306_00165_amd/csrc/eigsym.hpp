// Symmetric eigen-decomposition on the host (POD of snapshot windows).
#pragma once
#include <vector>

namespace pcfv {

// A: n x n symmetric, row-major; on success A holds the eigenvectors as
// columns (A[i * n + j] = component i of vector j) and w the eigenvalues,
// both in decreasing order of eigenvalue.  Returns false if the QR iteration
// does not converge.
bool eig_symmetric(int n, std::vector<double>& A, std::vector<double>& w);

}  // namespace pcfv
