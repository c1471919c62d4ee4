// DMD extrapolation (Sec. 6): the small dense algebra, on the host in
// extended precision, given the Gram matrix of the snapshot differences.
#pragma once
#include <string>
#include <vector>

namespace pcfv {

// Relative singular-value threshold that defines the numerical rank r* of the
// snapshot matrix.
constexpr double kDmdRankTol = 1e-7;

// Snapshots psi_1..psi_M (M >= 3) are represented by the Gram matrix
// Ge[i][j] = e_i . e_j (row-major, M x M) of E = [psi_1, psi_2 - psi_1, ..,
// psi_M - psi_{M-1}], which keeps the small variations of a converging
// window resolved.  Ge must be accurate well beyond double precision (the
// Cholesky factor inherits its error times cond(E)^2); the device Gram is
// accumulated in double-double.  For each rank r = 1..r*, coef[r-1] receives
// the M-1 real coefficients c with psi_s(r) = sum_k c_k psi_{k+2}
// (k = 0..M-2), the steady state Re(b_1 phi_1) of the rank-r exact DMD (mode
// with the smallest |ln lambda|), and omega[r-1] its |omega| =
// |ln lambda_1| / dtau.  Returns r* (0 if the window is degenerate); err gets
// a message on failure (return -1).
int dmd_candidates(const std::vector<long double>& Ge, int M, double dtau,
                   std::vector<std::vector<double>>& coef, std::vector<double>& omega,
                   std::string& err);

}  // namespace pcfv
