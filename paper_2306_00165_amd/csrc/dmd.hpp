// DMD extrapolation (Sec. 6): the small dense algebra, on the host in
// extended precision, given the Gram matrix of the snapshot differences.
#pragma once
#include <string>
#include <vector>

namespace pcfv {

// Relative singular-value threshold that defines the numerical rank r* of the
// snapshot matrix.
constexpr double kDmdRankTol = 1e-7;

// One extrapolation candidate: psi_s = sum_k coef[k] psi_{k+2} (k = 0..M-2).
struct DmdCandidate {
    int rank;                  // DMD truncation rank r
    int kind;                  // 0: Re(b_1 phi_1), the mode of the snapshot DMD with the
                               //    smallest |omega| (Sec. 6.2);
                               // 1: the fixed point of the affine model fitted to the
                               //    snapshot differences d_k = psi_{k+1} - psi_k:
                               //    psi_M + Re sum_{|lambda_q| < 1} b_q phi_q lambda_q / (1 - lambda_q)
    std::vector<double> coef;  // M - 1 real coefficients over psi_2..psi_M
};

// Ranks at which a model with numerical rank r* is fitted: r*, r* - 1,
// r* - 2, r* - 4, r* - 8, ... (>= 1).  Sec. 6.2 picks the rank r <= r* of
// least cost and found it at r*; trying every rank costs O(M^5) host work
// and M residual evaluations per window.
bool dmd_rank_tried(int r, int rstar);

// Snapshots psi_1..psi_M (M >= 3) are represented by the Gram matrix
// Ge[i][j] = e_i . e_j (row-major, M x M) of E = [psi_1, psi_2 - psi_1, ..,
// psi_M - psi_{M-1}], which keeps the small variations of a converging
// window resolved.  Ge must be accurate well beyond double precision (the
// Cholesky factor inherits its error times cond(E)^2); the device Gram is
// accumulated in double-double.  out receives, for the tried ranks r (see
// dmd_rank_tried) in increasing order, the kind-0 candidate of the rank-r
// exact DMD of the snapshot pairs (r tried for r*, the numerical rank of
// [psi_1 .. psi_{M-1}]) and the kind-1 candidate of the rank-r exact DMD of
// the difference pairs (r tried for r*_d, the numerical rank of
// [d_1 .. d_{M-2}]), amplitudes fitted at the last snapshot / difference, in
// the order (rank, kind).  Returns r* (0 if the window is degenerate: then
// no candidate); err gets a message on failure (return -1).
int dmd_candidates(const std::vector<long double>& Ge, int M, double dtau, std::vector<DmdCandidate>& out,
                   std::string& err);

}  // namespace pcfv
