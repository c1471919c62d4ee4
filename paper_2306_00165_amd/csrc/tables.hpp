// Host-side construction of the constant tables used by the pcfv kernels.
//
// Everything here runs once per context, on the host, in x87 extended
// precision (long double, 64-bit mantissa), and is rounded to double only
// when stored.  The tables are:
//   * fixed Ny x Ny operators in the Chebyshev index (derivative, Gauss-
//     Lobatto synthesis and analysis, Gram matrix, their products), and the
//     eigen-decomposition of the Dirichlet Chebyshev-tau second derivative
//     that turns every tau Helmholtz/Poisson solve into two fixed contractions
//     and a per-mode diagonal;
//   * per-Fourier-mode data: wavenumbers, those diagonals, the homogeneous
//     solutions and inverted 4x4 influence matrix of the Stokes solve, and the
//     diagonal of the W-orthogonal projection.
#pragma once
#include <string>
#include <vector>

namespace pcfv {

// Index of each fixed matrix in the table block.  Every matrix A (nout x nin)
// is stored transposed in an Ny x Ny slot: slot[m * Ny + n] = A[n][m].
enum FixedMat {
    M_C = 0,   // Gauss-Lobatto synthesis  C[j][n] = T_n(y_j)
    M_CD,      // C D: point values of the y-derivative
    M_CINV,    // C^{-1}: point values -> coefficients
    M_CINVT,   // C^{-T}
    M_D,       // Chebyshev derivative on coefficients
    M_D2,      // D^2
    M_DT,      // D^T
    M_G,       // Gram matrix int T_m T_n dy
    M_GINV,    // G^{-1}
    M_PL,      // Ny x (Ny-2): Z V (eigenbasis of the tau second derivative)
    M_PR,      // (Ny-2) x (Ny-2): V^{-1} (R Z)^{-1}
    M_PLT,     // (Ny-2) x Ny
    M_PRT,     // (Ny-2) x (Ny-2)
    M_MA,      // G^{-1} C^T
    M_MB,      // G^{-1} (C D)^T
    M_ML,      // G^{-1} (D^2)^T G
    M_DTG,     // D^T G
    M_PVL,     // Ny x (Ny-4): clamped basis times the simultaneous eigenvectors X
    M_PVLT,    // (Ny-4) x Ny
    M_PID,     // G-orthogonal projector onto Dirichlet polynomials
    M_PRD,     // (Ny-2) x Ny: Pr R D
    M_PRDT,    // Ny x (Ny-2)
    M_PRDPL,   // (Ny-2) x (Ny-2): Pr R D Pl
    M_PRDPLT,  // (Ny-2) x (Ny-2)
    M_DPL,     // Ny x (Ny-2): D Pl
    M_DPLT,    // (Ny-2) x Ny
    M_DPVL,    // Ny x (Ny-4): D PvL
    M_COUNT
};

// Per-mode scalars, MI_STRIDE doubles per mode.
enum ModeInfo { MI_A = 0, MI_B, MI_K2, MI_INVK2, MI_SIG, MI_WGT, MI_KX, MI_KZ, MI_STRIDE };

struct Tables {
    int N = 0, Nx = 0, Nz = 0, Kx = 0, Kz = 0, nkx = 0, nkz = 0, nmodes = 0;
    double lam = 0, nu = 0, alpha = 0, beta = 0;
    std::vector<double> mats;      // M_COUNT * N * N
    std::vector<double> minfo;     // nmodes * MI_STRIDE
    std::vector<double> dH;        // nmodes * N : 1/(sigma - nu mu_k)
    std::vector<double> dP;        // nmodes * N : 1/(kappa^2 - mu_k)
    std::vector<double> dproj;     // nmodes * N : 1/(1 + Lambda_k/kappa^2)
    std::vector<double> Vk;        // nmodes * 4 * N : homogeneous v responses
    std::vector<double> DVk;       // nmodes * 4 * N : their y-derivatives
    std::vector<double> Ainv;      // nmodes * 16    : inverse influence matrix (row-major)
    std::vector<double> twx;       // 2 * Nx : exp(2 pi i k / Nx)
    std::vector<double> twz;       // 2 * Nz
    std::vector<double> ygl;       // N Gauss-Lobatto points
    std::vector<double> mu;        // N-2 eigenvalues of the tau second derivative
    std::vector<int> indep;        // nmodes: position among independent modes
                                   // (kz > 0 or kx > 0) in storage order, -1 otherwise;
                                   // 0 for the (0,0) mode
    long long n_state = 0;
    double eig_residual = 0;       // max relative eigen-residual (diagnostic)
};

// Builds all tables; returns false and sets err on failure.
bool build_tables(double Lx, double Lz, double Re, int Nx, int Ny, int Nz, double dt,
                  Tables& t, std::string& err);

}  // namespace pcfv
