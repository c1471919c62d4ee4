// DMD extrapolation: host algebra in extended precision (see dmd.hpp).
//
// With E = [psi_1, psi_2 - psi_1, ...] and its Gram matrix Ge = R^T R
// (Cholesky), E = Q R for some Q with orthonormal columns, so every snapshot
// matrix is Q times a small matrix: X = [psi_1 .. psi_{M-1}] = Q R T_X,
// Y = [psi_2 .. psi_M] = Q R T_Y, psi_M = Q R 1 (T_X, T_Y: the first and last
// M-1 columns of the all-ones upper-triangular matrix).  Exact DMD (Sec. 6.1)
// then needs only M x M algebra:
//   R T_X = U Sigma V^T (one-sided Jacobi SVD), A~ = U^T R T_Y V Sigma^{-1},
//   A~ W = W Lambda (complex Schur by shifted QR), phi = Q (R T_Y V Sigma^{-1} W),
//   b = least squares of phi b = psi_M (complex Householder QR),
//   psi_s = Re(b_1 phi_1) = Y Re(V Sigma^{-1} w_1 b_1).
#include "dmd.hpp"

#include <algorithm>
#include <cmath>
#include <complex>

namespace pcfv {
namespace {

typedef long double ld;
typedef std::complex<ld> cld;

struct RM {  // real row-major matrix
    int r = 0, c = 0;
    std::vector<ld> a;
    RM() {}
    RM(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0L) {}
    ld& operator()(int i, int j) { return a[(size_t)i * c + j]; }
    ld operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

struct CM {  // complex row-major matrix
    int r = 0, c = 0;
    std::vector<cld> a;
    CM() {}
    CM(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, cld(0)) {}
    cld& operator()(int i, int j) { return a[(size_t)i * c + j]; }
    cld operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

// Upper Cholesky factor of a symmetric positive semi-definite matrix; rows of
// numerically zero pivots are left zero.
RM cholesky_upper(const RM& G) {
    const int n = G.r;
    RM R(n, n);
    ld maxd = 0;
    for (int i = 0; i < n; ++i) maxd = std::max(maxd, std::fabs(G(i, i)));
    for (int i = 0; i < n; ++i) {
        ld d = G(i, i);
        for (int k = 0; k < i; ++k) d -= R(k, i) * R(k, i);
        if (d <= 1e-30L * maxd) continue;
        const ld rii = std::sqrt(d);
        R(i, i) = rii;
        for (int j = i + 1; j < n; ++j) {
            ld s = G(i, j);
            for (int k = 0; k < i; ++k) s -= R(k, i) * R(k, j);
            R(i, j) = s / rii;
        }
    }
    return R;
}

// One-sided Jacobi SVD of A (m x n, m >= n): A = U diag(s) V^T, s descending.
void svd_jacobi(RM A, RM& U, std::vector<ld>& s, RM& V) {
    const int m = A.r, n = A.c;
    V = RM(n, n);
    for (int i = 0; i < n; ++i) V(i, i) = 1;
    for (int sweep = 0; sweep < 80; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                ld al = 0, be = 0, ga = 0;
                for (int i = 0; i < m; ++i) {
                    al += A(i, p) * A(i, p);
                    be += A(i, q) * A(i, q);
                    ga += A(i, p) * A(i, q);
                }
                if (ga == 0 || std::fabs(ga) <= 1e-19L * std::sqrt(al * be)) continue;
                rotated = true;
                const ld zeta = (be - al) / (2 * ga);
                const ld t = (zeta >= 0 ? 1 : -1) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
                const ld c = 1 / std::sqrt(1 + t * t), sn = c * t;
                for (int i = 0; i < m; ++i) {
                    const ld x = A(i, p), y = A(i, q);
                    A(i, p) = c * x - sn * y;
                    A(i, q) = sn * x + c * y;
                }
                for (int i = 0; i < n; ++i) {
                    const ld x = V(i, p), y = V(i, q);
                    V(i, p) = c * x - sn * y;
                    V(i, q) = sn * x + c * y;
                }
            }
        if (!rotated) break;
    }
    std::vector<int> order(n);
    std::vector<ld> norms(n);
    for (int j = 0; j < n; ++j) {
        ld t = 0;
        for (int i = 0; i < m; ++i) t += A(i, j) * A(i, j);
        norms[j] = std::sqrt(t);
        order[j] = j;
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) { return norms[a] > norms[b]; });
    U = RM(m, n);
    RM Vs(n, n);
    s.assign(n, 0);
    for (int jj = 0; jj < n; ++jj) {
        const int j = order[jj];
        s[jj] = norms[j];
        for (int i = 0; i < m; ++i) U(i, jj) = norms[j] > 0 ? A(i, j) / norms[j] : 0;
        for (int i = 0; i < n; ++i) Vs(i, jj) = V(i, j);
    }
    V = Vs;
}

// Eigen-decomposition of a general real matrix: Hessenberg reduction, complex
// single-shift QR (Wilkinson shifts) to the Schur form A = Z T Z^H, then
// eigenvectors by back substitution.  Returns false if QR does not converge.
bool eig_general(const RM& A, std::vector<cld>& lam, CM& W) {
    const int n = A.r;
    CM H(n, n), Z(n, n);
    for (int i = 0; i < n; ++i) {
        Z(i, i) = 1;
        for (int j = 0; j < n; ++j) H(i, j) = A(i, j);
    }
    // Householder reduction to upper Hessenberg form, accumulating Z.
    for (int k = 0; k < n - 2; ++k) {
        ld alpha2 = 0;
        for (int i = k + 1; i < n; ++i) alpha2 += std::norm(H(i, k));
        const ld alpha = std::sqrt(alpha2);
        if (alpha == 0) continue;
        const cld x0 = H(k + 1, k);
        const cld ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cld(1);
        std::vector<cld> v(n, cld(0));
        v[k + 1] = x0 + ph * alpha;
        for (int i = k + 2; i < n; ++i) v[i] = H(i, k);
        ld vn = 0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        if (vn == 0) continue;
        for (int j = 0; j < n; ++j) {  // H = (I - 2 v v^H / vn) H
            cld s = 0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * H(i, j);
            s *= 2.0L / vn;
            for (int i = k + 1; i < n; ++i) H(i, j) -= s * v[i];
        }
        for (int i = 0; i < n; ++i) {  // H = H (I - 2 v v^H / vn), Z likewise
            cld s = 0, t = 0;
            for (int j = k + 1; j < n; ++j) {
                s += H(i, j) * v[j];
                t += Z(i, j) * v[j];
            }
            s *= 2.0L / vn;
            t *= 2.0L / vn;
            for (int j = k + 1; j < n; ++j) {
                H(i, j) -= s * std::conj(v[j]);
                Z(i, j) -= t * std::conj(v[j]);
            }
        }
        for (int i = k + 2; i < n; ++i) H(i, k) = 0;
    }
    const ld eps = 4e-19L;
    int hi = n - 1, iter = 0, total = 0;
    std::vector<ld> cs(n);
    std::vector<cld> sn(n);
    while (hi > 0) {
        int l = hi;
        while (l > 0) {
            const ld s = std::abs(H(l - 1, l - 1)) + std::abs(H(l, l));
            if (std::abs(H(l, l - 1)) <= eps * (s > 0 ? s : 1)) {
                H(l, l - 1) = 0;
                break;
            }
            --l;
        }
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 20000) return false;
        ++iter;
        const cld a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
        const cld tr = a + d, det = a * d - b * c;
        const cld disc = std::sqrt(tr * tr / 4.0L - det);
        const cld m1 = tr / 2.0L + disc, m2 = tr / 2.0L - disc;
        cld mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
        if (iter % 10 == 9) mu = d + std::abs(c) * cld(0.75L, 0.5L);  // exceptional shift
        for (int k = l; k <= hi; ++k) H(k, k) -= mu;
        for (int k = l; k < hi; ++k) {  // Givens QR of the active block
            const cld x = H(k, k), y = H(k + 1, k);
            const ld r = std::sqrt(std::norm(x) + std::norm(y));
            ld cc;
            cld ss;
            if (r == 0) {
                cc = 1;
                ss = 0;
            } else if (std::abs(x) == 0) {
                cc = 0;
                ss = std::conj(y) / std::abs(y);
            } else {
                cc = std::abs(x) / r;
                ss = (x / std::abs(x)) * std::conj(y) / r;
            }
            cs[k] = cc;
            sn[k] = ss;
            for (int j = k; j < n; ++j) {
                const cld t1 = H(k, j), t2 = H(k + 1, j);
                H(k, j) = cc * t1 + ss * t2;
                H(k + 1, j) = -std::conj(ss) * t1 + cc * t2;
            }
        }
        for (int k = l; k < hi; ++k) {  // R Q, and accumulate Z
            const ld cc = cs[k];
            const cld ss = sn[k];
            for (int i = 0; i <= std::min(k + 1, hi); ++i) {
                const cld t1 = H(i, k), t2 = H(i, k + 1);
                H(i, k) = cc * t1 + std::conj(ss) * t2;
                H(i, k + 1) = -ss * t1 + cc * t2;
            }
            for (int i = 0; i < n; ++i) {
                const cld t1 = Z(i, k), t2 = Z(i, k + 1);
                Z(i, k) = cc * t1 + std::conj(ss) * t2;
                Z(i, k + 1) = -ss * t1 + cc * t2;
            }
        }
        for (int k = l; k <= hi; ++k) H(k, k) += mu;
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = H(i, i);
    // eigenvectors of the triangular T by back substitution, then W = Z X
    CM X(n, n);
    ld tnorm = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) tnorm = std::max(tnorm, std::abs(H(i, j)));
    for (int k = 0; k < n; ++k) {
        X(k, k) = 1;
        for (int i = k - 1; i >= 0; --i) {
            cld s = 0;
            for (int j = i + 1; j <= k; ++j) s += H(i, j) * X(j, k);
            cld dnm = H(i, i) - H(k, k);
            if (std::abs(dnm) < 1e-18L * tnorm) dnm = cld(1e-18L * tnorm, 0);
            X(i, k) = -s / dnm;
        }
    }
    W = CM(n, n);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            cld s = 0;
            for (int j = 0; j <= k; ++j) s += Z(i, j) * X(j, k);
            W(i, k) = s;
        }
    for (int k = 0; k < n; ++k) {  // unit columns
        ld nr = 0;
        for (int i = 0; i < n; ++i) nr += std::norm(W(i, k));
        nr = std::sqrt(nr);
        if (nr > 0)
            for (int i = 0; i < n; ++i) W(i, k) /= nr;
    }
    return true;
}

// Least squares min |P b - z| (P: m x r complex, m >= r) by Householder QR.
std::vector<cld> lstsq(CM P, std::vector<cld> z) {
    const int m = P.r, r = P.c;
    for (int k = 0; k < r; ++k) {
        ld alpha2 = 0;
        for (int i = k; i < m; ++i) alpha2 += std::norm(P(i, k));
        const ld alpha = std::sqrt(alpha2);
        if (alpha == 0) continue;
        const cld x0 = P(k, k);
        const cld ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cld(1);
        std::vector<cld> v(m, cld(0));
        v[k] = x0 + ph * alpha;
        for (int i = k + 1; i < m; ++i) v[i] = P(i, k);
        ld vn = 0;
        for (int i = k; i < m; ++i) vn += std::norm(v[i]);
        for (int j = k; j < r; ++j) {
            cld s = 0;
            for (int i = k; i < m; ++i) s += std::conj(v[i]) * P(i, j);
            s *= 2.0L / vn;
            for (int i = k; i < m; ++i) P(i, j) -= s * v[i];
        }
        cld s = 0;
        for (int i = k; i < m; ++i) s += std::conj(v[i]) * z[i];
        s *= 2.0L / vn;
        for (int i = k; i < m; ++i) z[i] -= s * v[i];
    }
    std::vector<cld> b(r, cld(0));
    for (int i = r - 1; i >= 0; --i) {
        cld s = z[i];
        for (int j = i + 1; j < r; ++j) s -= P(i, j) * b[j];
        b[i] = (std::abs(P(i, i)) > 0) ? s / P(i, i) : cld(0);
    }
    return b;
}

}  // namespace

namespace {

// Exact DMD of pairs (x_k, y_k) given in the orthonormal basis Q of the
// snapshot span: AX, AY (M x n) hold their Q-coordinates and AX = U S V^T;
// z holds those of the vector the amplitudes are fitted to.  The projections
// B = AY V S^{-1} and A~ = U^T B are formed once for the largest rank; the
// rank-r model uses their leading r columns (and r x r block).
struct DmdBasis {
    RM B, At;
};
DmdBasis dmd_basis(const RM& AY, const RM& U, const std::vector<ld>& s, const RM& V, int rmax) {
    const int M = AY.r, n = AY.c;
    DmdBasis d;
    d.B = RM(M, rmax);
    d.At = RM(rmax, rmax);
    for (int i = 0; i < M; ++i)
        for (int q = 0; q < rmax; ++q) {
            ld acc = 0;
            for (int k = 0; k < n; ++k) acc += AY(i, k) * V(k, q);
            d.B(i, q) = acc / s[q];
        }
    for (int p = 0; p < rmax; ++p)
        for (int q = 0; q < rmax; ++q) {
            ld acc = 0;
            for (int i = 0; i < M; ++i) acc += U(i, p) * d.B(i, q);
            d.At(p, q) = acc;
        }
    return d;
}

// The rank-r model: eigenvalues lam and, in wy (n x r), the coordinates over
// the y columns of every mode's amplitude times its eigenvector:
// sum_k wy(k, q) y_k = b_q phi_q.
struct DmdFit {
    std::vector<cld> lam;
    CM wy;
};
bool dmd_fit(const DmdBasis& d, const std::vector<ld>& z, const std::vector<ld>& s, const RM& V, int r, DmdFit& f,
             std::string& err) {
    const int M = d.B.r, n = V.r;
    RM At(r, r);
    for (int p = 0; p < r; ++p)
        for (int q = 0; q < r; ++q) At(p, q) = d.At(p, q);
    CM W;
    if (!eig_general(At, f.lam, W)) {
        err = "DMD eigenvalue iteration did not converge";
        return false;
    }
    CM P(M, r);  // phi = Q P
    for (int i = 0; i < M; ++i)
        for (int q = 0; q < r; ++q) {
            cld acc = 0;
            for (int p = 0; p < r; ++p) acc += d.B(i, p) * W(p, q);
            P(i, q) = acc;
        }
    std::vector<cld> zc(M);
    for (int i = 0; i < M; ++i) zc[i] = z[i];
    const std::vector<cld> b = lstsq(P, zc);
    f.wy = CM(n, r);   // phi_q = Y V_r Sigma_r^{-1} w_q
    for (int k = 0; k < n; ++k)
        for (int q = 0; q < r; ++q) {
            cld acc = 0;
            for (int p = 0; p < r; ++p) acc += V(k, p) / s[p] * W(p, q);
            f.wy(k, q) = acc * b[q];
        }
    return true;
}

}  // namespace

bool dmd_rank_tried(int r, int rstar) {
    if (r < 1 || r > rstar) return false;
    const int d = rstar - r;
    return d <= 2 || (d & (d - 1)) == 0;   // r*, r* - 1, r* - 2, r* - 4, r* - 8, ...
}

namespace {

int numerical_rank(const std::vector<ld>& s) {
    if (s.empty() || !(s[0] > 0)) return 0;
    int r = 0;
    while (r < (int)s.size() && s[r] > (ld)kDmdRankTol * s[0]) ++r;
    return r;
}

// Candidates from the Cholesky factor R of the Gram matrix (E = Q R), as
// coefficients over psi_2 .. psi_M (M - 1 each); see dmd.hpp.
int candidates_from_R(const RM& R, int M, double dtau, std::vector<DmdCandidate>& out, std::string& err) {
    (void)dtau;   // the candidates depend on the eigenvalues only through lambda
    const int n = M - 1;
    // (R T)[i][k] = sum_{j <= k} R[i][j]: Q-coordinates of psi_{k+1}
    RM RT(M, M);
    for (int i = 0; i < M; ++i) {
        ld acc = 0;
        for (int k = 0; k < M; ++k) {
            acc += R(i, k);
            RT(i, k) = acc;
        }
    }
    // kind 0: snapshot pairs (psi_k, psi_{k+1}), amplitudes at psi_M
    RM AX(M, n), AY(M, n);
    std::vector<ld> z(M);
    for (int i = 0; i < M; ++i) {
        for (int k = 0; k < n; ++k) {
            AX(i, k) = RT(i, k);
            AY(i, k) = RT(i, k + 1);
        }
        z[i] = RT(i, M - 1);
    }
    RM U, V;
    std::vector<ld> s;
    svd_jacobi(AX, U, s, V);
    const int rstar = numerical_rank(s);
    // kind 1: difference pairs (d_k, d_{k+1}), d_k = psi_{k+1} - psi_k = Q R e_{k+1},
    // amplitudes at the last difference
    const int nd = M - 2;
    RM DX(M, nd), DY(M, nd), Ud, Vd;
    std::vector<ld> zd(M), sd;
    for (int i = 0; i < M; ++i) {
        for (int k = 0; k < nd; ++k) {
            DX(i, k) = R(i, k + 1);
            DY(i, k) = R(i, k + 2);
        }
        zd[i] = R(i, M - 1);
    }
    svd_jacobi(DX, Ud, sd, Vd);
    const int rstar_d = (rstar > 0) ? numerical_rank(sd) : 0;
    const DmdBasis bs = dmd_basis(AY, U, s, V, rstar), bd = dmd_basis(DY, Ud, sd, Vd, rstar_d);
    for (int r = 1; r <= std::max(rstar, rstar_d); ++r) {
        if (!dmd_rank_tried(r, rstar) && !dmd_rank_tried(r, rstar_d)) continue;
        if (r <= rstar && dmd_rank_tried(r, rstar)) {   // Re(b_1 phi_1), the mode with the smallest |ln lambda|
            DmdFit f;
            if (!dmd_fit(bs, z, s, V, r, f, err)) return -1;
            int q1 = 0;
            for (int q = 1; q < r; ++q)
                if (std::abs(std::log(f.lam[q])) < std::abs(std::log(f.lam[q1]))) q1 = q;
            DmdCandidate c{r, 0, std::vector<double>(n)};
            for (int k = 0; k < n; ++k) c.coef[k] = (double)std::real(f.wy(k, q1));   // y_k = psi_{k+2}
            out.push_back(std::move(c));
        }
        if (r <= rstar_d && dmd_rank_tried(r, rstar_d)) {   // psi_M + Re sum_{|lambda|<1} b_q phi_q lambda_q / (1 - lambda_q)
            DmdFit f;
            if (!dmd_fit(bd, zd, sd, Vd, r, f, err)) return -1;
            std::vector<ld> cy(nd, 0);   // over y_k = d_{k+2} = psi_{k+3} - psi_{k+2}
            for (int q = 0; q < r; ++q) {
                if (!(std::abs(f.lam[q]) < 1)) continue;
                const cld g = f.lam[q] / (cld(1) - f.lam[q]);
                for (int k = 0; k < nd; ++k) cy[k] += std::real(f.wy(k, q) * g);
            }
            DmdCandidate c{r, 1, std::vector<double>(n, 0.0)};
            std::vector<ld> cp(n, 0);   // over psi_{j+2}, j = 0..n-1
            for (int k = 0; k < nd; ++k) {
                cp[k + 1] += cy[k];
                cp[k] -= cy[k];
            }
            cp[n - 1] += 1;   // psi_M
            for (int k = 0; k < n; ++k) c.coef[k] = (double)cp[k];
            out.push_back(std::move(c));
        }
    }
    return rstar;
}

}  // namespace

int dmd_candidates(const std::vector<long double>& Ge, int M, double dtau, std::vector<DmdCandidate>& out,
                   std::string& err) {
    out.clear();
    if (M < 3 || (int)Ge.size() != M * M || !(dtau > 0)) {
        err = "DMD needs at least 3 snapshots and dtau > 0";
        return -1;
    }
    RM G(M, M);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) G(i, j) = 0.5L * (Ge[(size_t)i * M + j] + Ge[(size_t)j * M + i]);
    return candidates_from_R(cholesky_upper(G), M, dtau, out, err);
}

}  // namespace pcfv
