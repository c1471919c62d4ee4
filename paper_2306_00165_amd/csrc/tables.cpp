// Host-side table construction in extended precision (see tables.hpp).
//
// The Chebyshev-tau Helmholtz problem  [(s - c D^2) x]_n = f_n, n <= N-3,
// x(+1) = x(-1) = 0  is solved in the Dirichlet basis Z (columns T_{k+2} - T_k):
// with R = "first N-2 rows", x = Z q and (R Z)(s I - c E) q = f where
// E = (R Z)^{-1} R D^2 Z.  E has real, negative, distinct eigenvalues mu_k; with
// E = V diag(mu) V^{-1},
//     x = Pl diag(1/(s - c mu)) Pr f,   Pl = Z V,  Pr = V^{-1} (R Z)^{-1}.
// Both Pl and Pr are independent of the Fourier mode, so on the device each
// tau solve is two fixed contractions and a per-mode diagonal.  E and its
// eigen-decomposition are formed in long double; doing this in double loses
// about 1e-10 in the transposed solve, long double keeps it near 1e-13.
#include "tables.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace pcfv {
namespace {

typedef long double ld;

struct Mat {
    int r = 0, c = 0;
    std::vector<ld> a;
    Mat() {}
    Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0L) {}
    ld& operator()(int i, int j) { return a[(size_t)i * c + j]; }
    ld operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

Mat mul(const Mat& A, const Mat& B) {
    Mat C(A.r, B.c);
    for (int i = 0; i < A.r; ++i)
        for (int k = 0; k < A.c; ++k) {
            ld aik = A(i, k);
            if (aik == 0) continue;
            for (int j = 0; j < B.c; ++j) C(i, j) += aik * B(k, j);
        }
    return C;
}

Mat tr(const Mat& A) {
    Mat T(A.c, A.r);
    for (int i = 0; i < A.r; ++i)
        for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
    return T;
}

Mat eye(int n) {
    Mat I(n, n);
    for (int i = 0; i < n; ++i) I(i, i) = 1;
    return I;
}

// Gauss-Jordan inverse with partial pivoting.
bool inverse(const Mat& A, Mat& out) {
    int n = A.r;
    Mat M = A;
    out = eye(n);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (std::fabs(M(i, col)) > std::fabs(M(piv, col))) piv = i;
        if (M(piv, col) == 0) return false;
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(M(piv, j), M(col, j));
                std::swap(out(piv, j), out(col, j));
            }
        ld inv = 1.0L / M(col, col);
        for (int j = 0; j < n; ++j) {
            M(col, j) *= inv;
            out(col, j) *= inv;
        }
        for (int i = 0; i < n; ++i) {
            if (i == col) continue;
            ld f = M(i, col);
            if (f == 0) continue;
            for (int j = 0; j < n; ++j) {
                M(i, j) -= f * M(col, j);
                out(i, j) -= f * out(col, j);
            }
        }
    }
    return true;
}

// Solve A x = b by LU with partial pivoting (A copied).
std::vector<ld> solve(Mat A, std::vector<ld> b) {
    int n = A.r;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (std::fabs(A(i, col)) > std::fabs(A(piv, col))) piv = i;
        if (piv != col) {
            for (int j = 0; j < n; ++j) std::swap(A(piv, j), A(col, j));
            std::swap(b[piv], b[col]);
        }
        if (A(col, col) == 0) A(col, col) = 1e-300L;
        for (int i = col + 1; i < n; ++i) {
            ld f = A(i, col) / A(col, col);
            if (f == 0) continue;
            for (int j = col; j < n; ++j) A(i, j) -= f * A(col, j);
            b[i] -= f * b[col];
        }
    }
    std::vector<ld> x(n);
    for (int i = n - 1; i >= 0; --i) {
        ld s = b[i];
        for (int j = i + 1; j < n; ++j) s -= A(i, j) * x[j];
        x[i] = s / A(i, i);
    }
    return x;
}

// Eigenvalues of a real matrix whose eigenvalues are real: Householder
// reduction to Hessenberg form, then single-shift QR with Wilkinson shifts and
// deflation (textbook Francis QR without the double shift).
bool eig_real(Mat H, std::vector<ld>& ev) {
    int n = H.r;
    ev.assign(n, 0);
    for (int k = 0; k < n - 2; ++k) {
        ld alpha = 0;
        for (int i = k + 1; i < n; ++i) alpha += H(i, k) * H(i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0) continue;
        if (H(k + 1, k) > 0) alpha = -alpha;
        std::vector<ld> v(n, 0);
        v[k + 1] = H(k + 1, k) - alpha;
        for (int i = k + 2; i < n; ++i) v[i] = H(i, k);
        ld vn = 0;
        for (int i = k + 1; i < n; ++i) vn += v[i] * v[i];
        if (vn == 0) continue;
        for (int j = 0; j < n; ++j) {  // H = (I - 2vv^T/vn) H
            ld s = 0;
            for (int i = k + 1; i < n; ++i) s += v[i] * H(i, j);
            s = 2 * s / vn;
            for (int i = k + 1; i < n; ++i) H(i, j) -= s * v[i];
        }
        for (int i = 0; i < n; ++i) {  // H = H (I - 2vv^T/vn)
            ld s = 0;
            for (int j = k + 1; j < n; ++j) s += H(i, j) * v[j];
            s = 2 * s / vn;
            for (int j = k + 1; j < n; ++j) H(i, j) -= s * v[j];
        }
        for (int i = k + 2; i < n; ++i) H(i, k) = 0;
    }
    const ld eps = 4e-19L;
    int hi = n - 1, iter = 0, total = 0;
    std::vector<ld> cs(n), sn(n);
    while (hi >= 0) {
        if (hi == 0) {
            ev[0] = H(0, 0);
            break;
        }
        int l = hi;
        while (l > 0) {
            ld s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (std::fabs(H(l, l - 1)) <= eps * s) {
                H(l, l - 1) = 0;
                break;
            }
            --l;
        }
        if (l == hi) {
            ev[hi] = H(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 100000) return false;
        ++iter;
        ld a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
        ld mu = d;
        ld half = (a - d) / 2;
        ld disc = half * half + b * c;
        if (disc >= 0) {
            ld sq = std::sqrt(disc);
            ld m1 = (a + d) / 2 + sq, m2 = (a + d) / 2 - sq;
            mu = (std::fabs(m1 - d) < std::fabs(m2 - d)) ? m1 : m2;
        }
        if (iter % 12 == 11) mu = d + std::fabs(c);  // exceptional shift
        for (int k = l; k <= hi; ++k) H(k, k) -= mu;
        for (int k = l; k < hi; ++k) {  // QR by Givens on rows k, k+1
            ld x = H(k, k), y = H(k + 1, k);
            ld r = std::sqrt(x * x + y * y);
            ld cc = (r == 0) ? 1 : x / r, ss = (r == 0) ? 0 : y / r;
            cs[k] = cc;
            sn[k] = ss;
            for (int j = k; j <= hi; ++j) {
                ld t1 = H(k, j), t2 = H(k + 1, j);
                H(k, j) = cc * t1 + ss * t2;
                H(k + 1, j) = -ss * t1 + cc * t2;
            }
        }
        for (int k = l; k < hi; ++k) {  // R Q
            ld cc = cs[k], ss = sn[k];
            for (int i = l; i <= std::min(k + 1, hi); ++i) {
                ld t1 = H(i, k), t2 = H(i, k + 1);
                H(i, k) = cc * t1 + ss * t2;
                H(i, k + 1) = -ss * t1 + cc * t2;
            }
        }
        for (int k = l; k <= hi; ++k) H(k, k) += mu;
    }
    return true;
}

// Right eigenvector for a known eigenvalue by inverse iteration.
std::vector<ld> eigvec(const Mat& A, ld mu) {
    int n = A.r;
    Mat B = A;
    ld shift = mu * (1 + 1e-15L) + 1e-30L;
    for (int i = 0; i < n; ++i) B(i, i) -= shift;
    std::vector<ld> x(n);
    for (int i = 0; i < n; ++i) x[i] = 1.0L / (1 + i) + ((i % 3) ? 0.25L : -0.5L);
    for (int it = 0; it < 4; ++it) {
        x = solve(B, x);
        ld m = 0;
        for (int i = 0; i < n; ++i)
            if (std::fabs(x[i]) > std::fabs(m)) m = x[i];
        for (int i = 0; i < n; ++i) x[i] /= m;
    }
    return x;
}

bool cholesky(const Mat& A, Mat& L) {
    int n = A.r;
    L = Mat(n, n);
    for (int j = 0; j < n; ++j) {
        ld s = A(j, j);
        for (int k = 0; k < j; ++k) s -= L(j, k) * L(j, k);
        if (s <= 0) return false;
        L(j, j) = std::sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            ld t = A(i, j);
            for (int k = 0; k < j; ++k) t -= L(i, k) * L(j, k);
            L(i, j) = t / L(j, j);
        }
    }
    return true;
}

// Cyclic Jacobi for a symmetric matrix: A = Q diag(w) Q^T.
void jacobi(Mat A, std::vector<ld>& w, Mat& Q) {
    int n = A.r;
    Q = eye(n);
    for (int sweep = 0; sweep < 100; ++sweep) {
        ld off = 0, dia = 0;
        for (int i = 0; i < n; ++i) {
            dia += A(i, i) * A(i, i);
            for (int j = i + 1; j < n; ++j) off += A(i, j) * A(i, j);
        }
        if (off <= 1e-40L * dia) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                ld apq = A(p, q);
                if (apq == 0) continue;
                ld theta = (A(q, q) - A(p, p)) / (2 * apq);
                ld t = (theta >= 0 ? 1 : -1) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                ld c = 1 / std::sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < n; ++k) {
                    ld akp = A(k, p), akq = A(k, q);
                    A(k, p) = c * akp - s * akq;
                    A(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    ld apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk - s * aqk;
                    A(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    ld qkp = Q(k, p), qkq = Q(k, q);
                    Q(k, p) = c * qkp - s * qkq;
                    Q(k, q) = s * qkp + c * qkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A(i, i);
}

const ld PI = 3.141592653589793238462643383279502884L;

Mat cheb_D(int N) {
    Mat D(N, N);
    for (int n = 0; n < N; ++n)
        for (int p = n + 1; p < N; ++p)
            if ((p + n) % 2 == 1) D(n, p) = 2.0L * p / (n == 0 ? 2 : 1);
    return D;
}

ld cos_pi_frac(long long num, long long den) {  // cos(pi num/den), exact reduction
    long long m = num % (2 * den);
    if (m < 0) m += 2 * den;
    return std::cos(PI * (ld)m / (ld)den);
}

void store(std::vector<double>& mats, int N, int slot, const Mat& A) {
    double* s = mats.data() + (size_t)slot * N * N;
    for (int n = 0; n < A.r; ++n)
        for (int m = 0; m < A.c; ++m) s[(size_t)m * N + n] = (double)A(n, m);
}

}  // namespace

bool build_tables(double Lx, double Lz, double Re, int Nx, int Ny, int Nz, double dt,
                  Tables& t, std::string& err) {
    const int N = Ny;
    t.N = N;
    t.Nx = Nx;
    t.Nz = Nz;
    t.Kx = Nx / 3 - 1;
    t.Kz = Nz / 3 - 1;
    t.nkx = 2 * t.Kx + 1;
    t.nkz = t.Kz + 1;
    t.nmodes = t.nkx * t.nkz;
    const ld lam = 1.0L / (ld)dt, nu = 1.0L / (ld)Re;
    const ld alpha = 2 * PI / (ld)Lx, beta = 2 * PI / (ld)Lz;
    t.lam = (double)lam;
    t.nu = (double)nu;
    t.alpha = (double)alpha;
    t.beta = (double)beta;

    // -- Chebyshev operators ---------------------------------------------------
    Mat D = cheb_D(N), D2 = mul(D, D), C(N, N), Cinv(N, N), G(N, N), Ginv;
    for (int j = 0; j < N; ++j)
        for (int n = 0; n < N; ++n) C(j, n) = cos_pi_frac((long long)n * j, N - 1);
    // discrete cosine inverse on Gauss-Lobatto points
    for (int n = 0; n < N; ++n)
        for (int j = 0; j < N; ++j) {
            ld cn = (n == 0 || n == N - 1) ? 2 : 1, cj = (j == 0 || j == N - 1) ? 2 : 1;
            Cinv(n, j) = 2.0L / ((N - 1) * cn * cj) * cos_pi_frac((long long)n * j, N - 1);
        }
    for (int m = 0; m < N; ++m)
        for (int n = 0; n < N; ++n)
            if ((m + n) % 2 == 0) {
                ld s = m + n, d = m - n;
                G(m, n) = 1.0L / (1 - s * s) + 1.0L / (1 - d * d);
            }
    if (!inverse(G, Ginv)) {
        err = "Gram matrix inversion failed";
        return false;
    }

    // -- eigenbasis of the Dirichlet tau second derivative ----------------------
    const int M = N - 2;
    Mat Z(N, M);
    for (int k = 0; k < M; ++k) {
        Z(k, k) = -1;
        Z(k + 2, k) = 1;
    }
    Mat RZ(M, M), RD2Z(M, M);
    Mat D2Z = mul(D2, Z);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            RZ(i, j) = Z(i, j);
            RD2Z(i, j) = D2Z(i, j);
        }
    Mat RZinv;
    if (!inverse(RZ, RZinv)) {
        err = "R Z inversion failed";
        return false;
    }
    Mat E = mul(RZinv, RD2Z);
    std::vector<ld> mu(M);
    Mat V(M, M);
    ld eres = 0;
    for (int par = 0; par < 2; ++par) {  // even and odd Chebyshev parity decouple
        std::vector<int> idx;
        for (int k = par; k < M; k += 2) idx.push_back(k);
        int m = (int)idx.size();
        if (m == 0) continue;
        Mat Ep(m, m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Ep(i, j) = E(idx[i], idx[j]);
        std::vector<ld> ev;
        if (!eig_real(Ep, ev)) {
            err = "eigenvalue iteration did not converge";
            return false;
        }
        std::sort(ev.begin(), ev.end());
        for (int q = 0; q < m; ++q) {
            std::vector<ld> x = eigvec(Ep, ev[q]);
            int col = idx[q];  // keep parity blocks on their own columns
            mu[col] = ev[q];
            for (int i = 0; i < m; ++i) V(idx[i], col) = x[i];
            ld rn = 0, xn = 0;
            for (int i = 0; i < m; ++i) {
                ld s = -ev[q] * x[i];
                for (int j = 0; j < m; ++j) s += Ep(i, j) * x[j];
                rn = std::max(rn, std::fabs(s));
                xn = std::max(xn, std::fabs(x[i]));
            }
            eres = std::max(eres, rn / (std::fabs(ev[q]) * xn));
        }
    }
    t.eig_residual = (double)eres;
    t.mu.resize(M);
    for (int k = 0; k < M; ++k) t.mu[k] = (double)mu[k];
    Mat Vinv;
    if (!inverse(V, Vinv)) {
        err = "eigenvector matrix is singular";
        return false;
    }
    Mat Pl = mul(Z, V), Pr = mul(Vinv, RZinv);

    // -- W-orthogonal projection tables -------------------------------------------
    const int M4 = N - 4;
    Mat Z4(N, M4);
    for (int k = 0; k < M4; ++k) {  // T_k - 2(k+2)/(k+3) T_{k+2} + (k+1)/(k+3) T_{k+4}
        Z4(k, k) = 1;
        Z4(k + 2, k) = -2.0L * (k + 2) / (k + 3);
        Z4(k + 4, k) = (ld)(k + 1) / (k + 3);
    }
    Mat DZ4 = mul(D, Z4);
    Mat A4 = mul(tr(Z4), mul(G, Z4)), B4 = mul(tr(DZ4), mul(G, DZ4)), L4, L4inv;
    if (!cholesky(A4, L4) || !inverse(L4, L4inv)) {
        err = "clamped Gram matrix is not positive definite";
        return false;
    }
    std::vector<ld> Lam;
    Mat Q4;
    jacobi(mul(L4inv, mul(B4, tr(L4inv))), Lam, Q4);
    Mat X4 = mul(tr(L4inv), Q4);
    Mat PvL = mul(Z4, X4);
    Mat Z2tGZ2inv;
    if (!inverse(mul(tr(Z), mul(G, Z)), Z2tGZ2inv)) {
        err = "Dirichlet Gram matrix inversion failed";
        return false;
    }
    Mat PiD = mul(Z, mul(Z2tGZ2inv, mul(tr(Z), G)));

    // -- store fixed matrices ------------------------------------------------------
    t.mats.assign((size_t)M_COUNT * N * N, 0.0);
    Mat CD = mul(C, D);
    store(t.mats, N, M_C, C);
    store(t.mats, N, M_CD, CD);
    store(t.mats, N, M_CINV, Cinv);
    store(t.mats, N, M_CINVT, tr(Cinv));
    store(t.mats, N, M_D, D);
    store(t.mats, N, M_D2, D2);
    store(t.mats, N, M_DT, tr(D));
    store(t.mats, N, M_G, G);
    store(t.mats, N, M_GINV, Ginv);
    store(t.mats, N, M_PL, Pl);
    store(t.mats, N, M_PR, Pr);
    store(t.mats, N, M_PLT, tr(Pl));
    store(t.mats, N, M_PRT, tr(Pr));
    store(t.mats, N, M_MA, mul(Ginv, tr(C)));
    store(t.mats, N, M_MB, mul(Ginv, tr(CD)));
    store(t.mats, N, M_ML, mul(Ginv, mul(tr(D2), G)));
    store(t.mats, N, M_DTG, mul(tr(D), G));
    store(t.mats, N, M_PVL, PvL);
    store(t.mats, N, M_PVLT, tr(PvL));
    store(t.mats, N, M_PID, PiD);
    // compositions used by the fused contraction phases of the kernels
    Mat RD(M, N);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < N; ++j) RD(i, j) = D(i, j);
    Mat PRD = mul(Pr, RD), PRDPL = mul(PRD, Pl), DPL = mul(D, Pl);
    store(t.mats, N, M_PRD, PRD);
    store(t.mats, N, M_PRDT, tr(PRD));
    store(t.mats, N, M_PRDPL, PRDPL);
    store(t.mats, N, M_PRDPLT, tr(PRDPL));
    store(t.mats, N, M_DPL, DPL);
    store(t.mats, N, M_DPLT, tr(DPL));
    store(t.mats, N, M_DPVL, mul(D, PvL));

    // -- per-mode tables -------------------------------------------------------------
    const int nm = t.nmodes;
    t.minfo.assign((size_t)nm * MI_STRIDE, 0.0);
    t.dH.assign((size_t)nm * N, 0.0);
    t.dP.assign((size_t)nm * N, 0.0);
    t.dproj.assign((size_t)nm * N, 0.0);
    t.Vk.assign((size_t)nm * 4 * N, 0.0);
    t.DVk.assign((size_t)nm * 4 * N, 0.0);
    t.Ainv.assign((size_t)nm * 16, 0.0);
    t.indep.assign(nm, -1);
    int nind = 0;
    auto hsolve = [&](ld s, ld c, const std::vector<ld>& f) {  // f: N-2 tau rows
        std::vector<ld> q(M, 0), x(N, 0);
        for (int k = 0; k < M; ++k) {
            ld acc = 0;
            for (int i = 0; i < M; ++i) acc += Pr(k, i) * f[i];
            q[k] = acc / (s - c * mu[k]);
        }
        for (int n = 0; n < N; ++n) {
            ld acc = 0;
            for (int k = 0; k < M; ++k) acc += Pl(n, k) * q[k];
            x[n] = acc;
        }
        return x;
    };
    auto dvec = [&](const std::vector<ld>& x) {
        std::vector<ld> y(N, 0);
        for (int n = 0; n < N; ++n) {
            ld acc = 0;
            for (int p = 0; p < N; ++p) acc += D(n, p) * x[p];
            y[n] = acc;
        }
        return y;
    };
    for (int ikx = 0; ikx < t.nkx; ++ikx)
        for (int kz = 0; kz < t.nkz; ++kz) {
            const int m = ikx * t.nkz + kz;
            const int kx = (ikx <= t.Kx) ? ikx : ikx - t.nkx;
            const ld a = alpha * kx, b = beta * kz, k2 = a * a + b * b;
            const ld sig = lam + nu * k2;
            double* mi = t.minfo.data() + (size_t)m * MI_STRIDE;
            mi[MI_A] = (double)a;
            mi[MI_B] = (double)b;
            mi[MI_K2] = (double)k2;
            mi[MI_INVK2] = (k2 > 0) ? (double)(1.0L / k2) : 0.0;
            mi[MI_SIG] = (double)sig;
            mi[MI_WGT] = (kz == 0) ? 0.5 : 1.0;
            mi[MI_KX] = kx;
            mi[MI_KZ] = kz;
            if (kz > 0 || kx > 0) t.indep[m] = nind++;
            if (kx == 0 && kz == 0) t.indep[m] = 0;
            for (int k = 0; k < M; ++k) t.dH[(size_t)m * N + k] = (double)(1.0L / (sig - nu * mu[k]));
            if (k2 == 0) continue;
            for (int k = 0; k < M; ++k) t.dP[(size_t)m * N + k] = (double)(1.0L / (k2 - mu[k]));
            for (int k = 0; k < M4; ++k)
                t.dproj[(size_t)m * N + k] = (double)(1.0L / (1.0L + Lam[k] / k2));
            // homogeneous responses of the influence-matrix method:
            // k = 0,1: pressure Dirichlet data p(+1) = 1, p(-1) = 1;
            // k = 2,3: tau residuals of the v equation in rows N-2, N-1.
            std::vector<ld> P[4], Vv[4], DVv[4];
            for (int k = 0; k < 4; ++k) {
                std::vector<ld> f(M, 0), lift(N, 0);
                if (k < 2) {
                    lift[0] = 0.5L;
                    lift[1] = (k == 0) ? 0.5L : -0.5L;
                    for (int i = 0; i < M; ++i) f[i] = -k2 * lift[i];
                } else {
                    std::vector<ld> e(N, 0);
                    e[N - 2 + (k - 2)] = 1;
                    std::vector<ld> h = dvec(e);
                    for (int i = 0; i < M; ++i) f[i] = -h[i];
                }
                std::vector<ld> p = hsolve(k2, 1.0L, f);
                for (int n = 0; n < N; ++n) p[n] += lift[n];
                std::vector<ld> dp = dvec(p), g(M);
                for (int i = 0; i < M; ++i) g[i] = -dp[i];
                P[k] = p;
                Vv[k] = hsolve(sig, nu, g);
                DVv[k] = dvec(Vv[k]);
            }
            Mat A(4, 4), Ai;
            for (int k = 0; k < 4; ++k) {
                ld sp = 0, sm = 0;
                for (int n = 0; n < N; ++n) {
                    sp += DVv[k][n];
                    sm += (n % 2 ? -1 : 1) * DVv[k][n];
                }
                A(0, k) = sp;
                A(1, k) = sm;
                A(2, k) = sig * Vv[k][N - 2] + 2.0L * (N - 1) * P[k][N - 1] - (k == 2 ? 1 : 0);
                A(3, k) = sig * Vv[k][N - 1] - (k == 3 ? 1 : 0);
            }
            if (!inverse(A, Ai)) {
                err = "influence matrix is singular";
                return false;
            }
            for (int i = 0; i < 16; ++i) t.Ainv[(size_t)m * 16 + i] = (double)Ai.a[i];
            for (int k = 0; k < 4; ++k)
                for (int n = 0; n < N; ++n) {
                    t.Vk[((size_t)m * 4 + k) * N + n] = (double)Vv[k][n];
                    t.DVk[((size_t)m * 4 + k) * N + n] = (double)DVv[k][n];
                }
        }
    t.n_state = 4LL * (t.Kx + 2LL * t.Kx * t.Kz + t.Kz) * (N - 3) + 2LL * (N - 2);

    t.twx.resize(2 * Nx);
    t.twz.resize(2 * Nz);
    for (int k = 0; k < Nx; ++k) {
        t.twx[2 * k] = (double)cos_pi_frac(2LL * k, Nx);
        t.twx[2 * k + 1] = (double)std::sin(2 * PI * (ld)k / (ld)Nx);
    }
    for (int k = 0; k < Nz; ++k) {
        t.twz[2 * k] = (double)cos_pi_frac(2LL * k, Nz);
        t.twz[2 * k + 1] = (double)std::sin(2 * PI * (ld)k / (ld)Nz);
    }
    t.ygl.resize(N);
    for (int j = 0; j < N; ++j) t.ygl[j] = (double)cos_pi_frac(j, N - 1);
    return true;
}

}  // namespace pcfv
