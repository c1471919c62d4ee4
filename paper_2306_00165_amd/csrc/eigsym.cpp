// Symmetric eigen-decomposition on the host (for the POD Gram matrix), after
// Golub & Van Loan, Matrix Computations, Sec. 8.3: Householder
// tridiagonalisation T = Q^T A Q (Algorithm 8.3.1) with Q accumulated, then
// implicit symmetric QR steps with the Wilkinson shift (Algorithm 8.3.2) on
// the unreduced blocks of T, deflating negligible off-diagonals (Algorithm
// 8.3.3), the Givens rotations accumulated into Q.
#include "eigsym.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace pcfv {

bool eig_symmetric(int n, std::vector<double>& A, std::vector<double>& w) {
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    std::vector<double> Q((size_t)n * n, 0.0);
    auto q = [&](int i, int j) -> double& { return Q[(size_t)i * n + j]; };
    for (int i = 0; i < n; ++i) q(i, i) = 1.0;
    std::vector<double> v(n), p(n), wv(n);
    // 1. tridiagonalisation
    for (int k = 0; k + 2 < n; ++k) {
        double sigma = 0.0;
        for (int i = k + 2; i < n; ++i) sigma += a(i, k) * a(i, k);
        const double x0 = a(k + 1, k);
        if (sigma == 0.0) continue;   // column already reduced
        const double mu = std::sqrt(x0 * x0 + sigma);
        // v = x - alpha e1 with alpha = -sign(x0) |x| (no cancellation), v0 = 1
        const double alpha = (x0 >= 0.0) ? -mu : mu;
        const double v0 = x0 - alpha;
        v[k + 1] = 1.0;
        for (int i = k + 2; i < n; ++i) v[i] = a(i, k) / v0;
        double vv = 0.0;
        for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
        const double beta = 2.0 / vv;
        // p = beta A22 v, w = p - (beta p.v / 2) v, A22 -= v w^T + w v^T
        for (int i = k + 1; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
            p[i] = beta * s;
        }
        double pv = 0.0;
        for (int i = k + 1; i < n; ++i) pv += p[i] * v[i];
        for (int i = k + 1; i < n; ++i) wv[i] = p[i] - 0.5 * beta * pv * v[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) a(i, j) -= v[i] * wv[j] + wv[i] * v[j];
        a(k + 1, k) = a(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
        // Q <- Q H, H = I - beta v v^T acting on columns k+1..n-1
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int j = k + 1; j < n; ++j) s += q(i, j) * v[j];
            s *= beta;
            for (int j = k + 1; j < n; ++j) q(i, j) -= s * v[j];
        }
    }
    std::vector<double> d(n), e(n, 0.0);   // e[i] couples i and i + 1
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
    // 2. implicit QR with Wilkinson shifts
    const double eps = 2.2e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            --hi;
            continue;
        }
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
        if (++guard > 60 * n) return false;
        const double dl = 0.5 * (d[hi - 1] - d[hi]), b2 = e[hi - 1] * e[hi - 1];
        const double mu = d[hi] - b2 / (dl + (dl >= 0.0 ? 1.0 : -1.0) * std::sqrt(dl * dl + b2));
        double x = d[lo] - mu, z = e[lo];
        for (int k = lo; k < hi; ++k) {
            const double r = std::hypot(x, z);
            const double c = (r == 0.0) ? 1.0 : x / r, s = (r == 0.0) ? 0.0 : -z / r;
            if (k > lo) e[k - 1] = r;
            const double ak = d[k], bk = e[k], ck = d[k + 1];
            d[k] = c * c * ak - 2.0 * c * s * bk + s * s * ck;
            d[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ck;
            e[k] = c * s * (ak - ck) + (c * c - s * s) * bk;
            if (k + 1 < hi) {
                z = -s * e[k + 1];
                e[k + 1] *= c;
                x = e[k];
            }
            for (int i = 0; i < n; ++i) {
                const double qk = q(i, k), qk1 = q(i, k + 1);
                q(i, k) = c * qk - s * qk1;
                q(i, k + 1) = s * qk + c * qk1;
            }
        }
    }
    // 3. sort by decreasing eigenvalue
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] > d[y]; });
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; ++i) a(i, j) = q(i, idx[j]);
    }
    return true;
}

}  // namespace pcfv
