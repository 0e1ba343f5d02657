// Host numerics of the BOAC surrogate (Eqs. 7-8): RBF covariance, Cholesky factor, its inverse, the
// GP weights and the log marginal likelihood, in FP64. Matrices are row-major n x n.
#include <algorithm>
#include <cmath>
#include <vector>

#include "gp_host.h"

namespace boac {

void gp_covariance(const double *u, int n, int d, double length, double amp, double noise, double *K) {
    const double inv = 1.0 / (2.0 * length * length);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double d2 = 0.0;
            for (int t = 0; t < d; ++t) {
                const double e = u[(size_t)i * d + t] - u[(size_t)j * d + t];
                d2 += e * e;
            }
            const double k = amp * std::exp(-d2 * inv);
            K[(size_t)i * n + j] = k;
            K[(size_t)j * n + i] = k;
        }
        K[(size_t)i * n + i] += noise;
    }
}

// Dot product of two contiguous rows with 8 independent partial sums (vectorisable; fixed order).
static double dot(const double *a, const double *b, int len) {
    double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int k = 0;
    for (; k + 8 <= len; k += 8)
        for (int t = 0; t < 8; ++t) p[t] += a[k + t] * b[k + t];
    double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    for (; k < len; ++k) s += a[k] * b[k];
    return s;
}

bool gp_cholesky(double *A, int n) {
    // row by row: L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj, L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)
    for (int i = 0; i < n; ++i) {
        double *Li = A + (size_t)i * n;
        for (int j = 0; j < i; ++j) {
            const double *Lj = A + (size_t)j * n;
            Li[j] = (Li[j] - dot(Li, Lj, j)) / Lj[j];
        }
        const double dgn = Li[i] - dot(Li, Li, i);
        if (!(dgn > 0.0) || !std::isfinite(dgn)) return false;
        Li[i] = std::sqrt(dgn);
        for (int j = i + 1; j < n; ++j) Li[j] = 0.0;
    }
    return true;
}

void gp_tri_inverse(const double *L, double *X, int n) {
    // X = L^-1 (lower): row i of L X = I gives X_ij = -(sum_{j<=k<i} L_ik X_kj) / L_ii for j < i.
    // Column-oriented: for each row i, X_i. = (e_i - sum_{k<i} L_ik X_k.) / L_ii
    std::fill(X, X + (size_t)n * n, 0.0);
    std::vector<double> row(n);
    for (int i = 0; i < n; ++i) {
        const double *Li = L + (size_t)i * n;
        std::fill(row.begin(), row.begin() + i + 1, 0.0);
        row[i] = 1.0;
        for (int k = 0; k < i; ++k) {
            const double l = Li[k];
            if (l == 0.0) continue;
            const double *Xk = X + (size_t)k * n;
            for (int j = 0; j <= k; ++j) row[j] -= l * Xk[j];
        }
        double *Xi = X + (size_t)i * n;
        const double inv = 1.0 / Li[i];
        for (int j = 0; j <= i; ++j) Xi[j] = row[j] * inv;
    }
}

void gp_chol_solve(const double *L, const double *b, double *x, int n) {
    std::vector<double> w(n);
    for (int i = 0; i < n; ++i) w[i] = (b[i] - dot(L + (size_t)i * n, w.data(), i)) / L[(size_t)i * n + i];
    for (int i = n - 1; i >= 0; --i) {
        double s = w[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
}

void gp_standardise(const double *y, int n, double *m0, double *s) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) m += y[i];
    m /= n;
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += (y[i] - m) * (y[i] - m);
    const double sd = n > 1 ? std::sqrt(v / (n - 1)) : 0.0;
    *m0 = m;
    *s = sd > 0.0 ? sd : 1.0;
}

bool gp_fit_fixed(const double *u, const double *y, int n, int d, double length, double amp, double noise,
                  double *L, double *alpha, double *m0, double *s, double *lml) {
    gp_standardise(y, n, m0, s);
    std::vector<double> z(n);
    for (int i = 0; i < n; ++i) z[i] = (y[i] - *m0) / *s;
    gp_covariance(u, n, d, length, amp, noise, L);
    if (!gp_cholesky(L, n)) return false;
    gp_chol_solve(L, z.data(), alpha, n);
    double q = 0.0, logdet = 0.0;
    for (int i = 0; i < n; ++i) {
        q += z[i] * alpha[i];
        logdet += std::log(L[(size_t)i * n + i]);
    }
    *lml = -0.5 * q - logdet - 0.5 * n * std::log(2.0 * M_PI);
    return true;
}

}  // namespace boac
