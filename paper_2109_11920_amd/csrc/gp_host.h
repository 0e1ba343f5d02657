// Host FP64 numerics of the BOAC surrogate (Eqs. 7-8). Row-major n x n matrices.
#pragma once

namespace boac {

// K_ij = amp exp(-|u_i - u_j|^2 / (2 length^2)) + noise [i == j]; u is [n][d].
void gp_covariance(const double *u, int n, int d, double length, double amp, double noise, double *K);
// In-place lower Cholesky factor (upper triangle zeroed); false if A is not positive definite.
bool gp_cholesky(double *A, int n);
// X = L^-1 for lower-triangular L (X lower, upper triangle zero).
void gp_tri_inverse(const double *L, double *X, int n);
// x = (L L^T)^-1 b.
void gp_chol_solve(const double *L, const double *b, double *x, int n);
// Sample mean and standard deviation (ddof 1; 1 when it is 0 or n = 1).
void gp_standardise(const double *y, int n, double *m0, double *s);
// Standardise y, factor K, alpha = K^-1 z, log marginal likelihood; L and alpha are outputs.
bool gp_fit_fixed(const double *u, const double *y, int n, int d, double length, double amp, double noise,
                  double *L, double *alpha, double *m0, double *s, double *lml);

}  // namespace boac
