"""Oracle: Gaussian-process surrogate, expected improvement and chaotic search of the BOAC outer loop
(FP64 NumPy/SciPy, test infrastructure only).

The method models the negative log-likelihood J(c) = -ln P of a candidate as a Gaussian process
(Eq. 7) with a radial-basis-function kernel (Eq. 8), and samples new candidates where the expected
improvement (Eqs. 9-10) is largest. Readings of the printed formulas:

  - Eq. (8) names the amplitude l and the length-scale sigma_0, the reverse of their roles in the
    formula; here k(u, u') = amp * exp(-|u - u'|^2 / (2 length^2)).
  - Eq. (10) as printed improves toward larger J; the method minimises J, so
    gamma = (J_best - mu(u) - xi) / sigma(u) and EI = sigma (gamma Phi(gamma) + phi(gamma)) (Eq. 9),
    0 where sigma = 0 and the improvement is not positive.
  - Model inputs u are the candidates mapped affinely onto the unit box [0, 1]^d of the search box;
    targets are standardised (mean m0, scale s: the sample standard deviation, 1 if it is 0); the
    kernel amplitude is 1 in standardised units; a fixed nugget `noise` is added to the diagonal;
    the length-scale is the one of a fixed geometric grid with the largest log marginal likelihood.
  - The paper's acquisition optimiser is a chaotic optimisation algorithm whose details it does not
    give; the reading is a two-stage chaotic search driven by the logistic map z <- 4 z (1 - z):
    a global stage that maps the chaotic sequence onto the whole box, then a local stage that maps it
    onto a box around the incumbent whose half-width shrinks geometrically.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import cho_solve, cholesky, solve_triangular
from scipy.stats import norm

LENGTH_GRID = np.geomspace(0.03, 3.0, 16)
NOISE = 1e-6


def rbf(U1: np.ndarray, U2: np.ndarray, amp: float, length: float) -> np.ndarray:
    """Eq. (8): amp * exp(-|u1 - u2|^2 / (2 length^2)) for every pair of rows."""
    d2 = np.sum((U1[:, None, :] - U2[None, :, :]) ** 2, axis=-1)
    return amp * np.exp(-d2 / (2.0 * length * length))


def to_unit(theta: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    return (np.asarray(theta, np.float64) - lo) / (hi - lo)


def from_unit(u: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    return lo + np.asarray(u, np.float64) * (hi - lo)


def standardise(y: np.ndarray):
    y = np.asarray(y, np.float64)
    m0 = float(np.mean(y))
    s = float(np.std(y, ddof=1)) if y.size > 1 else 0.0
    return m0, (s if s > 0 else 1.0)


class GP:
    """GP posterior of Eq. (7) for standardised targets z = (y - m0) / s at unit-box inputs U."""

    def __init__(self, U, y, length, amp=1.0, noise=NOISE):
        self.U = np.asarray(U, np.float64)
        self.y = np.asarray(y, np.float64)
        self.m0, self.s = standardise(self.y)
        self.z = (self.y - self.m0) / self.s
        self.length, self.amp, self.noise = float(length), float(amp), float(noise)
        K = rbf(self.U, self.U, self.amp, self.length) + self.noise * np.eye(len(self.U))
        self.L = cholesky(K, lower=True)
        self.alpha = cho_solve((self.L, True), self.z)

    def log_marginal_likelihood(self) -> float:
        n = len(self.z)
        return float(-0.5 * self.z @ self.alpha - np.sum(np.log(np.diag(self.L))) - 0.5 * n * math.log(2 * math.pi))

    def predict(self, Q):
        """Posterior mean and standard deviation of y (not z) at unit-box queries Q."""
        Ks = rbf(np.asarray(Q, np.float64), self.U, self.amp, self.length)
        mu_z = Ks @ self.alpha
        v = solve_triangular(self.L, Ks.T, lower=True)
        var_z = np.maximum(self.amp - np.sum(v * v, axis=0), 0.0)
        return self.m0 + self.s * mu_z, self.s * np.sqrt(var_z)


def fit_gp(U, y, grid=LENGTH_GRID, noise=NOISE, n_select=None) -> GP:
    """GP on every observation with the grid length-scale of largest log marginal likelihood (first one
    on ties). With n_select < n the likelihood is evaluated on the n_select observations of smallest y
    only (ties by index), a cheaper model selection for long runs."""
    U = np.asarray(U, np.float64)
    y = np.asarray(y, np.float64)
    idx = np.arange(len(y))
    if n_select is not None and 0 < n_select < len(y):
        idx = np.argsort(y, kind="stable")[:n_select]
    best = None
    for length in grid:
        lml = GP(U[idx], y[idx], length, 1.0, noise).log_marginal_likelihood()
        if best is None or lml > best[0]:
            best = (lml, length)
    return GP(U, y, best[1], 1.0, noise)


def expected_improvement(mu, sigma, best: float, xi: float):
    """Eqs. (9)-(10) for minimisation."""
    mu = np.asarray(mu, np.float64)
    sigma = np.asarray(sigma, np.float64)
    imp = best - mu - xi
    out = np.maximum(imp, 0.0)
    pos = sigma > 0
    g = imp[pos] / sigma[pos]
    out[pos] = sigma[pos] * (g * norm.cdf(g) + norm.pdf(g))
    return out


def logistic_map(z0, steps: int) -> np.ndarray:
    """z_{t+1} = 4 z_t (1 - z_t), t = 0..steps-1, for every entry of z0: array [steps + 1, ...]."""
    z = np.asarray(z0, np.float64).copy()
    out = [z.copy()]
    for _ in range(steps):
        z = 4.0 * z * (1.0 - z)
        out.append(z.copy())
    return np.stack(out)


def chaotic_search(fun, z0: np.ndarray, n_global: int, n_local: int, shrink: float = 0.9,
                   radius0: float = 0.25):
    """Maximise fun over [0, 1]^d. z0 [P, d] chaotic seeds in (0, 1) (P parallel chains).

    Global stage: n_global steps, every chain's point u = z. Local stage: n_local steps around the
    incumbent u*, u = clip(u* + r (2 z - 1), 0, 1) with r = radius0 shrink^t. Returns (u*, f*)."""
    z = np.asarray(z0, np.float64).copy()
    best_u, best_f = None, -np.inf

    def consider(U):
        nonlocal best_u, best_f
        f = fun(U)
        i = int(np.argmax(f))
        if f[i] > best_f:
            best_u, best_f = U[i].copy(), float(f[i])

    for _ in range(n_global):
        consider(z)
        z = 4.0 * z * (1.0 - z)
    r = radius0
    for _ in range(n_local):
        consider(np.clip(best_u[None, :] + r * (2.0 * z - 1.0), 0.0, 1.0))
        z = 4.0 * z * (1.0 - z)
        r *= shrink
    return best_u, best_f
