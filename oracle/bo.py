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
    give, and it proposes one candidate per cycle. The reading (the one the library's outer loop runs):
    P chains z in (0, 1)^d follow the logistic map z <- 4 z (1 - z), one step per evaluation round.
    Global stage: n_global rounds, each evaluating every chain's point u = z. Centres: greedily, in
    decreasing acquisition value, the evaluated points at least `exclusion` apart (unit-box distance),
    max(centres, q) of them. Local stage: n_local rounds; the first per = P // (number of centres)
    chains are split evenly over the centres (chain i * per + p serves centre i) and evaluate
    u = clip(centre + r (2 z - 1), 0, 1) with r = radius0 shrink^t; a centre moves to its best point of
    the round when that beats the centre's value. Every round keeps its per_step best points (ties by
    lower index) as the pool; the q proposals are taken from the pool greedily in decreasing value,
    each at least `exclusion` from the points already taken and from `taken`.
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


def _greedy(points, values, q, exclusion, taken):
    """Indices of up to q points in decreasing value (ties by lower index), each at least `exclusion`
    from every point in `taken` and from every point picked before it."""
    order = sorted(range(len(values)), key=lambda i: (-values[i], i))
    ref = [np.asarray(t, np.float64) for t in taken]
    picked = []
    for i in order:
        if len(picked) == q:
            break
        u = points[i]
        if all(float(np.sum((u - t) ** 2)) >= exclusion * exclusion for t in ref):
            picked.append(i)
            ref.append(u)
    return picked


def _best_of_round(U, values, per_step):
    """The per_step best points of one round (ties by lower index), in their original order."""
    if len(values) <= per_step:
        return U, values
    keep = sorted(sorted(range(len(values)), key=lambda i: (-values[i], i))[:per_step])
    return U[keep], values[keep]


def chaotic_search(fun, z0: np.ndarray, q: int, taken, n_global: int, n_local: int, centres: int,
                   radius0: float, shrink: float, exclusion: float, per_step: int):
    """Maximise the acquisition `fun` (rows of a [m, d] array -> [m] values) over [0, 1]^d by the
    two-stage chaotic search of the module header, from chains z0 [P, d] in (0, 1).

    Returns (proposals [<= q, d], largest value evaluated, number of evaluations)."""
    z = np.array(z0, dtype=np.float64)
    P, d = z.shape
    pool_u, pool_v = [], []
    evaluations = 0
    for _ in range(n_global):
        v = np.asarray(fun(z.copy()), np.float64)
        evaluations += P
        ku, kv = _best_of_round(z.copy(), v, per_step)
        pool_u += list(ku)
        pool_v += list(kv)
        z = 4.0 * z * (1.0 - z)
    n_c = min(max(centres, q), P)
    cidx = _greedy(pool_u, pool_v, n_c, exclusion, [])
    cen = [pool_u[i].copy() for i in cidx]
    cval = [pool_v[i] for i in cidx]
    per = max(1, P // max(1, len(cen)))
    r = radius0
    for _ in range(n_local):
        U = np.empty((len(cen) * per, d))
        for i in range(len(cen)):
            for p in range(per):
                U[i * per + p] = np.clip(cen[i] + r * (2.0 * z[i * per + p] - 1.0), 0.0, 1.0)
        v = np.asarray(fun(U), np.float64)
        evaluations += len(U)
        ku, kv = _best_of_round(U, v, per_step)
        pool_u += list(ku)
        pool_v += list(kv)
        for i in range(len(cen)):
            j = max(range(per), key=lambda p: (v[i * per + p], -p))   # first of the round's best
            if v[i * per + j] > cval[i]:
                cen[i] = U[i * per + j].copy()
                cval[i] = v[i * per + j]
        z = 4.0 * z * (1.0 - z)
        r *= shrink
    pick = _greedy(pool_u, pool_v, q, exclusion, list(np.asarray(taken, np.float64).reshape(-1, d)))
    return np.array([pool_u[i] for i in pick]).reshape(-1, d), float(max(pool_v)), evaluations
