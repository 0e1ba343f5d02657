"""Pins for the oracle's surrogate model and acquisition (oracle/bo.py): closed forms of the GP
posterior, the EI integral by quadrature, the logistic map's closed form, and planted mistakes."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle.bo as bo


def test_rbf_closed_form_and_psd():
    rng = np.random.default_rng(0)
    U = rng.uniform(size=(30, 8))
    K = bo.rbf(U, U, 2.0, 0.4)
    i, j = 3, 17
    assert K[i, j] == pytest.approx(2.0 * math.exp(-np.sum((U[i] - U[j]) ** 2) / (2 * 0.16)), rel=1e-15)
    assert np.allclose(np.diag(K), 2.0)
    assert np.linalg.eigvalsh(K).min() > -1e-12


def test_single_point_posterior_closed_form():
    # one observation y1 at u1: mu(u) = m0 + s k(u,u1) z1 / (amp + noise), var = amp - k^2 / (amp + noise);
    # with one point the standardised target is 0, so the mean is the observation itself everywhere
    u1 = np.array([[0.2, 0.7]])
    gp = bo.GP(u1, np.array([5.0]), 0.3, 1.0, 0.0)
    q = np.array([[0.5, 0.5], [0.2, 0.7]])
    mu, sd = gp.predict(q)
    d2 = np.sum((q - u1) ** 2, axis=1)
    k = np.exp(-d2 / (2 * 0.09))
    np.testing.assert_allclose(mu, 5.0, rtol=1e-15)
    np.testing.assert_allclose(sd, np.sqrt(np.maximum(1.0 - k * k, 0.0)), atol=1e-12)


def test_two_point_posterior_closed_form():
    # y = (0, 2): m0 = 1, s = sqrt(2), z = (-1, 1)/sqrt(2); with rho = k(u1, u2) the weights are
    # alpha = z / (1 - rho) (antisymmetric target), mean at u: m0 + s (k1 - k2) a, a = z2 / (1 - rho)
    U = np.array([[0.0], [0.5]])
    gp = bo.GP(U, np.array([0.0, 2.0]), 0.5, 1.0, 0.0)
    rho = math.exp(-0.25 / 0.5)
    q = np.array([[0.1], [0.9]])
    k1 = np.exp(-(q[:, 0] - 0.0) ** 2 / 0.5)
    k2 = np.exp(-(q[:, 0] - 0.5) ** 2 / 0.5)
    a = (1 / math.sqrt(2)) / (1 - rho)
    mu, sd = gp.predict(q)
    np.testing.assert_allclose(mu, 1.0 + math.sqrt(2) * (k2 - k1) * a, rtol=1e-12)
    # variance: 1 - [k1 k2] K^-1 [k1 k2]^T with K^-1 = [[1, -rho], [-rho, 1]] / (1 - rho^2)
    var = 1 - (k1 * k1 + k2 * k2 - 2 * rho * k1 * k2) / (1 - rho * rho)
    np.testing.assert_allclose(sd, math.sqrt(2) * np.sqrt(var), rtol=1e-10)


def test_posterior_interpolates_and_reverts_to_prior():
    rng = np.random.default_rng(1)
    U = rng.uniform(size=(25, 8))
    y = np.sin(3 * U[:, 0]) + U[:, 1] ** 2 + 10.0
    gp = bo.GP(U, y, 0.5, 1.0, 1e-10)
    mu, sd = gp.predict(U)
    np.testing.assert_allclose(mu, y, atol=1e-5)
    assert sd.max() < 1e-3
    far = np.full((1, 8), 50.0)
    mu_f, sd_f = gp.predict(far)
    assert mu_f[0] == pytest.approx(gp.m0, abs=1e-12)
    assert sd_f[0] == pytest.approx(gp.s, rel=1e-12)


def test_log_marginal_likelihood_matches_multivariate_normal():
    rng = np.random.default_rng(2)
    U = rng.uniform(size=(12, 3))
    y = rng.normal(size=12) * 3 + 1
    gp = bo.GP(U, y, 0.4, 1.0, 1e-3)
    K = bo.rbf(U, U, 1.0, 0.4) + 1e-3 * np.eye(12)
    ref = stats.multivariate_normal(np.zeros(12), K).logpdf(gp.z)
    assert gp.log_marginal_likelihood() == pytest.approx(ref, rel=1e-12)


def test_fit_gp_picks_the_best_grid_length():
    rng = np.random.default_rng(3)
    U = rng.uniform(size=(40, 2))
    y = np.cos(4 * U[:, 0]) * np.sin(3 * U[:, 1])
    gp = bo.fit_gp(U, y)
    lmls = [bo.GP(U, y, l).log_marginal_likelihood() for l in bo.LENGTH_GRID]
    assert gp.length == bo.LENGTH_GRID[int(np.argmax(lmls))]


@pytest.mark.parametrize("mu,sigma,best,xi", [(1.0, 0.5, 1.2, 0.0), (3.0, 2.0, 1.0, 0.1), (0.0, 1e-3, 0.5, 0.01),
                                              (-2.0, 0.7, -2.5, 0.05)])
def test_expected_improvement_equals_its_integral(mu, sigma, best, xi):
    # EI = E[max(0, best - xi - Y)], Y ~ N(mu, sigma^2), by adaptive quadrature
    f = lambda t: max(0.0, best - xi - t) * stats.norm.pdf(t, mu, sigma)
    ref, _ = integrate.quad(f, mu - 12 * sigma, mu + 12 * sigma, points=[best - xi], limit=200, epsabs=1e-14)
    got = bo.expected_improvement(np.array([mu]), np.array([sigma]), best, xi)[0]
    assert got == pytest.approx(ref, rel=1e-8, abs=1e-14)


def test_expected_improvement_without_uncertainty():
    ei = bo.expected_improvement(np.array([1.0, 3.0]), np.array([0.0, 0.0]), 2.0, 0.25)
    np.testing.assert_array_equal(ei, [0.75, 0.0])


def test_logistic_map_closed_form():
    # z_t = sin^2(2^t asin(sqrt(z_0))) for the fully chaotic logistic map; exact to rounding for small t
    z0 = np.array([0.123, 0.456, 0.789])
    seq = bo.logistic_map(z0, 12)
    ref = np.sin(2.0 ** np.arange(13)[:, None] * np.arcsin(np.sqrt(z0))[None, :]) ** 2
    np.testing.assert_allclose(seq, ref, atol=1e-9)
    assert np.all((seq > 0) & (seq < 1))


def _search(fun, z0, q=1, taken=(), **kw):
    args = dict(n_global=20, n_local=60, centres=4, radius0=0.1, shrink=0.85, exclusion=0.02, per_step=256)
    args.update(kw)
    return bo.chaotic_search(fun, z0, q, np.asarray(taken, np.float64).reshape(-1, z0.shape[1]), **args)


def test_chaotic_search_finds_a_known_maximum():
    target = np.array([0.31, 0.77, 0.52])
    fun = lambda U: -np.sum((U - target) ** 2, axis=1)
    z0 = np.random.default_rng(4).uniform(0.05, 0.95, size=(64, 3))
    U, f, m = _search(fun, z0)
    assert m == 20 * 64 + 60 * 64
    assert np.abs(U[0] - target).max() < 2e-3 and f > -1e-5 and fun(U)[0] == f


def test_chaotic_search_finds_both_modes_and_respects_exclusion():
    # two separated maxima of different heights: with q = 2 the proposals are the two peaks (in order
    # of height), and a third proposal is at least `exclusion` from both and from `taken`
    a, b = np.array([0.2, 0.3]), np.array([0.8, 0.7])
    fun = lambda U: (np.exp(-np.sum((U - a) ** 2, axis=1) / 0.001)
                     + 0.5 * np.exp(-np.sum((U - b) ** 2, axis=1) / 0.001))
    z0 = np.random.default_rng(5).uniform(0.05, 0.95, size=(256, 2))
    # exclusion 0.1: the first peak's shoulder there is exp(-10), below the second peak's 0.5
    U, f, _ = _search(fun, z0, q=3, taken=[[0.5, 0.5]], exclusion=0.1)
    assert np.abs(U[0] - a).max() < 5e-3 and np.abs(U[1] - b).max() < 5e-3
    assert f == pytest.approx(1.0, abs=1e-4)
    pts = np.vstack([U, [[0.5, 0.5]]])
    d2 = np.sum((pts[:, None] - pts[None]) ** 2, axis=-1) + np.eye(len(pts))
    assert d2.min() >= 0.1 ** 2


def test_planted_centre_never_moving_fails_the_maximum_pin(monkeypatch):
    # a local stage whose radius never shrinks (shrink = 1) cannot refine to the known maximum
    target = np.array([0.31, 0.77, 0.52])
    fun = lambda U: -np.sum((U - target) ** 2, axis=1)
    z0 = np.random.default_rng(4).uniform(0.05, 0.95, size=(64, 3))
    U, f, _ = _search(fun, z0, shrink=1.0)
    assert not (np.abs(U[0] - target).max() < 2e-3 and f > -1e-5)


def test_planted_sign_error_in_gamma_breaks_the_integral_pin():
    real = bo.expected_improvement

    def wrong(mu, sigma, best, xi):  # Eq. (10) as printed (improvement toward larger J)
        return real(2 * best - np.asarray(mu), sigma, best, -xi)

    mu, sigma, best, xi = 1.0, 0.5, 1.2, 0.0
    f = lambda t: max(0.0, best - xi - t) * stats.norm.pdf(t, mu, sigma)
    ref, _ = integrate.quad(f, mu - 12 * sigma, mu + 12 * sigma, points=[best - xi])
    assert abs(wrong(np.array([mu]), np.array([sigma]), best, xi)[0] - ref) > 1e-3


def test_fit_gp_selection_subset():
    rng = np.random.default_rng(5)
    U = rng.uniform(size=(60, 3))
    y = np.exp(2 * U[:, 0]) + U[:, 2]
    gp = bo.fit_gp(U, y, n_select=20)
    idx = np.argsort(y, kind="stable")[:20]
    lmls = [bo.GP(U[idx], y[idx], l).log_marginal_likelihood() for l in bo.LENGTH_GRID]
    assert gp.length == bo.LENGTH_GRID[int(np.argmax(lmls))]
    assert len(gp.y) == 60
