"""Pins for the oracle's head model and rasteriser (Eqs. 3-4), independent of the oracle's own code:
library Legendre routines, textbook special values, polar-area quadrature, exact symmetries and a
brute-force hard-edge supersampling."""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle
from oracle.head import (SUBSAMPLES, coverage_fractions, head_radius, legendre_all, rasterize_mu,
                         rasterize_mu_adjoint, smooth_coverage, smooth_coverage_slope)

TRUE = np.array([7.5, 0.0, 1.2, 0.0, -0.3, 0.0, 0.150, 0.250])
G128 = oracle.Geometry(128, 8, 128, 128, 0.2)


def test_legendre_matches_numpy_library():
    x = np.linspace(-1, 1, 101)
    P = legendre_all(x, 6)
    for k in range(6):
        e = np.zeros(k + 1)
        e[k] = 1
        np.testing.assert_allclose(P[k], npleg.legval(x, e), rtol=0, atol=1e-14)


def test_legendre_special_values():
    P1 = legendre_all(np.array([1.0, -1.0, 0.0]), 6)
    for k in range(6):
        assert P1[k, 0] == pytest.approx(1.0, abs=1e-15)
        assert P1[k, 1] == pytest.approx((-1.0) ** k, abs=1e-15)
    # P_k(0): 1, 0, -1/2, 0, 3/8, 0
    np.testing.assert_allclose(P1[:, 2], [1, 0, -0.5, 0, 3 / 8, 0], atol=1e-15)


def test_legendre_orthogonality_gauss_quadrature():
    x, w = npleg.leggauss(20)
    P = legendre_all(x, 6)
    gram = (P * w) @ P.T
    np.testing.assert_allclose(gram, np.diag([2 / (2 * n + 1) for n in range(6)]), atol=1e-13)


def test_coverage_function_values():
    h = 0.05
    d = np.array([-h, -h / 2, 0.0, h / 2, h, 0.3 * h])
    H = smooth_coverage(d, h)
    np.testing.assert_allclose(H[:5], [0, 0, 0.5, 1, 1], atol=1e-15)
    x = 0.3 + 0.5
    assert H[5] == pytest.approx(3 * x * x - 2 * x ** 3, abs=1e-15)
    # symmetric step: H(d) + H(-d) = 1; slope is the derivative
    dd = np.linspace(-h, h, 41)
    np.testing.assert_allclose(smooth_coverage(dd, h) + smooth_coverage(-dd, h), 1.0, atol=1e-15)
    eps = 1e-7
    fd = (smooth_coverage(dd + eps, h) - smooth_coverage(dd - eps, h)) / (2 * eps)
    np.testing.assert_allclose(smooth_coverage_slope(dd, h), fd, atol=2e-4)


def test_disc_area_closed_form():
    rho = 7.5
    fb, fo = coverage_fractions(G128, [rho, 0, 0, 0, 0, 0], 0.8)
    area = fb.sum() * G128.pixel ** 2
    assert area == pytest.approx(math.pi * rho ** 2, rel=2e-4)
    shell = (fo - fb).sum() * G128.pixel ** 2
    assert shell == pytest.approx(math.pi * ((rho + 0.8) ** 2 - rho ** 2), rel=2e-3)


def test_head_area_polar_quadrature():
    # area of {r < R(theta)} = 1/2 int_0^{2pi} R^2 dtheta (R > 0 for the true head); periodic
    # trapezoid rule with 10^4 nodes, written independently of the rasteriser
    th = np.linspace(0, 2 * np.pi, 10000, endpoint=False)
    ct = np.cos(th)
    R = (7.5 + 1.2 * 0.5 * (3 * ct ** 2 - 1) - 0.3 * (35 * ct ** 4 - 30 * ct ** 2 + 3) / 8)
    assert np.all(R > 0)
    area_q = 0.5 * np.mean(R ** 2) * 2 * np.pi
    assert area_q == pytest.approx(190.14, abs=0.01)
    fb, fo = coverage_fractions(G128, TRUE[:6], 0.8)
    assert fb.sum() * 0.04 == pytest.approx(area_q, rel=3e-4)
    shell_q = 0.5 * np.mean((R + 0.8) ** 2 - R ** 2) * 2 * np.pi
    assert (fo - fb).sum() * 0.04 == pytest.approx(shell_q, rel=3e-3)


def test_head_outline_extent():
    # along +x (theta = 0, cos = 1): R = sum c_k; along +y (cos = 0): c0 - c2/2 + 3 c4 / 8
    assert head_radius(TRUE[:6], np.array([1.0]))[0] == pytest.approx(7.5 + 1.2 - 0.3)
    assert head_radius(TRUE[:6], np.array([0.0]))[0] == pytest.approx(7.5 - 0.6 - 0.3 * 3 / 8)


def test_mirror_symmetry_and_bounds():
    mu = rasterize_mu(G128, TRUE, 0.8)
    np.testing.assert_allclose(mu, mu[::-1, :], atol=1e-15)
    fb, fo = coverage_fractions(G128, TRUE[:6], 0.8)
    assert fb.min() >= 0 and fo.max() <= 1 + 1e-15
    assert np.all(fo >= fb - 1e-15)
    # brain pixels deep inside carry mu_b; far outside is 0
    assert mu[64, 64] == pytest.approx(0.150, abs=1e-15)
    assert mu[0, 0] == 0.0


def test_mu_linear_in_attenuation_coefficients():
    fb, fo = coverage_fractions(G128, TRUE[:6], 0.8)
    t = TRUE.copy()
    t[6], t[7] = 0.37, -0.11
    np.testing.assert_allclose(rasterize_mu(G128, t, 0.8), 0.37 * fb - 0.11 * (fo - fb), atol=1e-15)


def test_partial_volume_vs_hard_supersampling():
    # brute force: 32 x 32 hard 0/1 samples per pixel, written out independently
    g = oracle.Geometry(32, 4, 32, 32, 0.8)
    c = [7.5, 0.4, 1.2, -0.5, -0.3, 0.2]
    fb, _ = coverage_fractions(g, c, 0.8)
    m = 32
    offs = (np.arange(m) - (m - 1) / 2) * (g.pixel / m)
    xc = (np.arange(g.n) - (g.n - 1) / 2) * g.pixel
    X = (xc[None, :, None, None] + offs[None, None, None, :])
    Y = (xc[:, None, None, None] + offs[None, None, :, None])
    r = np.hypot(X, Y)
    ct = X / r
    P = npleg.legvander(ct, 5)
    R = P @ np.array(c)
    hard = (r < R).mean(axis=(2, 3))
    assert np.abs(fb - hard).max() < 0.08
    assert abs(fb.sum() - hard.sum()) / hard.sum() < 2e-3


def test_raster_adjoint_is_the_jacobian_transpose():
    g = oracle.Geometry(40, 4, 40, 40, 0.45)
    rng = np.random.default_rng(3)
    theta = TRUE + np.array([0.1, 0.3, -0.2, 0.4, 0.1, -0.3, 0.01, -0.02])
    mu_bar = rng.standard_normal((g.n, g.n))
    grad = rasterize_mu_adjoint(g, theta, 0.8, mu_bar)
    for k in range(8):
        # the coverage is C^1 (its second derivative jumps at the ramp ends), so central
        # differences converge at O(h) near those points: use a small step
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = np.sum(mu_bar * (rasterize_mu(g, tp, 0.8) - rasterize_mu(g, tm, 0.8))) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-7, abs=1e-8)


def test_subsample_count_is_four():
    assert SUBSAMPLES == 4
