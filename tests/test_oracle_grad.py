"""Pins for the oracle's gradient: central finite differences of the oracle objective (FP64), and
planted-mistake checks showing that the exact pins fail when a plausible error is put into the oracle."""
import numpy as np
import pytest

import oracle
import oracle.adjoint
import oracle.projector
from oracle.phantom import activity_phantom, simulate

TRUE = np.array([7.5, 0.0, 1.2, 0.0, -0.3, 0.0, 0.150, 0.250])


def _problem(n=24, na=24, seed=0, counts=2e4):
    g = oracle.Geometry(n, na, n, n, 25.6 / n)
    f = activity_phantom(g, TRUE[:6], 0.8, [(2.0, 1.0, 1.2), (-3.0, -1.5, 1.0)], 1.0, 4.0)
    S, _ = simulate(g, TRUE, 0.8, f, counts, np.random.default_rng(seed))
    theta = TRUE + np.array([0.3, 0.2, -0.2, 0.1, 0.1, -0.1, 0.01, -0.02])
    return g, S.astype(float), theta


def _fd_check(g, S, theta, n_iter):
    J, grad = oracle.objective_and_grad(g, S, theta, 0.8, n_iter)
    J2 = oracle.evaluate(g, S, theta, 0.8, n_iter)[0]
    assert J == pytest.approx(J2, rel=1e-14)
    fd = oracle.central_difference(lambda th: oracle.evaluate(g, S, th, 0.8, n_iter)[0], theta,
                                   rel_step=1e-5, richardson=False)
    rel = np.linalg.norm(fd - grad) / np.linalg.norm(grad)
    return rel, fd, grad


def _pin_fd(g, S, theta, n_iter):
    rel, fd, grad = _fd_check(g, S, theta, n_iter)
    assert rel < 1e-6, (rel, fd, grad)
    np.testing.assert_allclose(grad, fd, rtol=1e-4, atol=1e-6 * np.linalg.norm(grad))


@pytest.mark.parametrize("n_iter", [0, 1, 4])
def test_gradient_matches_central_differences(n_iter):
    g, S, theta = _problem(seed=n_iter)
    _pin_fd(g, S, theta, n_iter)


def test_gradient_matches_richardson_differences():
    g, S, theta = _problem(n=20, na=16, seed=7)
    _, grad = oracle.objective_and_grad(g, S, theta, 0.8, 3)
    fd = oracle.central_difference(lambda th: oracle.evaluate(g, S, th, 0.8, 3)[0], theta,
                                   rel_step=1e-4, richardson=True)
    assert np.linalg.norm(fd - grad) / np.linalg.norm(grad) < 1e-6


# ---------------- planted mistakes (each must make a pin fail) ----------------

def _inclusive_suffix(m):
    return np.cumsum(m[..., ::-1], axis=-1)[..., ::-1]


def test_planted_inclusive_scan_breaks_exact_axis_pin(monkeypatch):
    from test_oracle_projector import _axis_projection_bruteforce
    n = 12
    g = oracle.Geometry(n, 4, n, n, 0.3)
    rng = np.random.default_rng(0)
    mu = rng.uniform(0, 0.4, (n, n))
    f = rng.uniform(0, 2, (n, n))
    monkeypatch.setattr(oracle.projector, "suffix_exclusive", _inclusive_suffix)
    y = oracle.projector.project(g, oracle.projector.attenuation(g, mu), f)
    assert not np.allclose(y[0], _axis_projection_bruteforce(mu, f, g.pixel, 0), rtol=1e-6)


def test_planted_adjoint_scan_direction_breaks_fd_pin(monkeypatch):
    g, S, theta = _problem(n=16, na=12, seed=1)
    monkeypatch.setattr(oracle.adjoint, "prefix_exclusive", oracle.projector.suffix_exclusive)
    with pytest.raises(AssertionError):
        _pin_fd(g, S, theta, 2)


def test_planted_missing_sensitivity_adjoint_breaks_fd_pin(monkeypatch):
    g, S, theta = _problem(n=16, na=12, seed=2)
    real = oracle.adjoint.sample_image

    calls = {"n": 0}

    def drop_last_call(gg, img):
        # the sensitivity adjoint is the last image sampling in the reverse sweep: zero it
        calls["n"] += 1
        out = real(gg, img)
        return out * 0.0 if calls["n"] == 2 + 2 * 2 else out

    monkeypatch.setattr(oracle.adjoint, "sample_image", drop_last_call)
    with pytest.raises(AssertionError):
        _pin_fd(g, S, theta, 2)


def test_planted_sign_error_in_ratio_adjoint_breaks_fd_pin(monkeypatch):
    g, S, theta = _problem(n=16, na=12, seed=3)
    real = oracle.adjoint.ratio
    monkeypatch.setattr(oracle.adjoint, "ratio", lambda m, y: -real(m, y))
    with pytest.raises(AssertionError):
        _pin_fd(g, S, theta, 2)


# ---------------- dR derivative and the envelope gradient ----------------

def test_raster_adjoint_delta_r_matches_central_differences():
    g = oracle.Geometry(20, 4, 20, 20, 1.0)
    theta = TRUE + np.array([0.2, 0.3, -0.4, 0.2, 0.1, -0.2, 0.01, 0.03])
    mu_bar = np.random.default_rng(4).normal(size=(20, 20))
    grad = oracle.rasterize_mu_adjoint(g, theta, 0.8, mu_bar, with_delta_r=True)
    assert grad.shape == (9,)
    np.testing.assert_array_equal(grad[:8], oracle.rasterize_mu_adjoint(g, theta, 0.8, mu_bar))
    h = 1e-5
    fd = (np.sum(mu_bar * oracle.rasterize_mu(g, theta, 0.8 + h))
          - np.sum(mu_bar * oracle.rasterize_mu(g, theta, 0.8 - h))) / (2 * h)
    assert grad[8] == pytest.approx(fd, rel=1e-6)
    # dR moves only the outer edge, whose attenuation is mu_c: a zero cranium coefficient removes it
    th0 = theta.copy()
    th0[7] = 0.0
    assert oracle.rasterize_mu_adjoint(g, th0, 0.8, mu_bar, with_delta_r=True)[8] == 0.0


@pytest.mark.parametrize("n_iter", [0, 3])
def test_delta_r_gradient_matches_central_differences(n_iter):
    g, S, theta = _problem(n=20, na=16, seed=11 + n_iter)
    J, grad = oracle.objective_and_grad(g, S, theta, 0.8, n_iter, with_delta_r=True)
    J8, grad8 = oracle.objective_and_grad(g, S, theta, 0.8, n_iter)
    assert J == J8
    np.testing.assert_array_equal(grad[:8], grad8)
    fd = oracle.central_difference(lambda d: oracle.evaluate(g, S, theta, float(d[0]), n_iter)[0],
                                   np.array([0.8]), rel_step=1e-4, richardson=True)[0]
    assert grad[8] == pytest.approx(fd, rel=1e-6)


def test_envelope_gradient_matches_central_differences_with_image_fixed():
    g, S, theta = _problem(n=20, na=16, seed=5)
    n_iter = 3
    J, grad = oracle.objective_and_envelope_grad(g, S, theta, 0.8, n_iter, with_delta_r=True)
    J_full, _ = oracle.objective_and_grad(g, S, theta, 0.8, n_iter)
    assert J == pytest.approx(J_full, rel=1e-14)
    fK = oracle.evaluate(g, S, theta, 0.8, n_iter)[1]
    th9 = np.concatenate([theta, [0.8]])
    fd = oracle.central_difference(
        lambda t: oracle.envelope_objective(g, S, t[:8], float(t[8]), fK), th9, rel_step=1e-4, richardson=True)
    assert np.linalg.norm(fd - grad) / np.linalg.norm(grad) < 1e-6, (fd, grad)


def test_envelope_gradient_equals_unrolled_gradient_without_iterations():
    # with K = 0 the reconstruction is F^0 = 1, which does not depend on theta: both gradients agree
    g, S, theta = _problem(n=16, na=12, seed=6)
    J1, g1 = oracle.objective_and_grad(g, S, theta, 0.8, 0, with_delta_r=True)
    J2, g2 = oracle.objective_and_envelope_grad(g, S, theta, 0.8, 0, with_delta_r=True)
    assert J1 == J2
    np.testing.assert_allclose(g2, g1, rtol=1e-12, atol=1e-12 * np.linalg.norm(g1))


def test_envelope_gradient_differs_from_unrolled_gradient_after_iterations():
    # the image's own dependence on theta is what the envelope variant drops
    g, S, theta = _problem(n=16, na=12, seed=6)
    _, g1 = oracle.objective_and_grad(g, S, theta, 0.8, 4)
    _, g2 = oracle.objective_and_envelope_grad(g, S, theta, 0.8, 4)
    assert np.linalg.norm(g2 - g1) / np.linalg.norm(g1) > 1e-3


def test_planted_stale_image_breaks_envelope_fd_pin(monkeypatch):
    # an envelope gradient taken at F^{K-1} instead of F^K must fail the fixed-image FD pin
    g, S, theta = _problem(n=16, na=12, seed=8)
    real = oracle.adjoint.mlem
    monkeypatch.setattr(oracle.adjoint, "mlem", lambda gg, att, m, k: real(gg, att, m, max(k - 1, 0)))
    _, grad = oracle.objective_and_envelope_grad(g, S, theta, 0.8, 3)
    fK = oracle.evaluate(g, S, theta, 0.8, 3)[1]
    fd = oracle.central_difference(lambda t: oracle.envelope_objective(g, S, t, 0.8, fK), theta,
                                   rel_step=1e-4, richardson=True)
    assert np.linalg.norm(fd - grad) / np.linalg.norm(grad) > 1e-4
