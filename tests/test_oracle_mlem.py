"""Pins for the oracle's MLEM and objective (Eq. 5, BOAC step 3): dense explicit-matrix MLEM from the
brute-force system matrix (8 x 8, and 16 x 16 with 16 and 24 angles), count preservation, monotone likelihood (Shepp-Vardi), fixed point, scale
invariance of the first iterate, and the Poisson log-pmf from scipy."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from oracle.mlem import log_factorial, mlem, neg_log_likelihood
from oracle.projector import attenuation, backproject, project, sensitivity

from test_oracle_projector import dense_system_bruteforce, dense_system_direct


def _dense_mlem(A, S, n_iter):
    s = A.sum(axis=0)
    f = np.ones(A.shape[1])
    for _ in range(n_iter):
        y = A @ f
        r = np.where(y > 0, S / np.where(y > 0, y, 1), 0)
        f = np.where(s > 0, f * (A.T @ r) / np.where(s > 0, s, 1), 0)
    return f


@pytest.mark.parametrize("na", [6, 10])
def test_dense_explicit_matrix_mlem(na):
    n = 8
    g = oracle.Geometry(n, na, n, n, 0.5)
    rng = np.random.default_rng(na)
    mu = rng.uniform(0, 0.3, (n, n))
    A = dense_system_bruteforce(g, mu)
    S = rng.poisson(5.0, size=A.shape[0]).astype(float)
    ref = _dense_mlem(A, S, 12)
    got = mlem(g, attenuation(g, mu), S.reshape(na, n), 12)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-11, atol=1e-13)


def _dense_16(na, seed):
    """16 x 16 problem: the system matrix from plain loops, from the projector's columns and from the
    backprojector's rows, and a Poisson sinogram."""
    n = 16
    g = oracle.Geometry(n, na, n, n, 0.5)
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0, 0.3, (n, n))
    A = dense_system_direct(g, mu)
    att = attenuation(g, mu)
    cols = np.stack([project(g, att, np.eye(n * n)[j].reshape(n, n)).ravel() for j in range(n * n)], 1)
    rows = np.stack([backproject(g, att, np.eye(g.n_rays)[i].reshape(na, n)).ravel() for i in range(g.n_rays)], 0)
    S = rng.poisson(A @ rng.uniform(0.5, 2.0, n * n)).astype(float)
    return g, mu, att, A, cols, rows, S


def _pin_dense_mlem_16(g, att, A, S, K=15):
    ref = _dense_mlem(A, S, K)
    got = mlem(g, att, S.reshape(g.n_angles, g.n_bins), K)
    np.testing.assert_allclose(got.ravel(), ref, rtol=1e-11, atol=1e-13 * ref.max())


@pytest.mark.parametrize("na", [16, 24])
def test_dense_explicit_matrix_mlem_16(na):
    # the plain-loop matrix equals the projector's columns and the backprojector's rows (so the two are
    # transposes), and dense NumPy MLEM on it equals the matrix-free oracle MLEM
    g, mu, att, A, cols, rows, S = _dense_16(na, seed=na)
    np.testing.assert_allclose(cols, A, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rows, A, rtol=1e-12, atol=1e-14)
    _pin_dense_mlem_16(g, att, A, S)


@pytest.mark.parametrize("mistake", ["unattenuated_sensitivity", "unguarded_ratio"])
def test_planted_mlem_mistakes_fail_the_dense_pin(monkeypatch, mistake):
    import importlib
    om = importlib.import_module("oracle.mlem")   # the module (the package re-exports a function of that name)
    g, mu, att, A, cols, rows, S = _dense_16(16, seed=16)
    if mistake == "unattenuated_sensitivity":
        # s computed from the plain Radon transform instead of A^T 1
        monkeypatch.setattr(om, "sensitivity", lambda gg, a: sensitivity(gg, np.ones_like(a)))
    else:
        # r = S / y everywhere, with zero counts replaced by one (a mistaken zero-count rule)
        monkeypatch.setattr(om, "ratio", lambda m, y: np.maximum(m, 1.0) / y)
    with pytest.raises(AssertionError):
        _pin_dense_mlem_16(g, att, A, S)


def _problem(n=24, na=24, seed=0):
    g = oracle.Geometry(n, na, n, n, 0.5)
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0, 0.25, (n, n))
    att = attenuation(g, mu)
    f_true = rng.uniform(0.5, 2, (n, n))
    S = rng.poisson(project(g, att, f_true)).astype(float)
    return g, att, S, f_true


def test_count_preservation_every_iteration():
    g, att, S, _ = _problem()
    _, hist = mlem(g, att, S, 8, history=True)
    for n in range(8):
        y_n = project(g, att, hist[n])
        y_next = project(g, att, hist[n + 1])
        assert y_next.sum() == pytest.approx(S[y_n > 0].sum(), rel=1e-12)


def test_log_likelihood_never_decreases_and_image_nonnegative():
    g, att, S, _ = _problem(seed=1)
    _, hist = mlem(g, att, S, 15, history=True)
    J = [neg_log_likelihood(S, project(g, att, f)) for f in hist]
    assert all(J[i + 1] <= J[i] + 1e-9 * abs(J[i]) for i in range(len(J) - 1))
    assert all(np.all(f >= 0) for f in hist)


def test_fixed_point():
    g, att, _, f_true = _problem(seed=2)
    S = project(g, att, f_true)
    f = mlem(g, att, S, 5, f0=f_true)
    np.testing.assert_allclose(f, f_true, rtol=1e-12)


def test_first_iterate_independent_of_start_scale():
    g, att, S, _ = _problem(seed=3)
    f1 = mlem(g, att, S, 3, f0=np.ones((g.n, g.n)))
    f2 = mlem(g, att, S, 3, f0=7.5 * np.ones((g.n, g.n)))
    np.testing.assert_allclose(f1, f2, rtol=1e-12)


def test_sensitivity_is_backprojected_ones():
    g, att, _, _ = _problem(seed=4)
    s = sensitivity(g, att)
    x = np.random.default_rng(9).uniform(size=(g.n, g.n))
    # <A x, 1> = <x, s>
    assert project(g, att, x).sum() == pytest.approx(np.sum(x * s), rel=1e-12)


def test_negative_log_likelihood_is_poisson_logpmf():
    rng = np.random.default_rng(5)
    y = rng.uniform(0.1, 40, 500)
    S = rng.poisson(y).astype(float)
    S[:10] = 0
    J = neg_log_likelihood(S, y)
    assert J == pytest.approx(-scipy.stats.poisson.logpmf(S, y).sum(), rel=1e-13)


def test_negative_log_likelihood_edge_cases():
    assert neg_log_likelihood(np.array([0.0, 0.0]), np.array([0.0, 2.0])) == pytest.approx(2.0)
    assert neg_log_likelihood(np.array([1.0]), np.array([0.0])) == math.inf


def test_log_factorial_exact_small():
    S = np.arange(0, 30, dtype=float)
    exact = np.array([sum(math.log(i) for i in range(2, int(v) + 1)) for v in S])
    np.testing.assert_allclose(log_factorial(S), exact, rtol=1e-13, atol=1e-13)


def test_objective_identity_after_count_preserving_step():
    # After an MLEM step with all y > 0, sum(y^K) = sum(S), so J = sum S - sum S ln y + sum ln S!
    g, att, S, _ = _problem(seed=6)
    f = mlem(g, att, S, 6)
    y = project(g, att, f)
    assert np.all(y > 0)
    J = neg_log_likelihood(S, y)
    alt = S.sum() - np.sum(S * np.log(y)) + np.sum(log_factorial(S))
    assert J == pytest.approx(alt, rel=1e-12)


def test_stored_slices_are_consistent(slice64, slice128):
    for d in (slice64, slice128):
        S = d["meas"].astype(float)
        assert S.sum() == pytest.approx(float(d["counts"]), rel=0.01)
        n = int(d["geometry"][0])
        assert S.shape == (int(d["geometry"][1]), int(d["geometry"][2]))
        assert d["activity"].shape == (n, n)
        assert d["activity"].max() == pytest.approx(4.0, abs=1e-6)
