"""Pins for the oracle's attenuated projector (Eqs. 1-2): exact axis-aligned sums written out with
plain loops, the geometric-series value of a uniform block, the uniform-disc closed form of the
attenuated line integral, the mu = 0 reduction, rotation equivariance, the adjoint identity and
brute-force dense matrices."""
import math

import numpy as np
import pytest

import oracle
from oracle.head import coverage_fractions
from oracle.projector import (attenuation, backproject, prefix_exclusive, project, sensitivity,
                              suffix_exclusive)


def _axis_projection_bruteforce(mu, f, dx, direction):
    """Attenuated sums along image axes with plain loops. direction: 0 -> rays along +y (phi = 0),
    1 -> along -x (phi = 90), 2 -> along -y (phi = 180), 3 -> along +x (phi = 270).
    Returns y[b] with b the bin index of that angle."""
    n = mu.shape[0]
    y = np.zeros(n)
    for b in range(n):
        if direction == 0:       # bin b -> column b, photons travel toward increasing row
            line_mu = [mu[i, b] for i in range(n)]
            line_f = [f[i, b] for i in range(n)]
        elif direction == 1:     # bin b -> row b, photons travel toward decreasing column
            line_mu = [mu[b, l] for l in range(n - 1, -1, -1)]
            line_f = [f[b, l] for l in range(n - 1, -1, -1)]
        elif direction == 2:     # bin b -> column n-1-b, photons toward decreasing row
            line_mu = [mu[i, n - 1 - b] for i in range(n - 1, -1, -1)]
            line_f = [f[i, n - 1 - b] for i in range(n - 1, -1, -1)]
        else:                    # bin b -> row n-1-b, photons toward increasing column
            line_mu = [mu[n - 1 - b, l] for l in range(n)]
            line_f = [f[n - 1 - b, l] for l in range(n)]
        # line_* run from the far end to the detector
        total = 0.0
        for k in range(n):
            ahead = sum(line_mu[k + 1:])
            total += math.exp(-dx * (0.5 * line_mu[k] + ahead)) * line_f[k]
        y[b] = dx * total
    return y


@pytest.mark.parametrize("n", [12, 16])
def test_axis_aligned_angles_exact(n):
    g = oracle.Geometry(n, 4, n, n, 0.3)
    rng = np.random.default_rng(n)
    mu = rng.uniform(0, 0.4, (n, n))
    f = rng.uniform(0, 2, (n, n))
    y = project(g, attenuation(g, mu), f)
    for a in range(4):
        np.testing.assert_allclose(y[a], _axis_projection_bruteforce(mu, f, g.pixel, a),
                                   rtol=1e-13, atol=1e-14)


def test_uniform_block_geometric_series():
    n, dx, mu0, length = 32, 0.25, 0.3, 9
    g = oracle.Geometry(n, 4, n, n, dx)
    mu = np.zeros((n, n))
    f = np.zeros((n, n))
    col, r0 = 11, 7
    mu[r0:r0 + length, col] = mu0
    f[r0:r0 + length, col] = 1.0
    y = project(g, attenuation(g, mu), f)
    expected = dx * (1 - math.exp(-mu0 * length * dx)) / (2 * math.sinh(mu0 * dx / 2))
    assert y[0, col] == pytest.approx(expected, rel=1e-14)


def test_mu_zero_is_plain_radon_column_sums():
    n = 20
    g = oracle.Geometry(n, 8, n, n, 0.5)
    f = np.random.default_rng(0).uniform(0, 1, (n, n))
    y = project(g, attenuation(g, np.zeros((n, n))), f)
    np.testing.assert_allclose(y[0], g.pixel * f.sum(axis=0), rtol=1e-14)
    np.testing.assert_allclose(y[4], g.pixel * f.sum(axis=0)[::-1], rtol=1e-13)


def _disc_error(n, mu0, rho=5.0, fov=16.0):
    g = oracle.Geometry(n, 4, n, n, fov / n)
    fb, _ = coverage_fractions(g, [rho, 0, 0, 0, 0, 0], 0.0)
    y = project(g, attenuation(g, mu0 * fb), fb)
    s = (np.arange(n) - (n - 1) / 2) * g.pixel
    inner = np.abs(s) < rho - 0.6
    L = np.sqrt(rho ** 2 - s[inner] ** 2)
    exact = (1 - np.exp(-2 * mu0 * L)) / mu0 if mu0 > 0 else 2 * L
    err = np.abs(y[:, inner] - exact[None, :]).max() / exact.max()
    return err


@pytest.mark.parametrize("mu0", [0.0, 0.15])
def test_uniform_disc_closed_form_converges(mu0):
    # S(s) = f0 (1 - exp(-2 mu0 L)) / mu0 with chord half-length L = sqrt(rho^2 - s^2)
    errs = [_disc_error(n, mu0) for n in (32, 64, 128)]
    assert errs[-1] < 2e-3
    assert errs[1] < errs[0] and errs[2] < errs[1]
    rate = math.log2(errs[1] / errs[2])
    assert rate > 0.9     # first order or better in the pixel size


def test_rotation_by_quarter_turn_shifts_angles():
    n, na = 24, 16
    g = oracle.Geometry(n, na, n, n, 0.4)
    rng = np.random.default_rng(1)
    mu = rng.uniform(0, 0.3, (n, n))
    f = rng.uniform(0, 1, (n, n))
    y = project(g, attenuation(g, mu), f)
    # np.rot90 gives A'(X, Y) = A(-Y, X): the image turned by -90 deg, so its sinogram at angle
    # phi equals the original's at phi + 90 deg
    y_rot = project(g, attenuation(g, np.rot90(mu)), np.rot90(f))
    np.testing.assert_allclose(y_rot, np.roll(y, -na // 4, axis=0), rtol=1e-12, atol=1e-13)


def test_attenuated_below_unattenuated_and_linear():
    n = 20
    g = oracle.Geometry(n, 12, n, n, 0.5)
    rng = np.random.default_rng(2)
    mu = rng.uniform(0, 0.3, (n, n))
    f1, f2 = rng.uniform(0, 1, (2, n, n))
    att = attenuation(g, mu)
    assert np.all(att <= 1.0) and np.all(att > 0)
    y_mu = project(g, att, f1)
    y_0 = project(g, np.ones_like(att), f1)
    assert np.all(y_mu <= y_0 + 1e-15)
    np.testing.assert_allclose(project(g, att, 2 * f1 - 3 * f2),
                               2 * y_mu - 3 * project(g, att, f2), rtol=1e-12, atol=1e-12)


def test_adjoint_identity():
    n = 32
    g = oracle.Geometry(n, 24, n, n, 0.4)
    rng = np.random.default_rng(4)
    att = attenuation(g, rng.uniform(0, 0.3, (n, n)))
    x = rng.standard_normal((n, n))
    z = rng.standard_normal((g.n_angles, g.n_bins))
    lhs = np.sum(project(g, att, x) * z)
    rhs = np.sum(x * backproject(g, att, z))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_scan_transpose():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 4, 17))
    z = rng.standard_normal((3, 4, 17))
    assert np.sum(suffix_exclusive(x) * z) == pytest.approx(np.sum(x * prefix_exclusive(z)), rel=1e-13)
    np.testing.assert_allclose(suffix_exclusive(x)[..., 3], x[..., 4:].sum(axis=-1), rtol=1e-13)
    np.testing.assert_array_equal(suffix_exclusive(x)[..., -1], 0.0)


def _bilinear_bruteforce(img, u, v):
    n = img.shape[0]
    l0, i0 = math.floor(u), math.floor(v)
    fu, fv = u - l0, v - i0
    val = 0.0
    for di, dl, w in ((0, 0, (1 - fu) * (1 - fv)), (0, 1, fu * (1 - fv)), (1, 0, (1 - fu) * fv),
                      (1, 1, fu * fv)):
        i, l = i0 + di, l0 + dl
        if 0 <= i < n and 0 <= l < n:
            val += w * img[i, l]
    return val


def dense_system_bruteforce(g, mu):
    """A[(a,b), j] from plain loops: bilinear sampling, midpoint scan toward the detector, dx weights."""
    n = g.n
    A = np.zeros((g.n_angles * g.n_bins, n * n))
    for a in range(g.n_angles):
        phi = 2 * math.pi * a / g.n_angles
        c, s = math.cos(phi), math.sin(phi)
        for b in range(g.n_bins):
            sb = (b - (g.n_bins - 1) / 2) * n * g.pixel / g.n_bins
            pts = []
            for k in range(g.n_samples):
                tk = (k - (g.n_samples - 1) / 2) * g.pixel
                x, y = sb * c - tk * s, sb * s + tk * c
                pts.append((x / g.pixel + (n - 1) / 2, y / g.pixel + (n - 1) / 2))
            m = [_bilinear_bruteforce(mu, u, v) for u, v in pts]
            for k, (u, v) in enumerate(pts):
                att = math.exp(-g.pixel * (0.5 * m[k] + sum(m[k + 1:])))
                for j in range(n * n):
                    e = np.zeros(n * n)
                    e[j] = 1
                    w = _bilinear_bruteforce(e.reshape(n, n), u, v)
                    if w:
                        A[a * g.n_bins + b, j] += g.pixel * att * w
    return A


def dense_system_direct(g, mu):
    """A[(a,b), j] from plain loops with the bilinear corner weights written out: for a sample at pixel
    coordinates (u, v) the pixels (floor v + {0,1}, floor u + {0,1}) get (1-fu or fu)(1-fv or fv),
    taps outside the grid dropped; midpoint scan toward the detector, dx weights. Cost linear in the
    sample count, so usable at 16 x 16."""
    n = g.n
    A = np.zeros((g.n_angles * g.n_bins, n * n))

    def taps(u, v):
        l0, i0 = math.floor(u), math.floor(v)
        fu, fv = u - l0, v - i0
        out = []
        for di, wv in ((0, 1.0 - fv), (1, fv)):
            for dl, wu in ((0, 1.0 - fu), (1, fu)):
                i, l = i0 + di, l0 + dl
                if 0 <= i < n and 0 <= l < n and wu * wv != 0.0:
                    out.append((i * n + l, wu * wv))
        return out

    for a in range(g.n_angles):
        phi = 2 * math.pi * a / g.n_angles
        c, s = math.cos(phi), math.sin(phi)
        for b in range(g.n_bins):
            sb = (b - (g.n_bins - 1) / 2) * n * g.pixel / g.n_bins
            tp = []
            for k in range(g.n_samples):
                tk = (k - (g.n_samples - 1) / 2) * g.pixel
                x, y = sb * c - tk * s, sb * s + tk * c
                tp.append(taps(x / g.pixel + (n - 1) / 2, y / g.pixel + (n - 1) / 2))
            m = [sum(w * mu.flat[j] for j, w in t) for t in tp]
            for k in range(g.n_samples):
                att = math.exp(-g.pixel * (0.5 * m[k] + sum(m[k + 1:])))
                for j, w in tp[k]:
                    A[a * g.n_bins + b, j] += g.pixel * att * w
    return A


def test_dense_matrix_direct_equals_unit_image_bruteforce():
    n = 8
    g = oracle.Geometry(n, 6, n, n, 0.5)
    mu = np.random.default_rng(7).uniform(0, 0.4, (n, n))
    np.testing.assert_allclose(dense_system_direct(g, mu), dense_system_bruteforce(g, mu), rtol=1e-13, atol=1e-15)


def test_dense_matrix_bruteforce_matches_projector_and_transpose():
    n = 8
    g = oracle.Geometry(n, 6, n, n, 0.5)
    rng = np.random.default_rng(6)
    mu = rng.uniform(0, 0.4, (n, n))
    A = dense_system_bruteforce(g, mu)
    att = attenuation(g, mu)
    cols = np.stack([project(g, att, np.eye(n * n)[j].reshape(n, n)).ravel() for j in range(n * n)], 1)
    rows = np.stack([backproject(g, att, np.eye(g.n_rays)[i].reshape(g.n_angles, g.n_bins)).ravel()
                     for i in range(g.n_rays)], 0)
    np.testing.assert_allclose(cols, A, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rows, A, rtol=1e-12, atol=1e-14)


def test_sensitivity_positive_on_grid():
    g = oracle.Geometry(16, 8, 16, 16, 0.5)
    s = sensitivity(g, attenuation(g, np.full((16, 16), 0.2)))
    assert np.all(s > 0)


def test_oversampled_simulator_reduces_to_plain_at_factor_one():
    from oracle.phantom import activity_phantom, simulate, simulate_oversampled
    g = oracle.Geometry(24, 12, 24, 24, 25.6 / 24)
    th = np.array([7.5, 0.0, 1.2, 0.0, -0.3, 0.0, 0.15, 0.25])
    disks = [(1.0, 0.5, 1.2)]
    S1, y1, f1 = simulate_oversampled(g, th, 0.8, disks, 1.0, 4.0, 3e4, np.random.default_rng(5), factor=1)
    f = activity_phantom(g, th[:6], 0.8, disks, 1.0, 4.0)
    S0, y0 = simulate(g, th, 0.8, f, 3e4, np.random.default_rng(5))
    np.testing.assert_array_equal(f1, f)
    np.testing.assert_array_equal(y1, y0)
    np.testing.assert_array_equal(S1, S0)


def test_oversampled_simulator_approaches_the_continuous_model():
    # uniform disc of activity and attenuation (closed form per ray): the bin-averaged closed form is
    # matched better by the 2x-oversampled projection than by the plain one
    from oracle.phantom import simulate_oversampled
    n, na = 32, 8
    g = oracle.Geometry(n, na, n, n, 25.6 / n)
    rho, mu0 = 7.0, 0.15
    th = np.array([rho, 0, 0, 0, 0, 0, mu0, 0.0])      # a disc head: mu = mu0 inside, nothing in the shell
    rng = np.random.default_rng(0)
    _, y2, _ = simulate_oversampled(g, th, 0.8, [], 1.0, 4.0, 1.0, rng, factor=2)
    _, y1, _ = simulate_oversampled(g, th, 0.8, [], 1.0, 4.0, 1.0, rng, factor=1)
    # closed form S(s) = (1 - exp(-2 mu0 L)) / mu0, L = sqrt(rho^2 - s^2), averaged over each bin
    ds = n * g.pixel / n
    s_fine = (np.arange(n * 64) - (n * 64 - 1) / 2.0) * ds / 64
    L = np.sqrt(np.maximum(rho * rho - s_fine * s_fine, 0.0))
    ref = ((1.0 - np.exp(-2.0 * mu0 * L)) / mu0).reshape(n, 64).mean(axis=1)
    ref = np.tile(ref / ref.sum() / na, (na, 1))
    e1 = np.abs(y1 - ref).sum() / ref.sum()
    e2 = np.abs(y2 - ref).sum() / ref.sum()
    assert e2 < 0.8 * e1, (e1, e2)
