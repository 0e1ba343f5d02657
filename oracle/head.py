"""Oracle: Legendre head model and partial-volume attenuation map (FP64, test infrastructure only).

Eq. (3) models the head outline as a truncated Legendre series with the first six polynomials; the
printed argument of P_k is the polar angle itself, which would make the outline discontinuous for odd
k, so the oracle reads it as R(theta) = sum_{k=0}^{5} c_k P_k(cos theta), theta measured from +x,
counter-clockwise, about the image centre (cos theta = x / r).

Eq. (4) sets mu = mu_b inside R, mu_c in the shell R < r < R + dR, 0 beyond, and leaves r = R
undefined. The rasteriser gives every pixel a partial-volume fraction: 4 x 4 sub-samples per pixel
(spacing h = pixel/4, offsets (p - 1.5) h), each with the C^1 coverage
H(d) = S(clamp(d/h + 1/2, 0, 1)), S(x) = 3x^2 - 2x^3, of its signed distance d = R(theta_q) - r_q
(brain) or d + dR (brain + cranium). fb = mean H(d_b), fo = mean H(d_b + dR), and
mu = mu_b fb + mu_c (fo - fb). Eq. (4) is taken literally where R < 0.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, pixel_coords

N_LEGENDRE = 6
SUBSAMPLES = 4


def legendre_all(x: np.ndarray, count: int = N_LEGENDRE) -> np.ndarray:
    """P_0..P_{count-1} at x by Bonnet's recurrence (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty((count,) + x.shape)
    out[0] = 1.0
    if count > 1:
        out[1] = x
    for n in range(1, count - 1):
        out[n + 1] = ((2 * n + 1) * x * out[n] - n * out[n - 1]) / (n + 1)
    return out


def head_radius(c, cos_t: np.ndarray) -> np.ndarray:
    """R = sum_k c_k P_k(cos theta), Eq. (3) under the cos-theta reading."""
    P = legendre_all(cos_t, len(c))
    return np.tensordot(np.asarray(c, dtype=np.float64), P, axes=1)


def smooth_coverage(d: np.ndarray, h: float) -> np.ndarray:
    x = np.clip(d / h + 0.5, 0.0, 1.0)
    return x * x * (3.0 - 2.0 * x)


def smooth_coverage_slope(d: np.ndarray, h: float) -> np.ndarray:
    """dH/dd: 6 x (1 - x) / h inside the ramp, 0 outside."""
    x = np.clip(d / h + 0.5, 0.0, 1.0)
    return 6.0 * x * (1.0 - x) / h


def subsample_polar(g: Geometry):
    """Sub-sample radius r_q and cos(theta_q), each shaped [n, n, s*s] (pixel row, pixel col, q)."""
    h = g.pixel / SUBSAMPLES
    offs = (np.arange(SUBSAMPLES) - (SUBSAMPLES - 1) / 2.0) * h
    xc = pixel_coords(g)
    # q enumerates (row offset, col offset) with the column offset fastest
    ys = (xc[:, None] + offs[None, :])            # [n, s]
    xs = (xc[:, None] + offs[None, :])
    Y = ys[:, None, :, None] * np.ones((1, g.n, 1, SUBSAMPLES))
    X = xs[None, :, None, :] * np.ones((g.n, 1, SUBSAMPLES, 1))
    Y = Y.reshape(g.n, g.n, SUBSAMPLES * SUBSAMPLES)
    X = X.reshape(g.n, g.n, SUBSAMPLES * SUBSAMPLES)
    r = np.hypot(X, Y)
    # r = 0 only for a sub-sample exactly at the centre, which the offsets above never produce
    cos_t = np.where(r > 1e-12, X / np.where(r > 1e-12, r, 1.0), 1.0)
    return r, cos_t


def coverage_fractions(g: Geometry, c, delta_r: float):
    """(fb, fo): brain and brain+cranium coverage fractions per pixel, each n x n."""
    h = g.pixel / SUBSAMPLES
    r, cos_t = subsample_polar(g)
    R = head_radius(c, cos_t)
    d_b = R - r
    fb = smooth_coverage(d_b, h).mean(axis=-1)
    fo = smooth_coverage(d_b + delta_r, h).mean(axis=-1)
    return fb, fo


def rasterize_mu(g: Geometry, theta, delta_r: float) -> np.ndarray:
    """Attenuation map (1/cm) of candidate theta = (c_0..c_5, mu_b, mu_c), Eq. (4) with partial volume."""
    theta = np.asarray(theta, dtype=np.float64)
    fb, fo = coverage_fractions(g, theta[:6], delta_r)
    return theta[6] * fb + theta[7] * (fo - fb)


def rasterize_mu_adjoint(g: Geometry, theta, delta_r: float, mu_bar: np.ndarray,
                         with_delta_r: bool = False) -> np.ndarray:
    """Gradient of sum_j mu_bar_j mu_j(theta) with respect to theta (8 values), followed by its
    derivative with respect to the cranium thickness dR when with_delta_r is set (9 values)."""
    theta = np.asarray(theta, dtype=np.float64)
    c, mu_b, mu_c = theta[:6], theta[6], theta[7]
    h = g.pixel / SUBSAMPLES
    r, cos_t = subsample_polar(g)
    P = legendre_all(cos_t, 6)                       # [6, n, n, q]
    R = np.tensordot(c, P, axes=1)
    d_b = R - r
    fb = smooth_coverage(d_b, h).mean(axis=-1)
    fo = smooth_coverage(d_b + delta_r, h).mean(axis=-1)
    # d mu_j / d R_q = (mu_b - mu_c) H'(d_b) / s^2 + mu_c H'(d_b + dR) / s^2, and dR_q/dc_k = P_k
    dmu_dR = ((mu_b - mu_c) * smooth_coverage_slope(d_b, h)
              + mu_c * smooth_coverage_slope(d_b + delta_r, h)) / d_b.shape[-1]
    weight = mu_bar[:, :, None] * dmu_dR              # [n, n, q]
    grad = np.empty(9 if with_delta_r else 8)
    grad[:6] = np.tensordot(P, weight, axes=([1, 2, 3], [0, 1, 2]))
    grad[6] = np.sum(mu_bar * fb)
    grad[7] = np.sum(mu_bar * (fo - fb))
    if with_delta_r:
        # dR enters only through fo: d mu_j / d dR = mu_c mean_q H'(d_b + dR)
        grad[8] = mu_c * np.sum(mu_bar * smooth_coverage_slope(d_b + delta_r, h).mean(axis=-1))
    return grad
