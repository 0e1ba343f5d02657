"""Oracle: scanner geometry and the bilinear sampling matrix W (FP64, test infrastructure only).

Discretisation of the attenuated Radon transform, Eq. (1): the paper fixes neither the angle set, the
detector layout nor the interpolation, so the oracle uses these readings:

* angles phi_a = 2 pi a / N_a over the full 360 deg (the simulation study uses projections over the
  full angular range);
* pixel (i, l) has centre x_l = (l - (N-1)/2) dx, y_i = (i - (N-1)/2) dx, arrays indexed [i][l];
* bin b sits at offset s_b = (b - (N_b-1)/2) N dx / N_b, sample k of a ray at t_k = (k - (N_t-1)/2) dx;
  the sample point is p = s_b (cos phi, sin phi) + t_k (-sin phi, cos phi) and photons travel
  toward +t, so the detector is at the k = N_t - 1 end;
* the image (activity or attenuation) is read at p by bilinear interpolation on the pixel-centre
  lattice with zero outside the grid; the same matrix W serves both images.

Rows of W are ordered (a, b, k) with k fastest; columns are i * N + l.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Geometry:
    n: int            # image is n x n
    n_angles: int     # N_a, over 360 degrees
    n_bins: int       # N_b
    n_samples: int    # N_t, samples per ray, spacing = pixel
    pixel: float      # cm

    @property
    def centre(self) -> float:
        return (self.n - 1) / 2.0

    @property
    def n_rays(self) -> int:
        return self.n_angles * self.n_bins


def angles(g: Geometry) -> np.ndarray:
    return 2.0 * np.pi * np.arange(g.n_angles) / g.n_angles


def pixel_coords(g: Geometry) -> np.ndarray:
    """Centre coordinate (cm) of pixel index 0..n-1 along either axis."""
    return (np.arange(g.n) - g.centre) * g.pixel


def bin_offsets(g: Geometry) -> np.ndarray:
    return (np.arange(g.n_bins) - (g.n_bins - 1) / 2.0) * (g.n * g.pixel / g.n_bins)


def sample_offsets(g: Geometry) -> np.ndarray:
    return (np.arange(g.n_samples) - (g.n_samples - 1) / 2.0) * g.pixel


def sample_points(g: Geometry, phi: float):
    """(x, y) in cm of every sample of angle phi, each shaped [n_bins, n_samples]."""
    s = bin_offsets(g)[:, None]
    t = sample_offsets(g)[None, :]
    c, sn = np.cos(phi), np.sin(phi)
    return s * c - t * sn, s * sn + t * c


def bilinear_taps(g: Geometry, x: np.ndarray, y: np.ndarray):
    """The four bilinear taps of each point: lists of (row i, col l, weight) arrays, weights of taps
    outside the grid removed (zero padding)."""
    u = x / g.pixel + g.centre          # continuous column index
    v = y / g.pixel + g.centre          # continuous row index
    l0 = np.floor(u)
    i0 = np.floor(v)
    fu = u - l0
    fv = v - i0
    l0 = l0.astype(np.int64)
    i0 = i0.astype(np.int64)
    taps = []
    for di, dl, w in ((0, 0, (1 - fu) * (1 - fv)), (0, 1, fu * (1 - fv)),
                      (1, 0, (1 - fu) * fv), (1, 1, fu * fv)):
        ii = i0 + di
        ll = l0 + dl
        taps.append((ii, ll, w))
    return taps


@lru_cache(maxsize=8)
def sampling_matrix(g: Geometry) -> sp.csr_matrix:
    """W: (N_a*N_b*N_t) x (N*N) bilinear sampling of an image at every sample of every ray."""
    n_per_angle = g.n_bins * g.n_samples
    rows, cols, vals = [], [], []
    for a, phi in enumerate(angles(g)):
        x, y = sample_points(g, phi)
        base = a * n_per_angle + np.arange(n_per_angle).reshape(g.n_bins, g.n_samples)
        for ii, ll, w in bilinear_taps(g, x, y):
            keep = (ii >= 0) & (ii < g.n) & (ll >= 0) & (ll < g.n) & (w != 0.0)
            rows.append(base[keep])
            cols.append(ii[keep] * g.n + ll[keep])
            vals.append(w[keep])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(g.n_angles * n_per_angle, g.n * g.n))


def sample_image(g: Geometry, img: np.ndarray) -> np.ndarray:
    """(W img) reshaped [N_a, N_b, N_t]."""
    W = sampling_matrix(g)
    return (W @ np.asarray(img, dtype=np.float64).ravel()).reshape(g.n_angles, g.n_bins, g.n_samples)


def sample_image_transpose(g: Geometry, field: np.ndarray) -> np.ndarray:
    """W^T field for a sample-domain field [N_a, N_b, N_t]; returns an n x n image."""
    W = sampling_matrix(g)
    return (W.T @ np.asarray(field, dtype=np.float64).ravel()).reshape(g.n, g.n)
