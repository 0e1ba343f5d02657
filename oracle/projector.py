"""Oracle: attenuated projector A^mu and its exact transpose (FP64, test infrastructure only).

Eq. (1) integrates the activity along each ray, weighted by exp(-int mu) from the emission point to
the detector; Eq. (2) writes the discrete result as S = A^mu F. The oracle discretises both integrals
on the ray samples (spacing dx):

* inner integral (half-self / midpoint rule, scanned toward the detector):
      L_abk = dx * ( m_abk / 2 + sum_{k' > k} m_abk' ),  m = W mu,  att_abk = exp(-L_abk)
* outer integral:
      y_ab = dx * sum_k att_abk (W F)_abk
* the backprojector is the exact transpose of that map:
      (A^T z)_j = dx * sum_{a,b,k} W_{abk,j} att_abk z_ab.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, sample_image, sample_image_transpose


def suffix_exclusive(m: np.ndarray) -> np.ndarray:
    """sum_{k' > k} m[..., k'] along the last axis, scanned from the detector end."""
    out = np.zeros_like(m)
    # running sum starting at the detector end; out[..., k] excludes m[..., k]
    inclusive = np.cumsum(m[..., ::-1], axis=-1)[..., ::-1]
    out[..., :-1] = inclusive[..., 1:]
    return out


def prefix_exclusive(m: np.ndarray) -> np.ndarray:
    """sum_{k' < k} m[..., k'] along the last axis (the transpose of suffix_exclusive)."""
    out = np.zeros_like(m)
    inclusive = np.cumsum(m, axis=-1)
    out[..., 1:] = inclusive[..., :-1]
    return out


def line_integrals(g: Geometry, mu: np.ndarray) -> np.ndarray:
    """L[a, b, k]: attenuation path integral from sample k to the detector."""
    m = sample_image(g, mu)
    return g.pixel * (0.5 * m + suffix_exclusive(m))


def attenuation(g: Geometry, mu: np.ndarray) -> np.ndarray:
    """att[a, b, k] = exp(-L[a, b, k])."""
    return np.exp(-line_integrals(g, mu))


def project(g: Geometry, att: np.ndarray, img: np.ndarray) -> np.ndarray:
    """y = A^mu img, shaped [N_a, N_b]."""
    return g.pixel * np.sum(att * sample_image(g, img), axis=-1)


def backproject(g: Geometry, att: np.ndarray, sino: np.ndarray) -> np.ndarray:
    """(A^mu)^T sino, an n x n image."""
    return g.pixel * sample_image_transpose(g, att * np.asarray(sino, dtype=np.float64)[:, :, None])


def sensitivity(g: Geometry, att: np.ndarray) -> np.ndarray:
    """s = (A^mu)^T 1."""
    return backproject(g, att, np.ones((g.n_angles, g.n_bins)))
