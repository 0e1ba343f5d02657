"""Oracle: MLEM reconstruction and the Poisson negative log-likelihood (FP64, test infrastructure only).

MLEM (Shepp and Vardi) is the reconstruction the method runs for every candidate, a fixed number of
iterations (BOAC step 3). The paper gives neither the starting image nor the zero-division rules;
the oracle's reading:

    F^0 = 1 on every pixel;  s = (A^mu)^T 1;
    y^n = A^mu F^n;  r^n_i = S_i / y^n_i if y^n_i > 0 else 0;
    F^{n+1} = F^n * ((A^mu)^T r^n) / s   (0 where s <= 0).

The goodness of fit is the Poisson log-likelihood of Eq. (5); its last term prints an index j that
can only mean ln S_i!. The method minimises the negative log-likelihood, evaluated here at the
reconstructed image (one extra projection y = A^mu F^K):

    J = sum_i [ y_i - S_i ln y_i + ln Gamma(S_i + 1) ],

a term with S_i = 0 contributes y_i, and y_i <= 0 with S_i > 0 makes J = +inf.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry
from .head import rasterize_mu
from .projector import attenuation, backproject, project, sensitivity


def ratio(meas: np.ndarray, y: np.ndarray) -> np.ndarray:
    out = np.zeros_like(y)
    pos = y > 0
    out[pos] = meas[pos] / y[pos]
    return out


def mlem(g: Geometry, att: np.ndarray, meas: np.ndarray, n_iter: int, f0=None, history=False):
    """Run n_iter MLEM iterations; returns F^K (and the list F^0..F^K when history is set)."""
    meas = np.asarray(meas, dtype=np.float64)
    s = sensitivity(g, att)
    f = np.ones((g.n, g.n)) if f0 is None else np.array(f0, dtype=np.float64)
    hist = [f.copy()]
    for _ in range(n_iter):
        y = project(g, att, f)
        back = backproject(g, att, ratio(meas, y))
        f = np.where(s > 0, f * back / np.where(s > 0, s, 1.0), 0.0)
        hist.append(f.copy())
    return (f, hist) if history else f


def log_factorial(meas: np.ndarray) -> np.ndarray:
    """ln Gamma(S + 1) per bin, from the standard library's lgamma."""
    return np.vectorize(lambda v: math.lgamma(v + 1.0), otypes=[np.float64])(np.asarray(meas, np.float64))


def neg_log_likelihood(meas: np.ndarray, y: np.ndarray) -> float:
    """J = sum_i [y_i - S_i ln y_i + ln S_i!], the negative of Eq. (5)."""
    meas = np.asarray(meas, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if np.any((y <= 0) & (meas > 0)):
        return math.inf
    terms = y.copy()
    pos = meas > 0
    terms[pos] = y[pos] - meas[pos] * np.log(y[pos])
    return float(np.sum(terms) + np.sum(log_factorial(meas)))


def evaluate(g: Geometry, meas: np.ndarray, theta, delta_r: float, n_iter: int):
    """One candidate: rasterise mu, build att, run MLEM, score. Returns (J, F^K, mu)."""
    mu = rasterize_mu(g, theta, delta_r)
    att = attenuation(g, mu)
    f = mlem(g, att, meas, n_iter)
    y = project(g, att, f)
    return neg_log_likelihood(meas, y), f, mu
