"""Oracle: exact gradient of the discrete objective with respect to (c_0..c_5, mu_b, mu_c) and dR.

The paper's joint problem (Eq. 6) minimises -ln P over the image and the head coefficients; BOAC
searches the coefficients with Bayesian optimisation and gets the image from a fixed number of MLEM
iterations. The gradient here is the exact derivative of the discrete J(theta) as computed by
``oracle.mlem.evaluate``: through the rasteriser, the attenuation scan, the sensitivity image, all
K unrolled MLEM iterations and the final projection (S and F^0 are constants; the cranium thickness
dR is a constant of the search, and its derivative is returned on request). It is plain reverse mode
over stored iterates, with no fusion: every adjoint line below undoes one forward line.

The envelope gradient is the cheaper variant: the joint objective of Eq. (6) differentiated in the
head parameters with the image held at the reconstruction F^K (one projection adjoint instead of the
reverse sweep through the iterations).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, sample_image, sample_image_transpose
from .head import rasterize_mu, rasterize_mu_adjoint
from .mlem import mlem, neg_log_likelihood, ratio
from .projector import attenuation, backproject, prefix_exclusive, project, sensitivity


def _theta_bar(g: Geometry, theta, delta_r: float, att: np.ndarray, att_bar: np.ndarray, with_delta_r: bool):
    """Pull an adjoint of the attenuation factors back to the head parameters."""
    dx = g.pixel
    # att = exp(-L)
    L_bar = -att * att_bar
    # L_k = dx (m_k / 2 + sum_{k'>k} m_k')  =>  m_bar_k = dx (L_bar_k / 2 + sum_{k'<k} L_bar_k')
    m_bar = dx * (0.5 * L_bar + prefix_exclusive(L_bar))
    # m = W mu
    mu_bar = sample_image_transpose(g, m_bar)
    return rasterize_mu_adjoint(g, theta, delta_r, mu_bar, with_delta_r)


def _final_ybar(meas: np.ndarray, yK: np.ndarray) -> np.ndarray:
    # J = sum_i y_i - S_i ln y_i + const, y = A F^K
    # d/dy (y - S ln y) = 1 - S/y where y > 0; a bin with S = 0 contributes y (slope 1) anywhere
    return np.where(yK > 0, 1.0 - ratio(meas, yK), np.where(meas == 0, 1.0, 0.0))


def objective_and_grad(g: Geometry, meas: np.ndarray, theta, delta_r: float, n_iter: int,
                       with_delta_r: bool = False):
    """Returns (J, grad[8]), or (J, grad[9]) with dJ/d(dR) last when with_delta_r is set."""
    dx = g.pixel
    meas = np.asarray(meas, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)

    # ---- forward, keeping every iterate ----
    mu = rasterize_mu(g, theta, delta_r)
    att = attenuation(g, mu)
    s = sensitivity(g, att)
    s_pos = s > 0
    s_safe = np.where(s_pos, s, 1.0)
    F = [np.ones((g.n, g.n))]
    Y, R, B = [], [], []
    for _ in range(n_iter):
        y = project(g, att, F[-1])
        r = ratio(meas, y)
        b = backproject(g, att, r)
        Y.append(y)
        R.append(r)
        B.append(b)
        F.append(np.where(s_pos, F[-1] * b / s_safe, 0.0))
    yK = project(g, att, F[-1])
    J = neg_log_likelihood(meas, yK)

    # ---- reverse ----
    ybar = _final_ybar(meas, yK)
    att_bar = dx * ybar[:, :, None] * sample_image(g, F[-1])
    f_bar = backproject(g, att, ybar)
    s_bar = np.zeros((g.n, g.n))
    for n in range(n_iter - 1, -1, -1):
        # F^{n+1} = F^n * b^n / s
        b_bar = np.where(s_pos, f_bar * F[n] / s_safe, 0.0)
        s_bar -= np.where(s_pos, f_bar * F[n + 1] / s_safe, 0.0)
        f_bar_direct = np.where(s_pos, f_bar * B[n] / s_safe, 0.0)
        # b^n = dx W^T (att * r^n)
        wb = sample_image(g, b_bar)
        r_bar = dx * np.sum(att * wb, axis=-1)
        att_bar += dx * R[n][:, :, None] * wb
        # r^n = S / y^n where y^n > 0
        y_pos = Y[n] > 0
        y_bar = np.where(y_pos, -r_bar * R[n] / np.where(y_pos, Y[n], 1.0), 0.0)
        # y^n = dx sum_k att * (W F^n)
        att_bar += dx * y_bar[:, :, None] * sample_image(g, F[n])
        f_bar = f_bar_direct + backproject(g, att, y_bar)
    # s = dx W^T (att * 1)
    att_bar += dx * sample_image(g, s_bar)
    return J, _theta_bar(g, theta, delta_r, att, att_bar, with_delta_r)


def envelope_objective(g: Geometry, meas: np.ndarray, theta, delta_r: float, f_fixed: np.ndarray) -> float:
    """J_F(theta) = sum_i [y_i - S_i ln y_i + ln S_i!] at y = A^{mu(theta)} F with the image F held fixed:
    the joint objective of Eq. (6) (negated log-likelihood) as a function of the head parameters alone."""
    att = attenuation(g, rasterize_mu(g, theta, delta_r))
    return neg_log_likelihood(meas, project(g, att, f_fixed))


def objective_and_envelope_grad(g: Geometry, meas: np.ndarray, theta, delta_r: float, n_iter: int,
                                with_delta_r: bool = False):
    """J at F^K(theta) and the envelope gradient: the derivative of envelope_objective at F = F^K(theta),
    i.e. the reconstruction is treated as a constant (exact when F^K maximises the likelihood for this
    attenuation map; an approximation of the unrolled gradient after finitely many iterations).
    Returns (J, grad[8]) or (J, grad[9]) with dR last."""
    dx = g.pixel
    meas = np.asarray(meas, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    att = attenuation(g, rasterize_mu(g, theta, delta_r))
    fK = mlem(g, att, meas, n_iter)
    yK = project(g, att, fK)
    J = neg_log_likelihood(meas, yK)
    # y = dx sum_k att * (W F): att_bar = dx ybar (W F)
    att_bar = dx * _final_ybar(meas, yK)[:, :, None] * sample_image(g, fK)
    return J, _theta_bar(g, theta, delta_r, att, att_bar, with_delta_r)


def central_difference(fun, theta, rel_step: float = 1e-4, richardson: bool = True):
    """Central finite differences of a scalar fun(theta) with h_k = rel_step * |theta_k| (rel_step
    absolute when theta_k = 0); with Richardson extrapolation over h and h/2."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.empty_like(theta)
    for k in range(theta.size):
        h = rel_step * abs(theta[k]) if theta[k] != 0 else rel_step

        def d(step):
            tp = theta.copy()
            tm = theta.copy()
            tp[k] += step
            tm[k] -= step
            return (fun(tp) - fun(tm)) / (2 * step)

        if richardson:
            out[k] = (4.0 * d(h / 2) - d(h)) / 3.0
        else:
            out[k] = d(h)
    return out
