"""Pins for the oracle's image-quality scores: special cases with closed forms."""
import math

import numpy as np
import pytest

import oracle.metrics as om


def test_gaussian_window_is_normalised_and_symmetric():
    w = om.gaussian_window()
    assert w.shape == (11, 11) and w.sum() == pytest.approx(1.0, rel=1e-15)
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    assert w[5, 5] / w[5, 6] == pytest.approx(math.exp(1 / (2 * 1.5 ** 2)), rel=1e-14)


def test_ssim_identity_and_symmetry_of_structure():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(20, 20))
    assert om.ssim(x, x) == pytest.approx(1.0, abs=1e-15)


def test_ssim_of_constant_images_is_the_luminance_term():
    # constant images: zero local variances, SSIM = (2ab + C1) / (a^2 + b^2 + C1) with C1 from the
    # reference's range; a reference with one corner pixel changed sets L while leaving most windows flat
    y = np.full((14, 14), 2.0)
    y[0, 0] = 3.0                        # L = 1; only windows touching (0,0) see it
    x = np.full((14, 14), 1.5)
    c1 = 0.01 ** 2
    got = om.ssim(x, y)
    flat = (2 * 1.5 * 2.0 + c1) / (1.5 ** 2 + 2.0 ** 2 + c1)
    # 16 window positions, one of which contains (0,0)
    w = om.gaussian_window()
    my = 2.0 + w[0, 0]
    vy = np.sum(w * (np.where(np.arange(11)[:, None] + np.arange(11)[None, :] == 0, 3.0, 2.0) - my) ** 2)
    c2 = 0.03 ** 2
    corner = (2 * 1.5 * my + c1) * c2 / ((1.5 ** 2 + my ** 2 + c1) * (vy + c2))
    assert got == pytest.approx((15 * flat + corner) / 16, rel=1e-12)


def test_cnr_closed_form():
    x = np.zeros((4, 4))
    hot = np.zeros((4, 4), bool)
    bg = np.zeros((4, 4), bool)
    x[0, :2] = 5.0
    hot[0, :2] = True
    x[2:, :] = np.array([[1, 2, 3, 4], [1, 2, 3, 4]])
    bg[2:, :] = True
    # background mean 2.5, population std sqrt(1.25)
    assert om.cnr(x, hot, bg) == pytest.approx((5 - 2.5) / math.sqrt(1.25), rel=1e-15)


def test_psnr_closed_form():
    y = np.zeros((10, 10))
    y[3, 3] = 4.0
    x = y + 0.5
    assert om.psnr(x, y) == pytest.approx(10 * math.log10(16 / 0.25), rel=1e-15)
