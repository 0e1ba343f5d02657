"""Oracle: image-quality scores of the simulation study (SSIM, CNR, PSNR), written from their
definitions with plain loops (FP64, test infrastructure only).

The paper scores reconstructions against the true emission image with SSIM (Wang et al.), the
contrast-to-noise ratio between a region of interest and the background, and the peak signal-to-noise
ratio, without giving parameters. Readings:

  - SSIM: the standard parameters of Wang et al. (11 x 11 Gaussian window, sigma 1.5, normalised to sum 1;
    K1 = 0.01, K2 = 0.03; dynamic range L = max - min of the reference), local statistics over every
    window position that lies inside the image ("valid" positions), mean of the SSIM map.
  - CNR = (mean over the hot region - mean over the background) / standard deviation over the background
    (population standard deviation); hot region: pixels wholly inside a hot disk; background: pixels of
    the brain region touched by no disk.
  - PSNR = 10 log10(max(reference)^2 / MSE) in dB.
"""
from __future__ import annotations

import math

import numpy as np

SSIM_WINDOW = 11
SSIM_SIGMA = 1.5
SSIM_K1, SSIM_K2 = 0.01, 0.03


def gaussian_window(size: int = SSIM_WINDOW, sigma: float = SSIM_SIGMA) -> np.ndarray:
    r = (size - 1) / 2.0
    w = np.empty((size, size))
    for i in range(size):
        for j in range(size):
            w[i, j] = math.exp(-((i - r) ** 2 + (j - r) ** 2) / (2.0 * sigma * sigma))
    return w / w.sum()


def ssim(x: np.ndarray, ref: np.ndarray) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(ref, np.float64)
    L = float(y.max() - y.min())
    c1, c2 = (SSIM_K1 * L) ** 2, (SSIM_K2 * L) ** 2
    w = gaussian_window()
    k = w.shape[0]
    vals = []
    for i in range(x.shape[0] - k + 1):
        for j in range(x.shape[1] - k + 1):
            a = x[i:i + k, j:j + k]
            b = y[i:i + k, j:j + k]
            mx, my = float(np.sum(w * a)), float(np.sum(w * b))
            vx = float(np.sum(w * (a - mx) ** 2))
            vy = float(np.sum(w * (b - my) ** 2))
            cxy = float(np.sum(w * (a - mx) * (b - my)))
            vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))


def cnr(x: np.ndarray, hot: np.ndarray, background: np.ndarray) -> float:
    x = np.asarray(x, np.float64)
    h = [x[i, j] for i in range(x.shape[0]) for j in range(x.shape[1]) if hot[i, j]]
    b = [x[i, j] for i in range(x.shape[0]) for j in range(x.shape[1]) if background[i, j]]
    mb = sum(b) / len(b)
    sb = math.sqrt(sum((v - mb) ** 2 for v in b) / len(b))
    return (sum(h) / len(h) - mb) / sb


def psnr(x: np.ndarray, ref: np.ndarray) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(ref, np.float64)
    mse = float(np.mean((x - y) ** 2))
    return 10.0 * math.log10(float(y.max()) ** 2 / mse)
