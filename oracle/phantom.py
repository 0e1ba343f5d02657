"""Oracle: synthetic phantom and noisy sinogram simulation (FP64, test infrastructure only).

The paper simulates attenuated, Poisson-noisy sinograms from numerical phantoms whose images are not
published. The stand-in family: activity 1 inside the true head's brain region plus three hot disks
of radius 0.8-1.5 cm at 4x activity (overlaps take the maximum), rasterised with the same sub-sample
coverage as the attenuation map. Disk centres are uniform in the head's bounding box and accepted
when 64 points on the disk's rim lie inside the outline. The noiseless sinogram is the oracle
projector applied with the true attenuation map (the same projector reconstructs it), scaled to the
slice's total counts, then each bin is a Poisson draw. The oversampled variant simulates on a finer
grid than the reconstruction uses (the paper's 72-angle geometry is run that way).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, pixel_coords
from .head import SUBSAMPLES, coverage_fractions, head_radius, rasterize_mu, smooth_coverage
from .projector import attenuation, project


def disk_coverage(g: Geometry, cx: float, cy: float, rho: float) -> np.ndarray:
    h = g.pixel / SUBSAMPLES
    offs = (np.arange(SUBSAMPLES) - (SUBSAMPLES - 1) / 2.0) * h
    xc = pixel_coords(g)
    ys = (xc[:, None] + offs[None, :])[:, None, :, None]
    xs = (xc[:, None] + offs[None, :])[None, :, None, :]
    d = rho - np.hypot(xs - cx, ys - cy)
    return smooth_coverage(d, h).reshape(g.n, g.n, -1).mean(axis=-1)


def place_disks(c, proposals, n_disks: int, r_lo: float, r_hi: float):
    """Accept (cx, cy, rho) proposals whose 64 rim points lie strictly inside R(theta)."""
    th = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
    rmax = float(np.max(head_radius(c, np.cos(th))))
    alpha = 2.0 * np.pi * np.arange(64) / 64
    disks = []
    while len(disks) < n_disks:
        ur, ux, uy = next(proposals)
        rho = r_lo + (r_hi - r_lo) * ur
        cx = -rmax + 2.0 * rmax * ux
        cy = -rmax + 2.0 * rmax * uy
        px = cx + rho * np.cos(alpha)
        py = cy + rho * np.sin(alpha)
        rr = np.hypot(px, py)
        inside = rr < head_radius(c, px / np.where(rr > 0, rr, 1.0))
        if np.all(inside):
            disks.append((cx, cy, rho))
    return disks


def activity_phantom(g: Geometry, c, delta_r: float, disks, background: float, hot: float):
    fb, _ = coverage_fractions(g, c, delta_r)
    hotmap = np.zeros((g.n, g.n))
    for cx, cy, rho in disks:
        hotmap = np.maximum(hotmap, disk_coverage(g, cx, cy, rho))
    return background * fb + (hot - background) * hotmap


def simulate_oversampled(g: Geometry, theta_true, delta_r: float, disks, background: float, hot: float,
                         counts: float, noise_rng: np.random.Generator, factor: int = 2):
    """Noisy sinogram of geometry g simulated on a grid `factor` times finer than the one that
    reconstructs it, so that the model does not generate its own data (no inverse crime): phantom and
    attenuation map at pixel/factor, rays at factor x the bins and samples; each bin of g is the sum of
    its `factor` sub-bins (they tile it). Returns (S [N_a, N_b], noiseless mean, fine activity)."""
    gf = Geometry(g.n * factor, g.n_angles, g.n_bins * factor, g.n_samples * factor, g.pixel / factor)
    f = activity_phantom(gf, theta_true[:6], delta_r, disks, background, hot)
    att = attenuation(gf, rasterize_mu(gf, theta_true, delta_r))
    fine = project(gf, att, f)
    ybar = fine.reshape(g.n_angles, g.n_bins, factor).sum(axis=-1)
    ybar = ybar * (counts / ybar.sum())
    return noise_rng.poisson(ybar), ybar, f


def simulate(g: Geometry, theta_true, delta_r: float, activity: np.ndarray, counts: float,
             noise_rng: np.random.Generator):
    """(S integer counts [N_a, N_b], noiseless mean [N_a, N_b])."""
    mu = rasterize_mu(g, theta_true, delta_r)
    att = attenuation(g, mu)
    ybar = project(g, att, activity)
    ybar = ybar * (counts / ybar.sum())
    return noise_rng.poisson(ybar), ybar
