"""BOAC against reconstruction without attenuation correction (the paper's simulation study, Table I),
on seeded synthetic cases.

For every case (a noisy 72-angle sinogram simulated on a 2x finer grid, its true activity and head):
  - BOAC: the outer loop (bo.BOAC) picks the head parameters, then MLEM reconstructs with mu(theta_best);
  - NAC: MLEM with mu = 0;
  - AC with the true head, as a reference;
and each reconstruction, divided by the simulation's count scale (total counts over the total projection
of the true activity through the true attenuation), is scored against the true activity with SSIM, CNR
and PSNR (the paper's three scores, parameters of Wang et al. for SSIM). The shape of Table I is reproduced, not its numbers: the
paper's phantoms are not published.

    python -m paper_2109_11920_amd.study --inputs tests/golden/study_cases.npz [--cycles 8] [--gradient envelope]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch
from numpy.lib.stride_tricks import sliding_window_view

from .api import Context, Geometry
from .bo import BOAC

SSIM_K1, SSIM_K2 = 0.01, 0.03


def _window(size=11, sigma=1.5):
    r = np.arange(size) - (size - 1) / 2.0
    g = np.exp(-(r[:, None] ** 2 + r[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim(x: np.ndarray, ref: np.ndarray) -> float:
    """Mean SSIM over every window position inside the image (11 x 11 Gaussian, sigma 1.5, K1 0.01, K2 0.03,
    L = range of the reference)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(ref, np.float64)
    w = _window()
    L = float(y.max() - y.min())
    c1, c2 = (SSIM_K1 * L) ** 2, (SSIM_K2 * L) ** 2
    X = sliding_window_view(x, w.shape)
    Y = sliding_window_view(y, w.shape)
    mx = np.tensordot(X, w, axes=([2, 3], [0, 1]))
    my = np.tensordot(Y, w, axes=([2, 3], [0, 1]))
    dx = X - mx[:, :, None, None]
    dy = Y - my[:, :, None, None]
    vx = np.tensordot(dx * dx, w, axes=([2, 3], [0, 1]))
    vy = np.tensordot(dy * dy, w, axes=([2, 3], [0, 1]))
    cxy = np.tensordot(dx * dy, w, axes=([2, 3], [0, 1]))
    m = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return float(m.mean())


def cnr(x: np.ndarray, hot: np.ndarray, background: np.ndarray) -> float:
    """(mean over hot - mean over background) / population std over background."""
    x = np.asarray(x, np.float64)
    b = x[background]
    d, sd = x[hot].mean() - b.mean(), b.std()
    if sd == 0.0:  # a flat background (the true activity itself): the contrast's sign as an infinity
        return float(np.sign(d) * np.inf) if d != 0.0 else float("nan")
    return float(d / sd)


def psnr(x: np.ndarray, ref: np.ndarray) -> float:
    x = np.asarray(x, np.float64)
    y = np.asarray(ref, np.float64)
    mse = float(np.mean((x - y) ** 2))
    return float("inf") if mse == 0.0 else float(10.0 * np.log10(y.max() ** 2 / mse))


def regions(activity: np.ndarray, background: float = 1.0, hot: float = 4.0):
    """Hot region: pixels wholly inside a hot disk; background: brain pixels that no disk touches."""
    a = np.asarray(activity, np.float64)
    return np.abs(a - hot) < 1e-6, np.abs(a - background) < 1e-6


def scores(F, activity):
    hot, bg = regions(activity)
    return {"ssim": ssim(F, activity), "cnr": cnr(F, hot, bg), "psnr": psnr(F, activity)}


def run_case(ctx: Context, d, k: int, n_iter: int, cycles: int, gradient, seed: int, return_images: bool = False):
    """Scores of case k; with return_images also the three reconstructions ("images": boac, nac,
    ac_true_head, in activity units) and the BOAC head parameters' float32 values ("theta_boac_f32")."""
    n, na, nb, nt = (int(v) for v in d[f"case{k}_geometry"])
    g = Geometry(n, na, nb, nt, float(d[f"case{k}_pixel"]))
    dev = ctx.device
    meas = torch.as_tensor(d[f"case{k}_meas"].astype(np.float32), device=dev)
    truth = np.asarray(d[f"case{k}_theta"], np.float64)
    act = np.asarray(d[f"case{k}_activity"], np.float64)
    dr = float(d[f"case{k}_delta_r"])
    t0 = time.perf_counter()
    bo = BOAC(ctx, g, meas, delta_r=dr, n_iter=n_iter, seed=seed + k, gradient=gradient)
    th, J = bo.run(cycles)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    cand = torch.as_tensor(np.stack([th, truth]).astype(np.float32), device=dev)
    Jc, F, _ = ctx.objective(g, meas, cand, dr, n_iter, want_image=True)
    # reconstructions carry the simulation's count scale; compare in the phantom's activity units:
    # kappa = total counts / total projection of the true activity through the true attenuation
    mu_true = ctx.rasterize_mu(g, cand[1:2].contiguous(), dr)
    y_true = ctx.project(g, mu_true, torch.as_tensor(act[None].astype(np.float32), device=dev))
    kappa = float(meas.double().sum() / y_true.double().sum())
    F = F.double().cpu().numpy() / kappa
    F_nac = ctx.mlem(g, torch.zeros((1, n, n), device=dev), meas, n_iter)[0].double().cpu().numpy() / kappa
    out = {"case": "ABC"[k] if k < 3 else str(k), "theta_true": truth.tolist(), "theta_boac": th.tolist(),
           "J_boac": float(Jc[0]), "J_true_head": float(Jc[1]), "bo_seconds": round(secs, 3), "kappa": kappa,
           "evaluations": int(sum(len(c.J) for c in bo.cycles)),
           "boac": scores(F[0], act), "nac": scores(F_nac, act), "ac_true_head": scores(F[1], act)}
    if return_images:
        out["images"] = {"boac": F[0], "nac": F_nac, "ac_true_head": F[1]}
        out["theta_boac_f32"] = cand[0].double().cpu().numpy()
    return out


def table(rows) -> str:
    lines = ["| Case | Method | SSIM | CNR | PSNR (dB) |", "|---|---|---|---|---|"]
    for r in rows:
        for name, key in (("MLEM-BOAC", "boac"), ("MLEM-NAC", "nac"), ("MLEM-AC (true head)", "ac_true_head")):
            s = r[key]
            lines.append(f"| {r['case']} | {name} | {s['ssim']:.3f} | {s['cnr']:.2f} | {s['psnr']:.2f} |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--inputs", required=True)
    ap.add_argument("--n-iter", type=int, default=30)
    ap.add_argument("--cycles", type=int, default=8)
    ap.add_argument("--gradient", default="envelope", choices=["none", "envelope", "unrolled"])
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args()
    d = np.load(a.inputs)
    with Context(0) as ctx:
        rows = [run_case(ctx, d, k, a.n_iter, a.cycles, None if a.gradient == "none" else a.gradient, a.seed)
                for k in range(int(d["n_cases"]))]
    print(table(rows))
    print(json.dumps({"study": rows}))


if __name__ == "__main__":
    main()
