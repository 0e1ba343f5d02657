"""Autotuner for libboac launch plans.

For each workload shape it times the candidate launch configurations of the ray kernels (threads per
workgroup x rays per thread) and of the pixel-tile backprojection (tile shape x candidates per
workgroup) on the current GPU, using the library's own per-launch HIP-event instrumentation, and
writes the winners to the plan cache the library reads at context creation (tune_cache.json next to
this file by default):

    python -m paper_2109_11920_amd.autotune [--out PATH] [--workloads batch256_n128,grad64_n128,...]

The committed cache holds the default workloads, the 72-angle slice (--workloads paper72_n128) and
every slice shape of uneven48 (--workloads uneven48).

Keys follow the library: "ray:<n>x<na>x<nb>x<nt>:<C>:<image components>" -> [block, rays per thread,
paired forward projection (one-component entries)]
and "back:<n>x<na>x<nb>x<nt>:<C>:0" -> [tile width, tile height, candidates per workgroup, XCD remap,
slid-block kernel]. A slid-block entry the geometry does not admit falls back to the library's default.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")

RAY_CONFIGS = [(256, 1), (256, 2), (256, 4), (512, 1), (512, 2), (512, 4), (1024, 1), (1024, 2), (1024, 4), (768, 1),
               (768, 2)]
# (tile width, tile height, candidates per workgroup, slid-block kernel: 0 general, 1 slot staging,
# 2 column-group staging)
BACK_CONFIGS = [(16, 16, 1, 0), (16, 16, 2, 0), (16, 16, 4, 0), (16, 16, 8, 0), (32, 16, 2, 0), (32, 16, 4, 0),
                (32, 32, 2, 0), (16, 16, 1, 1), (16, 16, 2, 1), (16, 16, 4, 1), (16, 16, 8, 1), (16, 16, 1, 2),
                (16, 16, 2, 2), (16, 16, 4, 2), (16, 16, 8, 2)]


def key(kind, g, C, extra):
    return f"{kind}:{g.n}x{g.n_angles}x{g.n_bins}x{g.n_samples}:{C}:{extra}"


def _time(geom, meas, cand, entries, kind, n_iter, grad=False, reps=2):
    import torch

    from .api import Context
    fd, path = tempfile.mkstemp(suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(entries, f)
    try:
        ctx = Context(0, tune_cache=path)
        run = (lambda: ctx.objective_grad(geom, meas, cand, 0.8, n_iter, 5)) if grad else \
            (lambda: ctx.objective(geom, meas, cand, 0.8, n_iter))
        run()
        torch.cuda.synchronize()
        ctx.reset_stats()
        ctx.set_profiling(True)
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        cnt, ms, _ = ctx.kernel_stats(kind)
        ctx.close()
        return ms / max(cnt, 1)
    finally:
        os.unlink(path)


def tune_workload(name: str, cache: dict, log=print):
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import synth

    from .api import Geometry
    w = synth.workload(name)
    cands = synth.workload_candidates(w)
    seen = set()
    for s, sl in enumerate(w.slices):
        g = Geometry(sl.n, sl.n_angles, sl.n_bins, sl.n_samples, sl.pixel)
        shape = (sl.n, sl.n_angles, sl.n_bins, sl.n_samples, w.n_cand)
        if shape in seen:
            continue
        seen.add(shape)
        rng = np.random.default_rng(s)
        # timing does not depend on the data: a smooth positive sinogram of the right shape
        meas = torch.as_tensor(rng.poisson(20.0, (sl.n_angles, sl.n_bins)).astype(np.float32), device="cuda")
        cand = torch.as_tensor(cands[s].astype(np.float32), device="cuda")
        C = cand.shape[0]
        K = 2
        grad = w.ckpt_every > 0
        best = None
        for pair in ((0, 1) if C >= 2 else (0,)):
            for blk, rpt in RAY_CONFIGS:
                e = dict(cache)
                e[key("ray", g, C, 1)] = [blk, rpt, pair]
                t = _time(g, meas, cand, e, "fwd", K)
                log(f"[tune] {name} {shape} ray block={blk} rpt={rpt} pair={pair}: {t * 1e3:.1f} us/launch")
                if best is None or t < best[0]:
                    best = (t, [blk, rpt, pair])
        cache[key("ray", g, C, 1)] = best[1]
        if grad:
            best = None
            for blk, rpt in RAY_CONFIGS:
                e = dict(cache)
                e[key("ray", g, C, 2)] = [blk, rpt]
                t = _time(g, meas, cand, e, "adj_ray", K, grad=True)
                log(f"[tune] {name} {shape} pair-ray block={blk} rpt={rpt}: {t * 1e3:.1f} us/launch")
                if best is None or t < best[0]:
                    best = (t, [blk, rpt])
            cache[key("ray", g, C, 2)] = best[1]
        best = None
        for tw, th, cg, slid in BACK_CONFIGS:
            if cg > C:
                continue
            e = dict(cache)
            e[key("back", g, C, 0)] = [tw, th, cg, 1, slid]
            t = _time(g, meas, cand, e, "back", K)
            log(f"[tune] {name} {shape} back tile={tw}x{th} cg={cg} slid={slid}: {t * 1e3:.1f} us/launch")
            if best is None or t < best[0]:
                best = (t, [tw, th, cg, 1, slid])
        remap_t = {}
        for remap in (0, 1):
            cfg = best[1][:3] + [remap, best[1][4]]
            e = dict(cache)
            e[key("back", g, C, 0)] = cfg
            t = _time(g, meas, cand, e, "back", K)
            log(f"[tune] {name} {shape} back tile={cfg[0]}x{cfg[1]} cg={cfg[2]} slid={cfg[4]} xcd_remap={remap}: "
                f"{t * 1e3:.1f} us/launch")
            remap_t[remap] = (t, cfg)
        # a candidate group's tiles on one XCD share its samples in that XCD's L2 (fewer HBM bytes: 0.98x
        # against 1.51x the algorithmic count on the 72-angle batch), so the remap stays unless running
        # without it is clearly faster; near-ties are timing noise
        best = remap_t[0] if remap_t[0][0] < 0.98 * remap_t[1][0] else remap_t[1]
        cache[key("back", g, C, 0)] = best[1]
        log(f"[tune] {name} {shape} -> ray {cache[key('ray', g, C, 1)]} back {best[1]}")
    return cache


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--workloads", default="batch256_n128,grad64_n128,plain_n128")
    a = ap.parse_args()
    cache = {}
    if os.path.exists(a.out):
        cache = json.load(open(a.out))
    for name in a.workloads.split(","):
        cache = tune_workload(name.strip(), cache, log=lambda m: print(m, flush=True))
        with open(a.out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    print("wrote", a.out)


if __name__ == "__main__":
    main()
