"""Benchmark: batched BOAC candidate evaluation on one MI355X.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3]

One step = one pass of the whole hot path over the 256-candidate batch on the 128 x 128, 128-angle,
128-bin slice (5e5 counts): rasterise mu(theta) for every candidate, build its attenuation tensor,
sensitivity image, 30 MLEM iterations, then the Poisson negative log-likelihood. value = candidates x
MLEM iterations per second (whole job; inputs resident in HBM before the timed region).

The same JSON line also carries: the unbatched GPU path (one candidate per call), the objective +
gradient rate on the 64-candidate adjoint workload (20 iterations, checkpoint every 5), the roofline
of the dominant kernel from HIP events recorded by the library around each launch during the timed
steps, and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLEM iters/s × candidates at 128², 128 angles; batched vs plain; obj+grad evals/s"
HBM_PEAK_GBS = 8000.0
DELTA_R = 0.8


def source_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2109_11920_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"fwd": ["kernels_ray.hip", "device_common.h", "launch.h"],
                  "back": ["kernels_back.hip", "device_common.h", "launch.h"],
                  "adj_ray": ["kernels_ray.hip", "device_common.h", "launch.h"]}


def read_traffic(kind, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_digest(KERNEL_SOURCES[kind]):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_name(kind, C):
    """Name of the kernel the plan cache selects for the 128^3 batch (the library picks the same)."""
    if kind == "fwd":
        return "k_fwd<RATIO>"
    try:
        with open(os.path.join(ROOT, "paper_2109_11920_amd", "tune_cache.json")) as f:
            e = json.load(f).get(f"back:128x128x128x128:{C}:0")
    except (OSError, ValueError):
        e = None
    if e and len(e) >= 5 and e[4] == 2:
        # 128 angles: the attenuation tensor holds half of them (opposed-ray pairing)
        if os.environ.get("BOAC_OPPOSED_RAYS", "1") != "0":
            return f"k_back_col4<{e[2]}, true, true> (MLEM gather, opposed-ray pairing)"
        return f"k_back_col4<{e[2]}, true, false> (MLEM gather)"
    if e and len(e) >= 5 and e[4]:
        return f"k_back_slid<{e[2]}, true> (MLEM gather)"
    if e:
        return f"k_back<{e[2]}, {e[0]}, {e[1]}, 1> (MLEM gather)"
    return "k_back (MLEM gather)"


_WORKER = {}


def _oracle_worker_init(S):
    import numpy as np

    import oracle
    og = oracle.Geometry(128, 128, 128, 128, 0.2)
    oracle.sampling_matrix(og)  # geometry setup outside the timed sample
    _WORKER.update(og=og, S=np.asarray(S, np.float64))


def _oracle_worker_eval(args):
    import oracle
    theta, n_iter = args
    return oracle.evaluate(_WORKER["og"], _WORKER["S"], theta, DELTA_R, n_iter)[0]


def cpu_baseline(workload_S, n_cand, n_iter, workers):
    """The FP64 oracle as it stands on a bounded sample of the batch: one thread, then one process per
    host core (candidate-parallel, the core count granted to this job)."""
    import multiprocessing as mp

    import numpy as np

    import oracle
    import synth
    og = oracle.Geometry(128, 128, 128, 128, 0.2)
    th = synth.draw_candidates(synth.candidate_stream(0), 256)
    S = workload_S.astype(np.float64)
    oracle.sampling_matrix(og)  # geometry setup outside the timed sample
    t0 = time.perf_counter()
    for c in range(n_cand):
        oracle.evaluate(og, S, th[c], DELTA_R, n_iter)
    dt = time.perf_counter() - t0
    single = n_cand * n_iter / dt
    # all cores: one process per core (fresh interpreters), each evaluating whole candidates
    n_par = 4 * workers
    with mp.get_context("spawn").Pool(workers, initializer=_oracle_worker_init, initargs=(S,)) as pool:
        pool.map(_oracle_worker_eval, [(th[c], 1) for c in range(workers)], chunksize=1)   # warm every worker
        t1 = time.perf_counter()
        pool.map(_oracle_worker_eval, [(th[c], n_iter) for c in range(n_par)], chunksize=1)
        dt_par = time.perf_counter() - t1
    par = n_par * n_iter / dt_par
    return {"value": round(par, 2), "unit": "cand·it/s", "cores": workers, "kind": "oracle",
            "host_cores": os.cpu_count(),
            "sample": f"{n_par} of the 256 candidates, {n_iter} MLEM iterations + objective each, FP64 NumPy/"
                      f"SciPy, one single-threaded process per core on {workers} cores, {dt_par:.1f} s",
            "single_thread": {"value": round(single, 2), "unit": "cand·it/s", "cores": 1,
                              "sample": f"{n_cand} candidates on one thread, {dt:.1f} s"}}


def full_tensor_bytes(n, na, nb, nt, K, paired):
    """Algorithmic HBM bytes of one candidate's evaluation (K MLEM iterations + objective):
    (2K+3) V + (4K+3) I + (3K+1) Y with V the attenuation tensor, I an image, Y a sinogram (FP32);
    with opposed-ray pairing the tensor is half the angles plus exp(-T) per held ray."""
    V = 4.0 * na * nb * nt
    I = 4.0 * n * n
    Y = 4.0 * na * nb
    if paired:
        V = V / 2 + Y / 2
    return (2 * K + 3) * V + (4 * K + 3) * I + (3 * K + 1) * Y


def gather_full_tensor_bytes(n, na, nb, nt):
    """Algorithmic bytes of one candidate's MLEM backprojection-and-update (V + Y + 3I, full tensor)."""
    return 4.0 * (na * nb * nt + na * nb + 3 * n * n)


def plain_line(ctx, g, S, theta, dev, reps=10):
    """The plain GPU method, unbatched: one candidate (the true head), 50 MLEM iterations + objective on
    the 128^2 / 128-angle slice, with the roofline of its dominant kernel from per-launch HIP events."""
    import numpy as np
    import torch

    cand = torch.as_tensor(np.asarray(theta, np.float32)[None], device=dev).contiguous()
    K = 50
    obj = torch.empty(1, device=dev)
    status = torch.empty(1, device=dev, dtype=torch.int32)
    stream = torch.cuda.current_stream(dev)
    for _ in range(2):
        ctx.objective(g, S, cand, DELTA_R, K, obj=obj, status=status)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        ctx.objective(g, S, cand, DELTA_R, K, obj=obj, status=status)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert bool(torch.isfinite(obj).all())
    ctx.reset_stats()
    ctx.set_profiling(True)
    for _ in range(reps):
        ctx.objective(g, S, cand, DELTA_R, K, obj=obj, status=status)
    torch.cuda.synchronize()
    ks = {k: ctx.kernel_stats(k) for k in ("att", "fwd", "back", "reduce")}
    ctx.set_profiling(False)
    dom = max(("fwd", "back"), key=lambda k: ks[k][1])
    cnt, kms, by = ks[dom]
    avg = kms / max(cnt, 1)
    ach = by / max(cnt, 1) / (avg / 1e3) / 1e9
    paired = os.environ.get("BOAC_OPPOSED_RAYS", "1") != "0"
    step = full_tensor_bytes(128, 128, 128, 128, K, paired)
    return {"value": round(K / (ms / 1e3), 1), "unit": "cand·it/s", "ms_per_evaluation": round(ms, 3),
            "us_per_iteration": round(1e3 * ms / K, 2),
            "kernel_ms_per_evaluation": {k: round(v[1] / reps, 4) for k, v in ks.items() if v[0]},
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "avg_launch_ms": round(avg, 4),
                         "bytes_per_launch": by / max(cnt, 1),
                         "step_frac_paired_bytes": round(step / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
            "what": "plain_n128: one candidate (true head), 128^2, 128 angles, 50 MLEM iterations + objective, "
                    "one call (C = 1)"}


def paper72_line(ctx, dev, reps=5):
    """The paper's angular sampling: 128^2 at 0.2 cm, 72 angles over 360 deg, data simulated on a 2x
    finer grid; 256 candidates, 30 iterations + objective, same step as the main line."""
    import numpy as np
    import torch

    import synth
    from paper_2109_11920_amd.api import Geometry
    d = np.load(os.path.join(ROOT, "tests", "golden", "slice_n128_a72.npz"))
    w = synth.workload("paper72_n128")
    g = Geometry(128, 72, 128, 128, 0.2)
    S = torch.as_tensor(d["meas"].astype(np.float32), device=dev)
    cand = torch.as_tensor(synth.workload_candidates(w)[0].astype(np.float32), device=dev)
    ctx.objective(g, S, cand, DELTA_R, w.n_iter)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        J, _, _ = ctx.objective(g, S, cand, DELTA_R, w.n_iter)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"value": round(cand.shape[0] * w.n_iter / (ms / 1e3), 1), "unit": "cand·it/s", "ms_per_step": round(ms, 3),
            "finite": bool(torch.isfinite(J).all()),
            "what": "128^2, 72 angles x 128 bins, 2x-oversampled data, 256 candidates, 30 iterations + objective"}


def uneven_slices(dev):
    """The 48 slices of the uneven batch (measured data from tests/golden, seeded candidates)."""
    import numpy as np
    import torch

    import synth
    from paper_2109_11920_amd.api import Geometry, SliceBatch
    du = np.load(os.path.join(ROOT, "tests", "golden", "uneven48.npz"))
    wu = synth.workload("uneven48")
    cu = synth.workload_candidates(wu)
    slices = []
    for s in range(int(du["n_slices"])):
        n, na, nb, nt = (int(v) for v in du[f"s{s:02d}_geometry"])
        gs = Geometry(n, na, nb, nt, float(du[f"s{s:02d}_pixel"]))
        slices.append(SliceBatch.make(gs, torch.as_tensor(du[f"s{s:02d}_meas"].astype(np.float32), device=dev),
                                      torch.as_tensor(cu[s].astype(np.float32), device=dev), with_grad=True))
    return slices, wu


KINDS = ("raster", "att", "fwd", "back", "reduce", "adj_ray", "adj_pix", "other")
KIND_KERNELS = {"fwd": "forward projections (k_fwd, k_fwd_pair)", "back": "backprojection gathers (k_back_col4)",
                "adj_ray": "reverse ray sweeps (k_adj_sweep, k_tail)", "att": "attenuation builds"}


def uneven_serial(ctx, dev, slices, wu, replay_ms=None):
    """One eager evaluation of the uneven batch with its launches serialised (one stream lane) and timed
    one by one with HIP events: kernel time and the library's algorithmic bytes per kind, the roofline
    of the kind with the most time, and the whole batch's bytes over the replay time."""
    import torch
    old = os.environ.get("BOAC_BATCH_LANES")
    os.environ["BOAC_BATCH_LANES"] = "1"
    st = torch.cuda.Stream(dev)
    try:
        ctx.reset_stats()
        ctx.set_profiling(True)
        st.wait_stream(torch.cuda.current_stream(dev))  # calls on one context do not overlap
        with torch.cuda.stream(st):
            ctx.evaluate_batch(slices, DELTA_R, wu.n_iter, wu.ckpt_every)
        st.synchronize()
        ks = {k: ctx.kernel_stats(k) for k in KINDS}
    finally:
        ctx.set_profiling(False)
        if old is None:
            del os.environ["BOAC_BATCH_LANES"]
        else:
            os.environ["BOAC_BATCH_LANES"] = old
    per = {k: {"launches": c, "ms": round(ms, 2), "GB": round(by / 1e9, 3),
               "TB/s": round(by / (ms / 1e3) / 1e12, 3) if ms > 0 else None}
           for k, (c, ms, by) in ks.items() if c}
    dom = max(("fwd", "back", "adj_ray"), key=lambda k: ks[k][1])
    c, ms, by = ks[dom]
    avg = ms / c
    ach = by / c / (avg / 1e3) / 1e9
    total_by = sum(v[2] for v in ks.values())
    total_ms = sum(v[1] for v in ks.values())
    out = {"kernel_ms_serial": round(total_ms, 1), "per_kind": per,
           "roofline": {"bound": "hbm", "kernel": f"{dom}: {KIND_KERNELS[dom]}, all slices", "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "avg_launch_ms": round(avg, 4), "bytes_per_launch": by / c, "launches": c,
                        "traffic": read_traffic(dom, "uneven48"),
                        "what": "one eager evaluation, launches serialised on one stream and timed by HIP events; "
                                "bytes: the library's algorithmic count per launch (attenuation tensors of the held "
                                "angles, images and sinograms)"},
           "batch_bytes_GB": round(total_by / 1e9, 2)}
    if replay_ms:
        out["step_frac_model_bytes"] = round(total_by / (replay_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def uneven_line(ctx, dev, serial=True):
    """The 48-slice uneven batch: N 96-256, 64-256 angles, 32 candidates each, 40 iterations, objective
    + gradient (checkpoint every 5), one captured batch over concurrent stream lanes; times one replay,
    then (serial) one serialised eager evaluation for the per-kind roofline."""
    import torch
    slices, wu = uneven_slices(dev)
    ustream = torch.cuda.Stream(dev)
    ustream.wait_stream(torch.cuda.current_stream(dev))  # calls on one context do not overlap
    with torch.cuda.stream(ustream):
        ctx.evaluate_batch(slices, DELTA_R, wu.n_iter, wu.ckpt_every)   # runs eagerly, then captures
        ctx.evaluate_batch(slices, DELTA_R, wu.n_iter, wu.ckpt_every)   # graph replay (warm)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ustream)
        ctx.evaluate_batch(slices, DELTA_R, wu.n_iter, wu.ckpt_every)
        e1.record(ustream)
    ustream.synchronize()
    ums = e0.elapsed_time(e1)
    n_eval = sum(sb.cand.shape[0] for sb in slices)
    ok = all(bool(torch.isfinite(sb.obj).all()) and bool(torch.isfinite(sb.grad).all()) for sb in slices)
    return {"value": round(n_eval * wu.n_iter / (ums / 1e3), 1), "unit": "cand·it/s",
            "obj_grad_evals_per_s": round(n_eval / (ums / 1e3), 1), "ms_per_batch": round(ums, 2), "finite": ok,
            **({"serialised": uneven_serial(ctx, dev, slices, wu, ums)} if serial else {}),
            "what": "48 slices N in {96,128,192,256}, 64-256 angles, 32 candidates each, 40 iterations, "
                    "objective + gradient, checkpoint 5, one graph replay"}


def persistent_line(ctx, g, S, cand, K, dev, steps):
    """The batch schedules side by side: the 256-candidate batch and the 48-slice uneven batch, each as one
    persistent launch (device work queue, per-lane completion counters) against the stream-lane graph,
    both timed as graph replays on one stream."""
    import numpy as np
    import torch

    import synth
    from paper_2109_11920_amd.api import Geometry, SliceBatch
    C = cand.shape[0]
    out = {}
    stream = torch.cuda.Stream(dev)

    def timed(slices, k, ck, reps):
        stream.wait_stream(torch.cuda.current_stream(dev))  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.evaluate_batch(slices, DELTA_R, k, ck)   # eager run, then capture
            ctx.evaluate_batch(slices, DELTA_R, k, ck)   # replay (warm)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                ctx.evaluate_batch(slices, DELTA_R, k, ck)
            e1.record(stream)
        stream.synchronize()
        return e0.elapsed_time(e1) / reps

    sb = [SliceBatch(g, S, cand, torch.empty(C, device=dev), None, torch.empty(C, device=dev, dtype=torch.int32))]
    du = np.load(os.path.join(ROOT, "tests", "golden", "uneven48.npz"))
    wu = synth.workload("uneven48")
    cu = synth.workload_candidates(wu)
    us = []
    for s in range(int(du["n_slices"])):
        n, na, nb, nt = (int(v) for v in du[f"s{s:02d}_geometry"])
        gs = Geometry(n, na, nb, nt, float(du[f"s{s:02d}_pixel"]))
        us.append(SliceBatch.make(gs, torch.as_tensor(du[f"s{s:02d}_meas"].astype(np.float32), device=dev),
                                  torch.as_tensor(cu[s].astype(np.float32), device=dev), with_grad=True))
    for mode in ("lanes", "persistent"):
        ctx.set_batch_mode(mode)
        b_ms = timed(sb, K, 5, steps)
        J = sb[0].obj.clone()
        u_ms = timed(us, wu.n_iter, wu.ckpt_every, 1)
        out[mode] = {"batch256_ms_per_step": round(b_ms, 3), "batch256_cand_it_per_s": round(C * K / (b_ms / 1e3), 1),
                     "uneven48_ms_per_batch": round(u_ms, 2),
                     "uneven48_obj_grad_evals_per_s": round(sum(x.cand.shape[0] for x in us) / (u_ms / 1e3), 1)}
        out[mode]["_J"] = J
    ctx.set_batch_mode("lanes")
    d = out["persistent"].pop("_J") - out["lanes"].pop("_J")
    out["batch256_J_max_abs_diff"] = float(d.abs().max())
    out["what"] = ("graph replays on one stream: batch256_n128 (256 candidates, 30 iterations + objective) and "
                   "uneven48 (objective + gradient); persistent = one launch of one 1024-thread workgroup per CU "
                   "taking tasks from a device queue; lanes = concurrent stream lanes")
    return out


def bo_line(ctx, g, S, truth):
    """The BOAC outer loop on the 128^2 slice: 64 initial candidates, then cycles of 64 proposals (EI by
    chaotic search; with the envelope gradient, part of each batch is a line search along -grad J),
    30 MLEM iterations per candidate. Plain and gradient-aware loops from the same seed."""
    import numpy as np
    import torch

    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd.bo import BOAC, LENGTH_GRID
    J_true = float(ctx.objective(g, S, torch.as_tensor(truth[None].astype(np.float32), device=S.device)
                                 .contiguous(), DELTA_R, 30)[0][0])
    out = {"J_true_head": round(J_true, 3), "what": "64 initial + 5 cycles x 64 proposals, 30 MLEM iterations "
                                                    "each, EI by chaotic search on the GPU"}
    for name, grad in (("plain", None), ("envelope_grad", "envelope")):
        bo = BOAC(ctx, g, S, n_iter=30, n_init=64, batch=64, seed=0, gradient=grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bo.run(6)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        th, J = bo.best()
        tm = {k: round(sum(c.timings.get(k, 0.0) for c in bo.cycles), 1) for k in ("fit_ms", "acquire_ms",
                                                                                     "evaluate_ms")}
        out[name] = {"seconds": round(wall, 3), "evaluations": int(sum(len(c.J) for c in bo.cycles)),
                     "best_J": round(J, 3), "best_J_minus_true": round(J - J_true, 3),
                     "unit_box_distance_to_true": round(float(np.linalg.norm((th - truth) / (bo.hi - bo.lo))), 4),
                     "best_J_per_cycle": [round(float(min(x.J.min() for x in bo.cycles[:k + 1])), 2)
                                          for k in range(len(bo.cycles))], **tm,
                     "ei_queries": int(sum(c.timings.get("ei_queries", 0) for c in bo.cycles))}
    out["gp_ei_kernel"] = gp_kernel_line(ctx, S.device)
    return out


def gp_kernel_line(ctx, dev):
    """The acquisition kernels alone at a larger model: 512 observations, 65536 queries, FP64."""
    import numpy as np
    import torch

    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd.bo import LENGTH_GRID
    rng = np.random.default_rng(0)
    n, M = 512, 1 << 16
    U = rng.uniform(size=(n, 8))
    y = 1e5 + 300 * np.sum((U - 0.4) ** 2, axis=1)
    model = gp_fit(U, y, LENGTH_GRID)
    q = torch.as_tensor(rng.uniform(size=(M, 8)), device=dev)
    ctx.gp_ei(model, q, float(y.min()), 0.0)
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.set_profiling(True)
    reps = 5
    for _ in range(reps):
        ctx.gp_ei(model, q, float(y.min()), 0.0)
    torch.cuda.synchronize()
    cnt, ms, _ = ctx.kernel_stats("gp")
    ctx.set_profiling(False)
    ms /= max(cnt, 1)
    flops = M * n * (n + 1 + 3 * 8 + 4)   # triangular product (FMA = 2), distances, mean and norm
    return {"n": n, "queries": M, "ms": round(ms, 3), "tflops": round(flops / ms / 1e9, 2),
            "bound": "alu", "peak_tflops": 78.6, "frac": round(flops / ms / 1e9 / 78.6, 4),
            "what": "k* + blocked triangular product (FP64 matrix cores) + EI, FP64 (exp not counted)"}


def grad_lines(ctx, g, S, dev, steps):
    """Objective + gradient on the 64-candidate draw (20 iterations, checkpoint every 5): the unrolled
    gradient against the forward evaluation, and the envelope gradient with dJ/d(dR)."""
    import numpy as np
    import torch

    import synth
    stream = torch.cuda.current_stream(dev)
    # ---- objective + gradient: 64 candidates, 20 iterations, checkpoint every 5
    wg = synth.workload("grad64_n128")
    cg = torch.as_tensor(synth.workload_candidates(wg)[0].astype(np.float32), device=dev)
    Kg = wg.n_iter
    ctx.objective_grad(g, S, cg, DELTA_R, Kg, wg.ckpt_every)
    ctx.objective(g, S, cg, DELTA_R, Kg)
    torch.cuda.synchronize()
    reps = max(2, steps // 2)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        _, G, st = ctx.objective_grad(g, S, cg, DELTA_R, Kg, wg.ckpt_every)
    e1.record(stream)
    for _ in range(reps):
        ctx.objective(g, S, cg, DELTA_R, Kg)
    e2.record(stream)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(G).all())
    grad_ms = e0.elapsed_time(e1) / reps
    fwd_ms = e1.elapsed_time(e2) / reps
    out = {}
    out["grad"] = {"value": round(cg.shape[0] / (grad_ms / 1e3), 1), "unit": "obj+grad evals/s",
                   "ms_per_batch": round(grad_ms, 3), "forward_ms_per_batch": round(fwd_ms, 3),
                   "grad_over_forward": round(grad_ms / fwd_ms, 3),
                   "what": "64 candidates, 20 iterations, checkpoint every 5"}

    # ---- envelope gradient (reconstruction held fixed) with dJ/d(dR), same 64 candidates
    ctx.objective_grad_ex(g, S, cg, DELTA_R, Kg, wg.ckpt_every, mode="envelope")
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        _, Ge, _ = ctx.objective_grad_ex(g, S, cg, DELTA_R, Kg, wg.ckpt_every, mode="envelope")
    e1.record(stream)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Ge).all())
    env_ms = e0.elapsed_time(e1) / reps
    out["grad_envelope"] = {"value": round(cg.shape[0] / (env_ms / 1e3), 1), "unit": "obj+grad evals/s",
                            "ms_per_batch": round(env_ms, 3), "grad_over_forward": round(env_ms / fwd_ms, 3),
                            "what": "64 candidates, 20 iterations, envelope gradient (F^K held fixed) "
                                    "with dJ/d(dR)"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-cands", type=int, default=32)
    ap.add_argument("--no-uneven", action="store_true", help="skip the 48-slice uneven batch line")
    ap.add_argument("--only-main", action="store_true", help="timed batch only (for profiler runs)")
    ap.add_argument("--no-bo", action="store_true", help="skip the BOAC outer-loop line")
    ap.add_argument("--only-grad", action="store_true", help="the gradient lines only (for profiler runs)")
    ap.add_argument("--only-gp", action="store_true", help="the acquisition-kernel line only (for profiler runs)")
    ap.add_argument("--only-paper72", action="store_true", help="the 72-angle line only (for profiler runs)")
    ap.add_argument("--only-uneven", action="store_true",
                    help="the uneven batch's replay only, without the serialised pass (for profiler runs)")
    ap.add_argument("--only-bo", action="store_true", help="the BOAC outer-loop line only")
    ap.add_argument("--only-uneven-serial", action="store_true",
                    help="one serialised eager evaluation of the uneven batch (for profiler runs)")
    ap.add_argument("--only-schedules", action="store_true", help="the batch-schedule comparison only")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run one 1 GiB device-to-device copy (counter calibration for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: candidates are independent and this build has no multi-GPU "
              "path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    # host cores granted to this job (OMP_NUM_THREADS states the share where it is set), for the
    # all-cores oracle leg: one single-threaded process per core
    workers = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1))
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"   # every oracle process is single-threaded

    import numpy as np
    import torch

    import synth
    from paper_2109_11920_amd.api import Context, Geometry, SliceBatch

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    d = np.load(os.path.join(ROOT, "tests", "golden", "slice_n128.npz"))
    S_np = d["meas"]
    g = Geometry(128, 128, 128, 128, 0.2)
    S = torch.as_tensor(S_np.astype(np.float32), device=dev)
    w = synth.workload("batch256_n128")
    cand = torch.as_tensor(synth.workload_candidates(w)[0].astype(np.float32), device=dev)
    C, K = cand.shape[0], w.n_iter
    ctx = Context(0)
    stream = torch.cuda.current_stream(dev)
    if args.copy_calib:
        src = torch.ones(1 << 28, device=dev)          # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only_schedules:
        print(json.dumps({"batch_schedules": persistent_line(ctx, g, S, cand, K, dev, max(3, args.steps // 2))}),
              flush=True)
        ctx.close()
        return
    if args.only_uneven_serial:
        slices, wu = uneven_slices(dev)
        uneven_serial(ctx, dev, slices, wu)   # the same pass once untimed: sizes scratch, uploads tables
        print(json.dumps({"uneven48_serialised": uneven_serial(ctx, dev, slices, wu)}), flush=True)
        ctx.close()
        return
    if args.only_uneven or args.only_gp or args.only_grad or args.only_bo or args.only_paper72:
        out = {}
        if args.only_paper72:
            out["paper72"] = paper72_line(ctx, dev)
        if args.only_bo:
            import numpy as np
            d = np.load(os.path.join(ROOT, "tests", "golden", "slice_n128.npz"))
            out["bo"] = bo_line(ctx, g, S, np.asarray(d["theta"], dtype=np.float64))
        if args.only_uneven:
            # the replayed batch alone (the serialised pass has a mode of its own, --only-uneven-serial)
            out["uneven48"] = uneven_line(ctx, dev, serial=False)
        if args.only_grad:
            out.update(grad_lines(ctx, g, S, dev, args.steps))
        if args.only_gp:
            out["gp_ei_kernel"] = gp_kernel_line(ctx, dev)
        print(json.dumps(out), flush=True)
        ctx.close()
        return
    # ---- main timed region: the 256-candidate batch, eager launches with per-kernel HIP events
    obj = torch.empty(C, device=dev)
    status = torch.empty(C, device=dev, dtype=torch.int32)
    for _ in range(args.warmup):
        ctx.objective(g, S, cand, DELTA_R, K, obj=obj, status=status)
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        ctx.objective(g, S, cand, DELTA_R, K, obj=obj, status=status)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_profiling(False)
    step_ms = ev0.elapsed_time(ev1) / args.steps
    kstats = {k: ctx.kernel_stats(k) for k in ("raster", "att", "fwd", "back", "reduce", "adj_ray", "adj_pix",
                                                "other")}
    J = obj.cpu().numpy()
    assert np.all(np.isfinite(J)) and int((status.cpu().numpy() & 3).max()) == 0
    value = C * K / (step_ms / 1e3)

    dom = max(("fwd", "back"), key=lambda k: kstats[k][1])
    cnt, ms, by = kstats[dom]
    avg_ms = ms / max(cnt, 1)
    bytes_per_launch = by / max(cnt, 1)
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    paired = os.environ.get("BOAC_OPPOSED_RAYS", "1") != "0"
    full_launch = C * gather_full_tensor_bytes(128, 128, 128, 128)
    step_full = C * full_tensor_bytes(128, 128, 128, 128, K, False)
    step_paired = C * full_tensor_bytes(128, 128, 128, 128, K, paired)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(dom, "batch256_n128"),
            "kernel": kernel_name(dom, C), "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": bytes_per_launch,
            "launches": cnt,
            "bytes_convention": "achieved/frac: the bytes this kernel must move as built (with opposed-ray "
                                "pairing the held half of the attenuation tensor plus exp(-T) per ray, the "
                                "ratio sinogram, F and s read, F written); frac_full_tensor_bytes: the full-tensor "
                                "count V + Y + 3I per candidate over the same time",
            "frac_full_tensor_bytes": round(full_launch / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "step": {"full_tensor_bytes": step_full, "paired_bytes": step_paired,
                     "frac_full_tensor_bytes": round(step_full / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "frac_paired_bytes": round(step_paired / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "what": "whole step: (2K+3) V + (4K+3) I + (3K+1) Y per candidate over the step time; "
                             "paired: V -> V/2 + exp(-T) per held ray"}}
    kernel_ms = {k: round(v[1] / args.steps, 3) for k, v in kstats.items() if v[0]}

    out = {"metric": METRIC, "value": round(value, 1), "unit": "cand·it/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "batch256_n128", "image": 128, "pixel_cm": 0.2, "angles": 128, "bins": 128,
                      "samples": 128, "counts": 5e5, "candidates": C, "mlem_iters": K,
                      "parallelism": "single-gpu"},
           "roofline": roof, "kernel_ms_per_step": kernel_ms}

    if not args.only_main:
        # ---- the same step replayed from a captured HIP graph
        gstream = torch.cuda.Stream(dev)
        sb = [SliceBatch(g, S, cand, torch.empty(C, device=dev), None, torch.empty(C, device=dev, dtype=torch.int32))]
        gstream.wait_stream(torch.cuda.current_stream(dev))  # calls on one context do not overlap
        with torch.cuda.stream(gstream):
            ctx.evaluate_batch(sb, DELTA_R, K)
            ctx.evaluate_batch(sb, DELTA_R, K)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(gstream)
            for _ in range(args.steps):
                ctx.evaluate_batch(sb, DELTA_R, K)
            e1.record(gstream)
        gstream.synchronize()
        graph_ms = e0.elapsed_time(e1) / args.steps
        assert torch.equal(sb[0].obj, obj)
        out["graph_ms_per_step"] = round(graph_ms, 3)

        # ---- unbatched GPU path: one candidate per call, same kernels, 30 iterations
        n_plain = 16
        o1 = torch.empty(1, device=dev)
        s1 = torch.empty(1, device=dev, dtype=torch.int32)
        ctx.objective(g, S, cand[:1].contiguous(), DELTA_R, K, obj=o1, status=s1)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        singles = [cand[c:c + 1].contiguous() for c in range(n_plain)]
        e0.record(stream)
        for c in range(n_plain):
            ctx.objective(g, S, singles[c], DELTA_R, K, obj=o1, status=s1)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_rate = n_plain * K / (e0.elapsed_time(e1) / 1e3)
        out["plain"] = {"value": round(plain_rate, 1), "unit": "cand·it/s",
                        "what": f"{n_plain} candidates, one call each (C=1), {K} iterations + objective"}
        out["batched_over_plain"] = round(value / plain_rate, 2)

        out.update(grad_lines(ctx, g, S, dev, args.steps))
        out["plain_n128"] = plain_line(ctx, g, S, np.asarray(d["theta"], dtype=np.float64), dev)

    if not args.only_main:
        out["paper72"] = paper72_line(ctx, dev)

    if not args.only_main and not args.no_uneven:
        out["uneven48"] = uneven_line(ctx, dev)
        out["batch_schedules"] = persistent_line(ctx, g, S, cand, K, dev, max(3, args.steps // 2))

    if not args.only_main and not args.no_bo:
        out["bo"] = bo_line(ctx, g, S, np.asarray(d["theta"], dtype=np.float64))

    if not args.no_cpu and not args.only_main:
        out["cpu_baseline"] = cpu_baseline(S_np, args.cpu_cands, K, workers)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
