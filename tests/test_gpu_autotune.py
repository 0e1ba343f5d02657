"""The launch-plan autotuner end to end on the GPU: it times every configuration of the one-candidate
64 x 64 workload, writes a plan cache, and a context reading that cache evaluates the workload to the
parity gates of the default plans and of the oracle."""
import json

import numpy as np
import pytest

from gpu_helpers import TOL, geom_pair, make_slice, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotuner_writes_a_cache_the_library_uses(tmp_path):
    import synth
    from paper_2109_11920_amd.api import Context, Geometry
    from paper_2109_11920_amd.autotune import key, tune_workload
    cache = tune_workload("smoke_n64", {}, log=lambda m: None)
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(cache))
    w = synth.workload("smoke_n64")
    sl = w.slices[0]
    g = Geometry(sl.n, sl.n_angles, sl.n_bins, sl.n_samples, sl.pixel)
    C = w.n_cand
    for kind, extra in (("ray", 1), ("back", 0)):
        assert key(kind, g, C, extra) in cache, (kind, sorted(cache))
    _, og = geom_pair(sl.n, sl.n_angles, sl.n_bins, sl.n_samples, pixel=sl.pixel)
    S, _ = make_slice(og, seed=51)
    th = synth.workload_candidates(w)[0]
    meas = torch.as_tensor(S, dtype=torch.float32, device="cuda")
    cand = torch.as_tensor(th.astype(np.float32), device="cuda")
    with Context(0, tune_cache=str(path)) as tuned, Context(0) as default:
        Jt, Ft, _ = tuned.objective(g, meas, cand, 0.8, 5, want_image=True)
        Jd, Fd, _ = default.objective(g, meas, cand, 0.8, 5, want_image=True)
    report("tuned vs default plans J", Jt.cpu().numpy(), Jd.cpu().numpy(), 1e-6)
    report("tuned vs default plans F^K", Ft.cpu().numpy(), Fd.cpu().numpy(), 1e-6)
    Jr = oracle.evaluate(og, S, np.asarray(th[0], np.float64), 0.8, 5)[0]
    report("tuned plans J vs oracle", Jt[:1].cpu().numpy(), np.array([Jr]), TOL)
