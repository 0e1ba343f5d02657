"""The BOAC-vs-NAC study on one synthetic case (72 angles, oversampled data): BOAC's reconstruction
scores above the one without attenuation correction, as in the paper's Table I, and the study's three
reconstructions and their scores equal the oracle's (MLEM with mu = 0 for NAC, with the true head and
with the BOAC head for AC) to the parity gates."""
import os

import numpy as np
import pytest

from gpu_helpers import TOL, geom_pair, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_boac_beats_nac_on_case_a():
    import oracle.metrics as om
    from paper_2109_11920_amd import study
    from paper_2109_11920_amd.api import Context
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "study_cases.npz"))
    K = 20
    with Context(0) as ctx:
        r = study.run_case(ctx, d, 0, n_iter=K, cycles=4, gradient="envelope", seed=0, return_images=True)
    print(study.table([r]))
    for k in ("boac", "nac", "ac_true_head"):
        assert all(np.isfinite(v) for v in r[k].values())
    assert r["boac"]["psnr"] > r["nac"]["psnr"] + 5
    assert r["boac"]["ssim"] > r["nac"]["ssim"]
    assert r["J_boac"] <= r["J_true_head"] + 0.01 * abs(r["J_true_head"])

    # the reconstructions against the oracle's MLEM (same float32 inputs), in activity units
    n, na, nb, nt = (int(v) for v in d["case0_geometry"])
    _, og = geom_pair(n, na, nb, nt, float(d["case0_pixel"]))
    S = d["case0_meas"].astype(np.float32).astype(np.float64)
    dr = float(np.float32(d["case0_delta_r"]))
    act = np.asarray(d["case0_activity"], np.float64)
    truth = np.asarray(d["case0_theta"], np.float32).astype(np.float64)
    kappa = r["kappa"]
    F_nac = oracle.mlem(og, oracle.attenuation(og, np.zeros((n, n))), S, K) / kappa
    F_true = oracle.evaluate(og, S, truth, dr, K)[1] / kappa
    F_boac = oracle.evaluate(og, S, r["theta_boac_f32"], dr, K)[1] / kappa
    ref = {"nac": F_nac, "ac_true_head": F_true, "boac": F_boac}
    for name, Fr in ref.items():
        report(f"study case A {name} F^K", r["images"][name], Fr, TOL)
        hot, bg = study.regions(act)
        want = {"ssim": om.ssim(Fr, act), "cnr": om.cnr(Fr, hot, bg), "psnr": om.psnr(Fr, act)}
        for m, v in want.items():
            print(f"[parity] study case A {name} {m}: gpu {r[name][m]:.6f} oracle {v:.6f}", flush=True)
            assert r[name][m] == pytest.approx(v, rel=1e-3, abs=1e-4)
