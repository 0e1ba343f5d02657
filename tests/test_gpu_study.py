"""The BOAC-vs-NAC study on one synthetic case (72 angles, oversampled data): BOAC's reconstruction
scores above the one without attenuation correction, as in the paper's Table I."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_boac_beats_nac_on_case_a():
    from paper_2109_11920_amd import study
    from paper_2109_11920_amd.api import Context
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "study_cases.npz"))
    with Context(0) as ctx:
        r = study.run_case(ctx, d, 0, n_iter=20, cycles=4, gradient="envelope", seed=0)
    print(study.table([r]))
    for k in ("boac", "nac", "ac_true_head"):
        assert all(np.isfinite(v) for v in r[k].values())
    assert r["boac"]["psnr"] > r["nac"]["psnr"] + 5
    assert r["boac"]["ssim"] > r["nac"]["ssim"]
    assert r["J_boac"] <= r["J_true_head"] + 0.01 * abs(r["J_true_head"])
