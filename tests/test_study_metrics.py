"""The study's image-quality scores (vectorised, in the package) against the oracle's loop
definitions on seeded images; and the region masks of the phantom family. No GPU."""
import numpy as np
import pytest

import oracle.metrics as om
from paper_2109_11920_amd import study


@pytest.mark.parametrize("shape", [(11, 11), (24, 30), (40, 40)])
def test_scores_match_oracle(shape):
    rng = np.random.default_rng(shape[0])
    ref = rng.uniform(0, 4, size=shape)
    x = ref + rng.normal(scale=0.3, size=shape)
    assert study.ssim(x, ref) == pytest.approx(om.ssim(x, ref), rel=1e-12)
    assert study.psnr(x, ref) == pytest.approx(om.psnr(x, ref), rel=1e-13)
    hot = ref > 3
    bg = ref < 1.5
    assert study.cnr(x, hot, bg) == pytest.approx(om.cnr(x, hot, bg), rel=1e-12)


def test_regions_of_the_phantom_family():
    import os
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "study_cases.npz"))
    for k in range(int(d["n_cases"])):
        a = d[f"case{k}_activity"].astype(np.float64)
        hot, bg = study.regions(a)
        assert hot.sum() > 20 and bg.sum() > 1000 and not np.any(hot & bg)
        # the true activity scores perfectly against itself
        s = study.scores(a, a)
        assert s["ssim"] == pytest.approx(1.0, abs=1e-12) and np.isinf(s["psnr"])
