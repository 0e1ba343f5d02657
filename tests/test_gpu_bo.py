"""The BOAC outer loop on the GPU: the initial design, surrogate cycles with batched proposals, the
gradient-aware line searches, and resuming from the journal (bit-identical continuation)."""
import os

import numpy as np
import pytest

from gpu_helpers import oracle, report, TOL

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_11920_amd.api import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problem(slice64):
    from paper_2109_11920_amd.api import Geometry
    g = Geometry(64, 64, 64, 64, 0.4)
    meas = torch.as_tensor(slice64["meas"].astype(np.float32), device="cuda")
    return g, meas, slice64


def _loop(ctx, problem, journal=None, gradient=None):
    from paper_2109_11920_amd.bo import BOAC
    g, meas, _ = problem
    return BOAC(ctx, g, meas, delta_r=DR, n_iter=10, n_init=24, batch=12, chains=512, n_global=6, n_local=10,
                centres=4, seed=3, gradient=gradient, journal=journal)


def test_bo_cycles_and_journal_resume(ctx, problem, tmp_path):
    from paper_2109_11920_amd.bo import BOAC
    a = _loop(ctx, problem, journal=str(tmp_path / "a.jsonl"))
    a.run(4)
    assert [c.index for c in a.cycles] == [0, 1, 2, 3]
    assert len(a.cycles[0].J) == 24 and all(len(c.J) == 12 for c in a.cycles[1:])
    th, J, _ = a.observations()
    assert np.all(np.isfinite(J))
    assert np.all(th >= a.lo - 1e-6) and np.all(th <= a.hi + 1e-6)
    assert all(c.max_ei >= 0 for c in a.cycles[1:])
    best_th, best_J = a.best()
    assert best_J <= a.cycles[0].J.min()
    for c in a.cycles[1:]:
        print(f"cycle {c.index}: best so far {min(x.J.min() for x in a.cycles[:c.index + 1]):.3f} "
              f"max EI/s {c.max_ei:.3e} length {c.length:.3g} {c.timings}")
    # the evaluator's objective for the incumbent against the oracle
    _, _, sl = problem
    og = oracle.Geometry(64, 64, 64, 64, float(np.float32(0.4)))
    Jr = oracle.evaluate(og, sl["meas"].astype(np.float64), best_th, DR, 10)[0]
    report("bo incumbent J", np.array([best_J]), np.array([Jr]), TOL)
    # interrupted after two cycles, resumed from the journal: the same proposals as uninterrupted
    b = _loop(ctx, problem, journal=str(tmp_path / "b.jsonl"))
    b.run(2)
    del b
    c = _loop(ctx, problem, journal=str(tmp_path / "b.jsonl"))
    assert len(c.cycles) == 2
    c.run(4)
    for k in (2, 3):
        np.testing.assert_array_equal(c.cycles[k].theta, a.cycles[k].theta)
        np.testing.assert_array_equal(c.cycles[k].J, a.cycles[k].J)
    with pytest.raises(ValueError):
        BOAC(ctx, problem[0], problem[1], delta_r=DR, n_iter=11, journal=str(tmp_path / "b.jsonl"))


@pytest.mark.parametrize("mode", ["envelope", "unrolled"])
def test_gradient_aware_cycles(ctx, problem, mode):
    bo = _loop(ctx, problem, gradient=mode)
    bo.run(3)
    th, J, G = bo.observations()
    assert G.shape == th.shape and np.all(np.isfinite(G))
    kinds = sum((c.kind for c in bo.cycles), [])
    assert "line" in kinds and "ei" in kinds
    # a line-search point lies on the ray from one of the incumbents along -grad (unit-box coordinates)
    c1 = bo.cycles[1]
    i = c1.kind.index("line")
    u = (c1.theta[i] - bo.lo) / (bo.hi - bo.lo)
    U0 = (bo.cycles[0].theta - bo.lo) / (bo.hi - bo.lo)
    G0 = bo.cycles[0].grad * (bo.hi - bo.lo)
    cosines = [np.dot(u - U0[j], -G0[j]) / (np.linalg.norm(u - U0[j]) * np.linalg.norm(G0[j]) + 1e-30)
               for j in np.argsort(bo.cycles[0].J)[:bo.line_starts]]
    assert max(cosines) > 0.99
    print(f"{mode}: best {bo.best()[1]:.3f} after {len(J)} evaluations")
