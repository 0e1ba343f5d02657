"""boac_objective_noalloc (no device allocation by the library; scratch in a fixed per-device array)
against boac_objective, through the C ABI: two calls in a row, the second on a smaller input, then a
candidate count that the fixed array holds only in chunks. Results equal the allocating entry point's to
the parity gates (bit for bit where both evaluate the same candidate chunks)."""
import numpy as np
import pytest

from gpu_helpers import TOL, cands, geom_pair, make_slice, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8


def _run(ctx, g, S, th, K):
    C = th.shape[0]
    meas = torch.as_tensor(S, dtype=torch.float32, device="cuda")
    cand = torch.as_tensor(th, dtype=torch.float32, device="cuda")
    J0, F0, st0 = ctx.objective(g, meas, cand, DR, K, want_image=True)
    obj = torch.full((C,), -1.0, device="cuda")
    status = torch.full((C,), 77, dtype=torch.int32, device="cuda")
    img = torch.full((C, g.n, g.n), -1.0, device="cuda")
    J1, F1, st1 = ctx.objective_noalloc(g, meas, cand, DR, K, obj, status, img)
    torch.cuda.synchronize()
    return (J0.cpu().numpy(), F0.cpu().numpy(), st0.cpu().numpy()), (J1.cpu().numpy(), F1.cpu().numpy(),
                                                                      st1.cpu().numpy())


def test_noalloc_matches_objective_two_calls_then_chunked():
    from paper_2109_11920_amd.api import Context
    with Context(0) as ctx:
        # call 1: 64 x 64, 64 angles, 12 candidates (one chunk)
        g, og = geom_pair(64, 64, pixel=0.4)
        S, _ = make_slice(og, seed=41)
        th = cands(42, 12)
        ref, got = _run(ctx, g, S, th, 8)
        report("noalloc 64^2 x12 J", got[0], ref[0], TOL)
        report("noalloc 64^2 x12 F^K", got[1], ref[1], TOL)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert np.array_equal(got[2], ref[2])
        # call 2, smaller: 40 x 40, 24 angles, 3 candidates; the array keeps call 1's contents
        g2, og2 = geom_pair(40, 24, 40, 40)
        S2, _ = make_slice(og2, seed=43)
        th2 = cands(44, 3)
        ref2, got2 = _run(ctx, g2, S2, th2, 5)
        report("noalloc 40^2 x3 J", got2[0], ref2[0], TOL)
        report("noalloc 40^2 x3 F^K", got2[1], ref2[1], TOL)
        assert np.array_equal(got2[0], ref2[0]) and np.array_equal(got2[2], ref2[2])
        Jr = oracle.evaluate(og2, S2, th2[1], DR, 5)[0]
        report("noalloc 40^2 cand 1 J vs oracle", got2[0][1:2], np.array([Jr]), TOL)
        # call 3: 128^3 with more candidates than the array holds at once (evaluated in chunks)
        g3, og3 = geom_pair(128, 128, pixel=0.2)
        S3, _ = make_slice(og3, seed=45)
        th3 = cands(46, 24)
        ref3, got3 = _run(ctx, g3, S3, th3, 4)
        report("noalloc 128^3 x24 (chunked) J", got3[0], ref3[0], TOL)
        report("noalloc 128^3 x24 (chunked) F^K", got3[1], ref3[1], TOL)
        assert np.array_equal(got3[2], ref3[2])
