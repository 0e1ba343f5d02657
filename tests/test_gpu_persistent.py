"""Persistent batch execution: the batch's launches recorded as tasks and run by one persistent launch
with a device work queue and per-lane completion counters. Results against the stream-lane schedule
(the same kernels; the reductions of the likelihood, the log-factorial constant and the raster adjoint
run on other workgroup sizes, so agreement is to FP32 rounding) and against the oracle; a graph replay
equals the first run; a dependency-wait bound tripped by the host ends every workgroup and the call
reports BOAC_ETIMEOUT, after which the context still evaluates correctly."""
import numpy as np
import pytest

from gpu_helpers import TOL, TOL_GRAD, cands, geom_pair, make_slice, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8
SHAPES = [((40, 24, 40, 40), 5, 11), ((64, 32, 64, 64), 6, 12), ((48, 20, 48, 48), 3, 13), ((96, 64, 96, 96), 9, 14)]


def _batch(with_grad):
    from paper_2109_11920_amd.api import SliceBatch
    out, host = [], []
    for shape, C, seed in SHAPES:
        g, og = geom_pair(*shape)
        S, _ = make_slice(og, seed=seed)
        th = cands(seed + 100, C)
        out.append(SliceBatch.make(g, torch.as_tensor(S, dtype=torch.float32, device="cuda"),
                                   torch.as_tensor(th, dtype=torch.float32, device="cuda"), with_grad))
        host.append((og, S, th))
    return out, host


def _run(ctx, slices, stream, K, ck=2):
    for sb in slices:
        sb.obj.fill_(-1)
        if sb.grad is not None:
            sb.grad.fill_(-1)
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch(slices, DR, K, ck)
    stream.synchronize()
    return [sb.obj.clone() for sb in slices], [None if sb.grad is None else sb.grad.clone() for sb in slices]


@pytest.mark.parametrize("with_grad", [False, True])
def test_persistent_batch_matches_lanes_and_oracle(with_grad):
    from paper_2109_11920_amd.api import Context
    K = 5
    slices, host = _batch(with_grad)
    stream = torch.cuda.Stream()
    with Context(0) as ctx:
        J_l, G_l = _run(ctx, slices, stream, K)
        ctx.set_batch_mode("persistent")
        print("[persistent] first run", flush=True)
        J_p, G_p = _run(ctx, slices, stream, K)
        print("[persistent] replay", flush=True)
        J_r, G_r = _run(ctx, slices, stream, K)
        for s in range(len(slices)):
            assert torch.equal(J_p[s], J_r[s])
            report(f"persistent vs lanes slice {s} J", J_p[s].cpu().numpy(), J_l[s].cpu().numpy(), 1e-6)
            if with_grad:
                assert torch.equal(G_p[s], G_r[s])
                report(f"persistent vs lanes slice {s} dJ", G_p[s].cpu().numpy(), G_l[s].cpu().numpy(), 1e-5)
        st = [sb.status.cpu().numpy() for sb in slices]
        assert all(np.all((x & 3) == 0) for x in st)
    for s in (0, 3):
        og, S, th = host[s]
        if with_grad:
            Jr, Gr = oracle.objective_and_grad(og, S, th[1], DR, K)
            report(f"persistent slice {s} cand 1 dJ vs oracle", G_p[s][1].cpu().numpy(), Gr, TOL_GRAD)
        else:
            Jr = oracle.evaluate(og, S, th[1], DR, K)[0]
        report(f"persistent slice {s} cand 1 J vs oracle", J_p[s][1:2].cpu().numpy(), np.array([Jr]), TOL)


def test_persistent_wait_bound_reports_timeout_and_recovers():
    from paper_2109_11920_amd.api import BoacError, Context
    slices, host = _batch(False)
    stream = torch.cuda.Stream()
    with Context(0) as ctx:
        ctx.set_batch_mode("persistent")
        J0, _ = _run(ctx, slices, stream, 4)
        # a bound of one poll: some workgroup finds its predecessor unfinished, records the error, and every
        # workgroup leaves the queue
        ctx.set_batch_mode("persistent", spin_limit=1)
        print("[persistent] tripped bound", flush=True)
        with pytest.raises(BoacError) as e:
            _run(ctx, slices, stream, 4)
        assert e.value.code == 5, str(e.value)
        ctx.set_batch_mode("persistent")
        J1, _ = _run(ctx, slices, stream, 4)
        for s in range(len(slices)):
            assert torch.equal(J0[s], J1[s])
