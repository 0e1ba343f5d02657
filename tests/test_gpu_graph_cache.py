"""The batch graph cache never replays a graph captured before a scratch reallocation.

The scratch generation is one counter per context: any buffer that grows (here the eager entry points'
scratch, grown by a larger objective call after batch A was captured) retires every graph captured
before it, since a graph cannot tell which of its buffers moved. The next batch A runs eagerly and is
captured afresh, and only the fresh graph is replayed afterwards. The library's graph counters show
which happened, so the check never depends on replaying a stale graph."""
import numpy as np
import pytest

from gpu_helpers import TOL, cands, geom_pair, make_slice, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8


def test_stale_graph_is_dropped_after_scratch_growth():
    from paper_2109_11920_amd.api import Context, SliceBatch
    g, og = geom_pair(40, 24, 40, 40)
    S, _ = make_slice(og, seed=3)
    meas = torch.as_tensor(S, dtype=torch.float32, device="cuda")
    th = cands(11, 4)
    stream = torch.cuda.Stream()
    with Context(0) as ctx:
        sb = SliceBatch.make(g, meas, torch.as_tensor(th, dtype=torch.float32, device="cuda"), with_grad=False)
        stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.evaluate_batch([sb], DR, 6)          # eager run, then capture
        stream.synchronize()
        J0 = sb.obj.clone()
        graphs, captures, replays, gen0 = ctx.graph_stats()
        assert (graphs, captures, replays) == (1, 1, 0)

        # a larger objective call grows the eager scratch: the scratch generation moves on
        big = torch.as_tensor(cands(12, 64), dtype=torch.float32, device="cuda")
        stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.objective(g, meas, big, DR, 2)
        stream.synchronize()
        gen1 = ctx.graph_stats()[3]
        assert gen1 > gen0

        sb.obj.fill_(0)
        stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.evaluate_batch([sb], DR, 6)          # stale graph dropped: eager run and a new capture
        stream.synchronize()
        graphs, captures, replays, _ = ctx.graph_stats()
        assert (graphs, captures, replays) == (1, 2, 0)
        assert torch.equal(sb.obj, J0)

        sb.obj.fill_(0)
        stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.evaluate_batch([sb], DR, 6)          # replay of the fresh graph
        stream.synchronize()
        graphs, captures, replays, _ = ctx.graph_stats()
        assert (graphs, captures, replays) == (1, 2, 1)
        assert torch.equal(sb.obj, J0)

    Jr = np.array([oracle.evaluate(og, S, th[c].astype(np.float64), DR, 6)[0] for c in range(4)])
    report("graph cache J (4 candidates)", J0.cpu().numpy(), Jr, TOL)
