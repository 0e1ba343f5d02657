"""The stream-lane schedule does not change results: a batch evaluated on 1, 3 or 8 lanes, and a
256-candidate slice evaluated whole or cut into 2 or 4 parts (BOAC_BATCH_SPLIT), give the same J and
gradients bit for bit (per-candidate arithmetic does not depend on the grouping). Each setting runs in
a context of its own, so no graph captured under another setting is replayed."""
import os

import numpy as np
import pytest

from gpu_helpers import TOL, cands, geom_pair, make_slice, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8
SHAPES = [((40, 24, 40, 40), 5, 21), ((64, 32, 64, 64), 6, 22), ((48, 20, 48, 48), 3, 23), ((96, 64, 96, 96), 9, 24),
          ((40, 16, 40, 40), 7, 25)]


def _slices(shapes, with_grad):
    from paper_2109_11920_amd.api import SliceBatch
    out = []
    for shape, C, seed in shapes:
        g, og = geom_pair(*shape)
        S, _ = make_slice(og, seed=seed)
        th = cands(seed + 100, C)
        out.append(SliceBatch.make(g, torch.as_tensor(S, dtype=torch.float32, device="cuda"),
                                   torch.as_tensor(th, dtype=torch.float32, device="cuda"), with_grad))
    return out


def _eval(env, slices, K, ck=2):
    from paper_2109_11920_amd.api import Context
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        with Context(0) as ctx:
            stream = torch.cuda.Stream()
            for sb in slices:
                sb.obj.fill_(-1)
                if sb.grad is not None:
                    sb.grad.fill_(-1)
            stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
            with torch.cuda.stream(stream):
                ctx.evaluate_batch(slices, DR, K, ck)
            stream.synchronize()
            return ([sb.obj.clone() for sb in slices],
                    [None if sb.grad is None else sb.grad.clone() for sb in slices])
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("with_grad", [False, True])
def test_lane_count_does_not_change_results(with_grad):
    slices = _slices(SHAPES, with_grad)
    ref = _eval({"BOAC_BATCH_LANES": "1"}, slices, 6)
    for lanes in ("3", "8"):
        got = _eval({"BOAC_BATCH_LANES": lanes}, slices, 6)
        for s in range(len(SHAPES)):
            assert torch.equal(got[0][s], ref[0][s]), (lanes, s)
            if with_grad:
                assert torch.equal(got[1][s], ref[1][s]), (lanes, s)
    print(f"[parity] lanes 1/3/8, {len(SHAPES)} slices, grad={with_grad}: bitwise equal", flush=True)


def test_slice_parts_do_not_change_results():
    # 256 candidates of one 40^2 slice: whole, in 2 parts and in 4 parts (parts of >= 64 candidates);
    # the J of sampled candidates against the oracle
    g, og = geom_pair(40, 24, 40, 40)
    S, _ = make_slice(og, seed=31)
    th = cands(131, 256)
    from paper_2109_11920_amd.api import SliceBatch
    sb = [SliceBatch.make(g, torch.as_tensor(S, dtype=torch.float32, device="cuda"),
                          torch.as_tensor(th, dtype=torch.float32, device="cuda"), False)]
    ref = _eval({"BOAC_BATCH_SPLIT": "1"}, sb, 5)[0][0]
    for parts in ("2", "4"):
        got = _eval({"BOAC_BATCH_SPLIT": parts}, sb, 5)[0][0]
        assert torch.equal(got, ref), parts
    idx = [0, 63, 64, 127, 128, 191, 192, 255]
    Jr = np.array([oracle.evaluate(og, S, th[c].astype(np.float64), DR, 5)[0] for c in idx])
    report("whole/2/4 parts J (8 candidates at the part edges)", ref.cpu().numpy()[idx], Jr, TOL)
