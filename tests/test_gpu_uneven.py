"""GPU parity on the uneven batch: 48 slices with N in {96,128,192,256} and 64-256 angles, 32 candidates
each, 40 MLEM iterations, objective and gradient (checkpoint every 5), in one captured batch. The oracle
scores sampled (slice, candidate) pairs one by one, including the 192- and 256-pixel slices whose ray
kernels run in row bands; the rest is checked through properties."""
import os

import numpy as np
import pytest

from gpu_helpers import TOL, TOL_GRAD, ROOT, f32, geom_pair, oracle, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8


@pytest.fixture(scope="module")
def uneven():
    import synth
    from paper_2109_11920_amd.api import Context, SliceBatch
    d = np.load(os.path.join(ROOT, "tests", "golden", "uneven48.npz"))
    w = synth.workload("uneven48")
    cands = synth.workload_candidates(w)
    ctx = Context(0)
    slices, host = [], []
    for s in range(int(d["n_slices"])):
        n, na, nb, nt = (int(v) for v in d[f"s{s:02d}_geometry"])
        g, og = geom_pair(n, na, nb, nt, float(d[f"s{s:02d}_pixel"]))
        S = d[f"s{s:02d}_meas"].astype(np.float64)
        th = f32(cands[s])
        slices.append(SliceBatch.make(g, torch.as_tensor(S, dtype=torch.float32, device="cuda"),
                                      torch.as_tensor(th, dtype=torch.float32, device="cuda"), with_grad=True))
        host.append((og, S, th))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch(slices, DR, w.n_iter, w.ckpt_every)
    stream.synchronize()
    yield ctx, slices, host, w, stream
    ctx.close()


def test_uneven_batch_all_finite(uneven):
    ctx, slices, host, w, _ = uneven
    for s, sb in enumerate(slices):
        J = sb.obj.cpu().numpy()
        G = sb.grad.cpu().numpy()
        st = sb.status.cpu().numpy()
        assert np.all(np.isfinite(J)) and np.all(np.isfinite(G)), s
        assert np.all((st & 3) == 0), (s, st)


def test_uneven_batch_replay_is_identical(uneven):
    ctx, slices, host, w, stream = uneven
    J0 = [sb.obj.clone() for sb in slices]
    G0 = [sb.grad.clone() for sb in slices]
    for sb in slices:
        sb.obj.fill_(0)
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch(slices, DR, w.n_iter, w.ckpt_every)   # graph replay
    stream.synchronize()
    for s, sb in enumerate(slices):
        assert torch.equal(sb.obj, J0[s]) and torch.equal(sb.grad, G0[s]), s


def _pick(host, n, na):
    for s, (og, S, th) in enumerate(host):
        if og.n == n and og.n_angles == na:
            return s
    return None


@pytest.mark.parametrize("n,na,c", [(256, 128, 5), (192, 64, 17), (128, 256, 30), (96, 96, 3)])
def test_uneven_batch_objective_samples(uneven, n, na, c):
    ctx, slices, host, w, _ = uneven
    s = _pick(host, n, na)
    if s is None:
        pytest.skip(f"no {n}/{na} slice in this layout")
    og, S, th = host[s]
    Jr = oracle.evaluate(og, S, th[c], DR, w.n_iter)[0]
    report(f"uneven slice {s} ({n}x{n}, {na} angles) J cand {c}", slices[s].obj[c:c + 1].cpu().numpy(),
           np.array([Jr]), TOL)


@pytest.mark.parametrize("n,na,c", [(96, 64, 7), (128, 96, 21), (192, 64, 9), (256, 64, 13)])
def test_uneven_batch_gradient_samples(uneven, n, na, c):
    ctx, slices, host, w, _ = uneven
    s = _pick(host, n, na)
    if s is None:
        pytest.skip(f"no {n}/{na} slice in this layout")
    og, S, th = host[s]
    Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, w.n_iter)
    G = slices[s].grad[c].cpu().numpy()
    print("   gpu   ", np.array2string(G, precision=5), "\n   oracle", np.array2string(Gr, precision=5))
    report(f"uneven slice {s} ({n}x{n}, {na} angles) J cand {c}", slices[s].obj[c:c + 1].cpu().numpy(),
           np.array([Jr]), TOL)
    report(f"uneven slice {s} ({n}x{n}, {na} angles) dJ cand {c}", G, Gr, TOL_GRAD)
