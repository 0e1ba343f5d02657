"""GPU parity: every C-ABI entry point against the FP64 oracle on the same seeded inputs.

Sizes span several pixel tiles and ray chunks with ragged tails; the banded LDS path (large n) and
non-square detector/ray counts are covered. Gates: relative L2 <= 1e-4 on maps, sinograms, images and
objectives, <= 1e-3 on gradients; every error is printed."""
import numpy as np
import pytest

from gpu_helpers import TOL, TOL_GRAD, cands, f32, geom_pair, make_slice, oracle, rel_l2, report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DR = 0.8


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_11920_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def dev(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype or torch.float32, device="cuda")


GEOMS = [
    # (n, n_angles, n_bins, n_samples): ragged tiles (40 = 32 + 8), ragged ray chunks, nb != n, nt != n;
    # bins and samples off the attenuation blocks (not multiples of 8 and 4: the ray kernels' 4-sample
    # groups then hold padding rows); the slid-block gather (one-bin window, >= 32 bins and samples)
    # with its block slid to the sinogram edges, column-group staged where the sample count is a
    # multiple of 4 (40) and slot staged where it is not (70, 50), and the
    # general gather for a two-bin window (62 bins on 48 pixels) and for a sinogram narrower than the
    # 32-bin block (26 bins, 30 samples)
    (40, 24, 40, 40),
    (70, 30, 70, 70),
    (48, 20, 62, 48),
    (36, 16, 36, 50),
    (28, 12, 26, 30),
]


@pytest.mark.parametrize("shape", GEOMS)
def test_rasterize(ctx, shape):
    g, og = geom_pair(*shape)
    th = cands(1, 5)
    mu = ctx.rasterize_mu(g, dev(th), DR).cpu().numpy()
    for c in range(5):
        report(f"mu {shape} cand {c}", mu[c], oracle.rasterize_mu(og, th[c], DR), TOL)


def test_rasterize_full_size(ctx):
    g, og = geom_pair(128, 128, pixel=0.2)
    th = cands(2, 4)
    mu = ctx.rasterize_mu(g, dev(th), DR).cpu().numpy()
    for c in range(4):
        report(f"mu 128 cand {c}", mu[c], oracle.rasterize_mu(og, th[c], DR), TOL)


def _mu_img(og, seed, C):
    rng = np.random.default_rng(seed)
    th = cands(seed, C)
    mus = np.stack([oracle.rasterize_mu(og, th[c], DR) for c in range(C)])
    imgs = rng.uniform(0.0, 2.0, (C, og.n, og.n))
    return f32(mus), f32(imgs)


@pytest.mark.parametrize("shape", GEOMS)
def test_project(ctx, shape):
    g, og = geom_pair(*shape)
    mus, imgs = _mu_img(og, 3, 3)
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    for c in range(3):
        ref = oracle.project(og, oracle.attenuation(og, mus[c]), imgs[c])
        report(f"project {shape} cand {c}", y[c], ref, TOL)


@pytest.mark.parametrize("shape", GEOMS)
def test_backproject_and_adjoint_identity(ctx, shape):
    g, og = geom_pair(*shape)
    mus, imgs = _mu_img(og, 4, 3)
    z = f32(np.random.default_rng(5).uniform(-1, 1, (3, og.n_angles, og.n_bins)))
    x = ctx.backproject(g, dev(mus), dev(z)).cpu().numpy()
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    for c in range(3):
        ref = oracle.backproject(og, oracle.attenuation(og, mus[c]), z[c])
        report(f"backproject {shape} cand {c}", x[c], ref, TOL)
        lhs = np.sum(y[c].astype(np.float64) * z[c])
        rhs = np.sum(imgs[c] * x[c].astype(np.float64))
        # normalised by the absolute inner product: z has both signs, so <Ax, z> itself cancels
        scale = min(np.sum(np.abs(y[c].astype(np.float64) * z[c])), np.sum(np.abs(imgs[c] * x[c])))
        adj = abs(lhs - rhs) / scale
        print(f"[parity] adjoint identity {shape} cand {c}: {adj:.3e}", flush=True)
        assert adj < 2e-5


def test_projector_exact_axis_angles(ctx):
    # 4 angles: 0/90/180/270 deg, samples on pixel centres; the oracle's exact sums
    g, og = geom_pair(32, 4, pixel=0.5)
    mus, imgs = _mu_img(og, 6, 2)
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    for c in range(2):
        report(f"axis angles cand {c}", y[c], oracle.project(og, oracle.attenuation(og, mus[c]), imgs[c]), 2e-6)


def test_mu_zero_reduces_to_plain_radon(ctx):
    g, og = geom_pair(40, 24)
    _, imgs = _mu_img(og, 7, 2)
    mus = np.zeros_like(imgs)
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    for c in range(2):
        ref = oracle.project(og, np.ones((og.n_angles, og.n_bins, og.n_samples)), imgs[c])
        report(f"mu=0 cand {c}", y[c], ref, TOL)


@pytest.mark.parametrize("n", [200, 256])
def test_banded_large_images(ctx, n):
    # images larger than one LDS stage: the row-band path of every ray kernel
    g, og = geom_pair(n, 12)
    mus, imgs = _mu_img(og, 8, 2)
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    z = f32(np.random.default_rng(9).uniform(0, 1, (2, og.n_angles, og.n_bins)))
    x = ctx.backproject(g, dev(mus), dev(z)).cpu().numpy()
    for c in range(2):
        att = oracle.attenuation(og, mus[c])
        report(f"banded project n={n} cand {c}", y[c], oracle.project(og, att, imgs[c]), TOL)
        report(f"banded backproject n={n} cand {c}", x[c], oracle.backproject(og, att, z[c]), TOL)


@pytest.mark.parametrize("shape", [(640, 8, 640, 640), (1024, 4, 1024, 1024)])
def test_many_row_bands(ctx, shape):
    # the largest admitted images: one image takes 11 and 27 row bands, the two-image stage of the
    # reverse sweeps 22 and 57 (each band still within one workgroup's LDS); the objective, the
    # unrolled and the envelope gradients against the oracle
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=41)
    th = cands(42, 2)
    J, G, st = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 1, 1, mode="unrolled")
    Je, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 1, 1, mode="envelope")
    Jf, _, _ = ctx.objective(g, dev(S), dev(th), DR, 1)
    assert torch.allclose(J, Jf, rtol=2e-6, atol=0) and torch.allclose(Je, Jf, rtol=2e-6, atol=0)
    J, G, Ge = J.cpu().numpy(), G.cpu().numpy(), Ge.cpu().numpy()
    for c in range(2):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 1, with_delta_r=True)
        report(f"bands {shape} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"bands {shape} cand {c} dJ", G[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 1, with_delta_r=True)
        report(f"bands {shape} cand {c} envelope dJ", Ge[c], Gr, TOL_GRAD)


@pytest.mark.parametrize("shape", [(2, 2, 2, 2), (3, 3, 6, 5), (16, 8192, 32, 16), (20, 6, 40, 1024)])
def test_extreme_shapes(ctx, shape):
    # the smallest image, an odd angle count (no opposed-ray pairing) with the widest bin window
    # (n_bins = 2 n), the largest angle count, the largest sample count: objective and the unrolled and
    # envelope gradients (with dJ/d(dR)) against the oracle
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=61)
    th = cands(62, 2)
    J, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 2, 1, mode="unrolled")
    Je, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 2, 1, mode="envelope")
    Jf, _, _ = ctx.objective(g, dev(S), dev(th), DR, 2)
    assert torch.allclose(J, Jf, rtol=2e-6, atol=0) and torch.allclose(Je, Jf, rtol=2e-6, atol=0)
    J, G, Ge = J.cpu().numpy(), G.cpu().numpy(), Ge.cpu().numpy()
    for c in range(2):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 2, with_delta_r=True)
        report(f"extreme {shape} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"extreme {shape} cand {c} dJ", G[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 2, with_delta_r=True)
        report(f"extreme {shape} cand {c} envelope dJ", Ge[c], Gr, TOL_GRAD)


def test_largest_candidate_count(ctx):
    # C = 2^20, the largest admitted count, on a small slice: sampled objectives against the oracle,
    # every objective finite, and each sample equal to its one-candidate evaluation bit for bit
    g, og = geom_pair(12, 8, 12, 12)
    S, _ = make_slice(og, seed=71)
    C = 1 << 20
    th = cands(72, C)
    J, _, _ = ctx.objective(g, dev(S), dev(th), DR, 2)
    assert bool(torch.isfinite(J).all())
    for c in (0, 1, 524287, C - 1):
        Jr = oracle.evaluate(og, S, th[c], DR, 2)[0]
        report(f"C = 2^20 J cand {c}", J[c:c + 1].cpu().numpy(), np.array([Jr]), TOL)
        J1, _, _ = ctx.objective(g, dev(S), dev(th[c:c + 1]), DR, 2)
        assert torch.equal(J1[0], J[c])


# drawn once from a seeded generator over the admitted sizes (n from 3 to 196, 2 to 39 angles, 2 to 2n
# bins, 2 to 2n + 19 samples): odd and even angle counts, bins above and below n, sample counts off
# the 4-sample groups, single-tile images, images on both sides of the paired-stage limit (140) and
# row-banded gradient images (150, 196)
RANDOM_GEOMS = [(15, 27, 4, 12), (17, 13, 31, 43), (196, 39, 32, 60), (150, 4, 51, 59), (196, 15, 105, 71),
                (47, 24, 76, 71), (196, 6, 192, 233), (90, 2, 38, 94), (3, 39, 5, 21), (47, 24, 34, 38),
                (7, 9, 11, 16), (150, 12, 217, 280), (150, 10, 111, 89), (141, 32, 126, 82)]


@pytest.mark.parametrize("shape", RANDOM_GEOMS)
def test_random_geometries(ctx, shape):
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=81)
    th = cands(82, 3)
    J, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 2, 1, mode="unrolled")
    Jf, _, _ = ctx.objective(g, dev(S), dev(th), DR, 2)
    assert torch.allclose(J, Jf, rtol=2e-6, atol=0)
    J, G = J.cpu().numpy(), G.cpu().numpy()
    for c in (1, 2):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 2, with_delta_r=True)
        report(f"random {shape} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"random {shape} cand {c} dJ", G[c], Gr, TOL_GRAD)


# a second seeded draw with candidate counts (one, the few-candidate plans, many) and pixel sizes:
# (n, n_angles, n_bins, n_samples, C, pixel_cm)
RANDOM_CASES = [(256, 13, 351, 359, 5, 0.3), (160, 2, 97, 98, 33, 0.1), (64, 98, 18, 118, 1, 0.37),
                (64, 42, 37, 107, 2, 0.5), (64, 61, 75, 82, 5, 0.81), (256, 14, 319, 137, 33, 0.29),
                (210, 4, 361, 245, 1, 0.13), (2, 18, 3, 23, 5, 0.93), (210, 13, 186, 206, 2, 0.32),
                (64, 119, 3, 16, 1, 0.72), (210, 5, 304, 149, 5, 0.85), (2, 80, 2, 13, 2, 0.89),
                (16, 62, 31, 44, 9, 0.77), (128, 57, 25, 68, 5, 0.56)]


@pytest.mark.parametrize("case", RANDOM_CASES)
def test_random_geometries_counts_and_pixels(ctx, case):
    n, na, nb, nt, C, px = case
    g, og = geom_pair(n, na, nb, nt, pixel=px)
    S, _ = make_slice(og, seed=91)
    th = cands(92, C)
    J, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 2, 1, mode="unrolled")
    Je, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 2, 1, mode="envelope")
    Jf, _, _ = ctx.objective(g, dev(S), dev(th), DR, 2)
    assert torch.allclose(J, Jf, rtol=2e-6, atol=0) and torch.allclose(Je, Jf, rtol=2e-6, atol=0)
    J, G, Ge = J.cpu().numpy(), G.cpu().numpy(), Ge.cpu().numpy()
    for c in sorted({0, C - 1}):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 2, with_delta_r=True)
        report(f"random {case} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"random {case} cand {c} dJ", G[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 2, with_delta_r=True)
        report(f"random {case} cand {c} envelope dJ", Ge[c], Gr, TOL_GRAD)


@pytest.mark.parametrize("case", RANDOM_CASES[::2])
def test_random_geometries_other_entry_points(ctx, case):
    # rasterisation, projection, backprojection and MLEM on the second draw's geometries
    n, na, nb, nt, C, px = case
    g, og = geom_pair(n, na, nb, nt, pixel=px)
    C = min(C, 3)
    th = cands(93, C)
    mu = ctx.rasterize_mu(g, dev(th), DR).cpu().numpy()
    rng = np.random.default_rng(94)
    imgs = f32(rng.uniform(0.0, 2.0, (C, n, n)))
    z = f32(rng.uniform(0.0, 1.0, (C, na, nb)))
    mus = f32(mu)
    y = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    x = ctx.backproject(g, dev(mus), dev(z)).cpu().numpy()
    S, _ = make_slice(og, seed=95)
    F = ctx.mlem(g, dev(mus), dev(S), 3).cpu().numpy()
    for c in range(C):
        report(f"random {case} mu cand {c}", mu[c], oracle.rasterize_mu(og, th[c], DR), TOL)
        att = oracle.attenuation(og, mus[c])
        report(f"random {case} project cand {c}", y[c], oracle.project(og, att, imgs[c]), TOL)
        report(f"random {case} backproject cand {c}", x[c], oracle.backproject(og, att, z[c]), TOL)
        report(f"random {case} mlem cand {c}", F[c], oracle.mlem(og, att, S, 3), TOL)


@pytest.mark.parametrize("shape,K", [((40, 24, 40, 40), 8), ((64, 64, 64, 64), 20)])
def test_mlem(ctx, shape, K):
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=11)
    mus, _ = _mu_img(og, 12, 2)
    F = ctx.mlem(g, dev(mus), dev(S), K).cpu().numpy()
    for c in range(2):
        ref = oracle.mlem(og, oracle.attenuation(og, mus[c]), S, K)
        report(f"mlem {shape} K={K} cand {c}", F[c], ref, TOL)


def test_mlem_from_a_given_start(ctx):
    # boac_mlem continues from the image passed in: a random positive start with a zero region (which
    # stays zero), and K = 0 (the start comes back unchanged)
    g, og = geom_pair(40, 24, 40, 40)
    S, _ = make_slice(og, seed=37)
    mus, _ = _mu_img(og, 38, 2)
    rng = np.random.default_rng(39)
    F0 = f32(rng.uniform(0.5, 2.0, (2, 40, 40)))
    F0[:, :8, :] = 0.0
    F = ctx.mlem(g, dev(mus), dev(S), 6, img=dev(F0)).cpu().numpy()
    F00 = ctx.mlem(g, dev(mus), dev(S), 0, img=dev(F0)).cpu().numpy()
    assert np.array_equal(F00, F0.astype(np.float32))
    for c in range(2):
        ref = oracle.mlem(og, oracle.attenuation(og, mus[c]), S, 6, f0=F0[c])
        report(f"mlem from a start cand {c}", F[c], ref, TOL)
        assert np.all(F[c][:8, :] == 0)


def test_objective_smoke_config(ctx, slice64):
    # 64 x 64, 0.4 cm, 64 angles, true head, 20 iterations
    g, og = geom_pair(64, 64, pixel=0.4)
    S = slice64["meas"].astype(np.float64)
    th = f32(slice64["theta"][None, :])
    J, img, st = ctx.objective(g, dev(S), dev(th), DR, 20, want_image=True)
    Jr, Fr, _ = oracle.evaluate(og, S, th[0], DR, 20)
    report("objective smoke J", J.cpu().numpy(), np.array([Jr]), TOL)
    report("objective smoke F^K", img.cpu().numpy()[0], Fr, TOL)
    assert int(st.cpu()[0]) == 0


def test_objective_plain_config(ctx, slice128):
    # 128 x 128, 0.2 cm, 128 angles, 5e5 counts, one candidate, 50 iterations
    g, og = geom_pair(128, 128, pixel=0.2)
    S = slice128["meas"].astype(np.float64)
    th = f32(slice128["theta"][None, :])
    J, img, st = ctx.objective(g, dev(S), dev(th), DR, 50, want_image=True)
    Jr, Fr, _ = oracle.evaluate(og, S, th[0], DR, 50)
    report("objective plain J", J.cpu().numpy(), np.array([Jr]), TOL)
    report("objective plain F^K", img.cpu().numpy()[0], Fr, TOL)


def test_objective_batch_matches_oracle_samples(ctx, slice128):
    # the 256-candidate batch, 30 iterations, in the launch configuration of the bench; the oracle
    # scores 16 candidates spread over the batch (every candidate group and XCD slot of the gather's
    # grid is touched by one of them) one by one, objective and reconstruction
    g, og = geom_pair(128, 128, pixel=0.2)
    S = slice128["meas"].astype(np.float64)
    import synth
    th = f32(synth.draw_candidates(synth.candidate_stream(0), 256))
    J, F, st = ctx.objective(g, dev(S), dev(th), DR, 30, want_image=True)
    J = J.cpu().numpy()
    st = st.cpu().numpy()
    assert np.all(np.isfinite(J))
    assert np.all((st & 3) == 0)
    for c in (0, 17, 34, 51, 68, 85, 102, 119, 137, 154, 171, 188, 205, 222, 239, 255):
        Jr, Fr, _ = oracle.evaluate(og, S, th[c], DR, 30)
        report(f"batch256 J cand {c}", J[c:c + 1], np.array([Jr]), TOL)
        report(f"batch256 F^K cand {c}", F[c].cpu().numpy(), Fr, TOL)


def test_objective_paper72_samples(ctx):
    # the paper's 72 angles over 360 deg at 128 x 128, data simulated on a 2x finer grid; the 256-candidate
    # draw of that workload, 30 iterations; the true head and three sampled candidates against the oracle
    import os
    import synth
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "slice_n128_a72.npz"))
    g, og = geom_pair(128, 72, 128, 128, pixel=0.2)
    S = d["meas"].astype(np.float64)
    th = f32(synth.workload_candidates(synth.workload("paper72_n128"))[0])
    th[0] = f32(d["theta"])
    J, img, st = ctx.objective(g, dev(S), dev(th), DR, 30, want_image=True)
    J = J.cpu().numpy()
    assert np.all(np.isfinite(J)) and np.all((st.cpu().numpy() & 3) == 0)
    for c in (0, 91, 200):
        Jr, Fr, _ = oracle.evaluate(og, S, th[c], DR, 30)
        report(f"paper72 J cand {c}", J[c:c + 1], np.array([Jr]), TOL)
        if c == 0:
            report("paper72 F^K true head", img.cpu().numpy()[0], Fr, TOL)


@pytest.mark.parametrize("shape", [(40, 24, 40, 40), (64, 64, 64, 64), (36, 25, 36, 36), (200, 16, 200, 200)])
def test_opposed_ray_pairing_matches_the_full_tensor(ctx, shape, monkeypatch):
    # even angle counts with the column-group gather hold half the angles plus exp(-T) per ray; the
    # result equals the full tensor's to FP32 rounding (odd counts always hold every angle)
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=31)
    th = dev(cands(32, 5))
    mu = ctx.rasterize_mu(g, th, DR)
    img = dev(np.random.default_rng(3).uniform(0.5, 2.0, (5,) + g.image_shape))
    sino = dev(np.random.default_rng(4).uniform(0.0, 3.0, (5,) + g.sino_shape))
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BOAC_OPPOSED_RAYS", flag)
        J, F, _ = ctx.objective(g, dev(S), th, DR, 6, want_image=True)
        y = ctx.project(g, mu, img)
        x = ctx.backproject(g, mu, sino)
        runs[flag] = [t.cpu().numpy() for t in (J, F, y, x)]
    for name, a, b in zip(("J", "F^K", "A f", "A^T z"), runs["1"], runs["0"]):
        report(f"pairing {shape} {name}", a, b, 2e-6)
    # the pair stays an exact transpose: <A f, z> = <f, A^T z>
    y, x = runs["1"][2].astype(np.float64), runs["1"][3].astype(np.float64)
    lhs = np.sum(y * sino.cpu().numpy())
    rhs = np.sum(img.cpu().numpy() * x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-5
    # and against the oracle
    Jr = oracle.evaluate(og, S, th[1].cpu().numpy().astype(np.float64), DR, 6)[0]
    report(f"pairing {shape} J vs oracle", runs["1"][0][1:2], np.array([Jr]), TOL)


@pytest.mark.parametrize("shape,K", [((40, 24, 40, 40), 4), ((64, 64, 64, 64), 3), ((32, 16, 32, 32), 0),
                                     ((192, 12, 192, 192), 2), ((256, 8, 256, 256), 1)])
def test_opposed_ray_pairing_in_the_gradients(ctx, shape, K, monkeypatch):
    # 192 and 256 pixels: the two-image ray kernels (and at 256 the one-image ones) run in row bands
    # the reverse sweeps and the tail carry the opposed ray's adjoint through att' = exp(-T) / att
    # (att_bar and a per-ray E_bar); the unrolled and envelope gradients equal the full tensor's to
    # FP32 rounding and the oracle's to the gate.
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=33)
    th = cands(34, 3)
    th[2] = f32(th[2] + np.array([0.3, 0.2, -0.2, 0.1, 0.1, -0.1, 0.01, -0.02]))
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BOAC_OPPOSED_RAYS", flag)
        out = []
        for mode in ("unrolled", "envelope"):
            J, G, st = ctx.objective_grad_ex(g, dev(S), dev(th), DR, K, 2, mode=mode)
            out += [J.cpu().numpy(), G.cpu().numpy()]
        runs[flag] = out
    for name, a, b in zip(("J", "dJ", "J env", "dJ env"), runs["1"], runs["0"]):
        report(f"pairing grad {shape} K={K} {name}", a, b, 2e-5)
    for c in range(3):
        _, Gr = oracle.objective_and_grad(og, S, th[c], DR, K, with_delta_r=True)
        report(f"pairing grad {shape} K={K} cand {c} dJ vs oracle", runs["1"][1][c], Gr, TOL_GRAD)
        _, Ge = oracle.objective_and_envelope_grad(og, S, th[c], DR, K, with_delta_r=True)
        report(f"pairing grad {shape} K={K} cand {c} envelope dJ vs oracle", runs["1"][3][c], Ge, TOL_GRAD)


def test_opposed_ray_pairing_under_heavy_attenuation(ctx, monkeypatch):
    # mu up to 2/cm over a 25.6 cm field: ray totals T near 40, opposed attenuations exp(-T) / att far
    # below 1e-10; paired and full tensors still agree, and both match the oracle
    g, og = geom_pair(48, 32)
    S, _ = make_slice(og, seed=35)
    th = cands(36, 3)
    th[1, 6:] = (1.5, 2.0)
    th[2, 6:] = (0.8, 1.2)
    th = f32(th)
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BOAC_OPPOSED_RAYS", flag)
        J, G, st = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 3, 2, mode="unrolled")
        runs[flag] = (J.cpu().numpy(), G.cpu().numpy(), st.cpu().numpy())
    assert np.all(np.isfinite(runs["1"][0])) and np.all(np.isfinite(runs["1"][1]))
    report("heavy attenuation J paired vs full", runs["1"][0], runs["0"][0], 1e-6)
    report("heavy attenuation dJ paired vs full", runs["1"][1], runs["0"][1], 1e-5)
    for c in (1, 2):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 3, with_delta_r=True)
        report(f"heavy attenuation cand {c} J", runs["1"][0][c:c + 1], np.array([Jr]), TOL)
        report(f"heavy attenuation cand {c} dJ", runs["1"][1][c], Gr, TOL_GRAD)


def test_count_preservation_on_gpu(ctx, slice128):
    g, og = geom_pair(128, 128, pixel=0.2)
    S = slice128["meas"].astype(np.float64)
    th = cands(13, 4)
    mu = ctx.rasterize_mu(g, dev(th), DR)
    F = ctx.mlem(g, mu, dev(S), 7)
    y = ctx.project(g, mu, F).cpu().numpy().astype(np.float64)
    for c in range(4):
        e = abs(y[c].sum() - S.sum()) / S.sum()
        print(f"[parity] count preservation cand {c}: {e:.3e}", flush=True)
        assert e < 1e-5


@pytest.mark.parametrize("C", [9, 130, 300])
def test_batched_equals_unbatched_and_deterministic(ctx, slice64, C):
    # 9, 130 and 300 candidates take different default ray plans (no plan-cache entry at 64 pixels:
    # 256-, 512- and 1024-thread paired projections with 1 or 2 rays per thread); every candidate's
    # result equals its one-candidate evaluation bit for bit
    g, og = geom_pair(64, 64, pixel=0.4)
    S = dev(slice64["meas"].astype(np.float64))
    th = cands(14, C)
    Jb, Fb, _ = ctx.objective(g, S, dev(th), DR, 6, want_image=True)
    Jb2, Fb2, _ = ctx.objective(g, S, dev(th), DR, 6, want_image=True)
    assert torch.equal(Jb, Jb2) and torch.equal(Fb, Fb2)
    for c in (0, C // 2, C - 1):
        J1, F1, _ = ctx.objective(g, S, dev(th[c:c + 1]), DR, 6, want_image=True)
        assert torch.equal(J1[0], Jb[c]) and torch.equal(F1[0], Fb[c])


def test_nac_candidate_and_status_bits(ctx, slice64):
    g, og = geom_pair(64, 64, pixel=0.4)
    S = slice64["meas"].astype(np.float64)
    th = cands(15, 4)
    th[1, 6:] = 0.0            # no attenuation correction (mu = 0)
    th[2, 0] = 1.0             # head outline dips below zero somewhere
    th[2, 2] = 3.0
    th[3, 0] = np.nan          # non-finite candidate
    J, _, st = ctx.objective(g, dev(S), dev(th), DR, 5)
    J = J.cpu().numpy()
    st = st.cpu().numpy()
    Jr = oracle.evaluate(og, S, th[1], DR, 5)[0]
    report("NAC J", J[1:2], np.array([Jr]), TOL)
    assert st[2] & 4
    assert st[3] & 2 and not np.isfinite(J[3])
    Sneg = S.copy()
    Sneg[0, 0] = -1.0
    _, _, st2 = ctx.objective(g, dev(Sneg), dev(th[:1]), DR, 2)
    assert int(st2.cpu()[0]) & 8


def test_zero_measurement(ctx):
    g, og = geom_pair(32, 16, pixel=0.8)
    S = np.zeros((16, 32))
    J, F, st = ctx.objective(g, dev(S), dev(cands(16, 2)), DR, 3, want_image=True)
    assert np.all(J.cpu().numpy() == 0.0)
    assert np.all(F.cpu().numpy() == 0.0)


@pytest.mark.parametrize("shape,K", [((40, 24, 40, 40), 4), ((48, 20, 62, 48), 3), ((32, 16, 32, 32), 0)])
def test_objective_grad_small(ctx, shape, K):
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=17)
    th = cands(18, 3)
    th[1] = f32(th[1] + np.array([0.3, 0.2, -0.2, 0.1, 0.1, -0.1, 0.01, -0.02]))
    J, G, st = ctx.objective_grad(g, dev(S), dev(th), DR, K, 2)
    J = J.cpu().numpy()
    G = G.cpu().numpy()
    for c in range(3):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, K)
        report(f"grad {shape} K={K} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        print("   gpu   ", np.array2string(G[c], precision=5), "\n   oracle", np.array2string(Gr, precision=5))
        report(f"grad {shape} K={K} cand {c} dJ", G[c], Gr, TOL_GRAD)


@pytest.mark.parametrize("shape,K", [((40, 24, 40, 40), 4), ((48, 20, 62, 48), 3), ((70, 30, 70, 70), 2),
                                     ((192, 12, 192, 192), 2), ((32, 16, 32, 32), 0)])
def test_envelope_gradient(ctx, shape, K):
    # reconstruction held fixed at F^K; 9 components (dR last). n = 192 takes the row-band tail.
    g, og = geom_pair(*shape)
    S, _ = make_slice(og, seed=23)
    th = cands(24, 3)
    th[1] = f32(th[1] + np.array([0.3, 0.2, -0.2, 0.1, 0.1, -0.1, 0.01, -0.02]))
    J, G, st = ctx.objective_grad_ex(g, dev(S), dev(th), DR, K, 5, mode="envelope")
    Jf, _, _ = ctx.objective(g, dev(S), dev(th), DR, K)
    # the objective alone may hold half the angles (opposed-ray pairing): equal to FP32 rounding
    assert torch.allclose(J, Jf, rtol=2e-6, atol=0)
    J = J.cpu().numpy()
    G = G.cpu().numpy()
    assert G.shape == (3, 9)
    for c in range(3):
        Jr, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, K, with_delta_r=True)
        report(f"envelope {shape} K={K} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        print("   gpu   ", np.array2string(G[c], precision=5), "\n   oracle", np.array2string(Gr, precision=5))
        report(f"envelope {shape} K={K} cand {c} dJ", G[c], Gr, TOL_GRAD)


def test_unrolled_gradient_with_delta_r(ctx):
    g, og = geom_pair(40, 24)
    S, _ = make_slice(og, seed=25)
    th = dev(cands(26, 3))
    J9, G9, _ = ctx.objective_grad_ex(g, dev(S), th, DR, 3, 2, mode="unrolled")
    J8, G8, _ = ctx.objective_grad(g, dev(S), th, DR, 3, 2)
    assert torch.equal(J9, J8) and torch.equal(G9[:, :8], G8)
    G9 = G9.cpu().numpy()
    for c in range(3):
        _, Gr = oracle.objective_and_grad(og, S, th[c].cpu().numpy().astype(np.float64), DR, 3, with_delta_r=True)
        report(f"unrolled+dR cand {c} dJ", G9[c], Gr, TOL_GRAD)
        report(f"unrolled+dR cand {c} dJ/d(dR)", G9[c, 8:], Gr[8:], TOL_GRAD)
    with pytest.raises(Exception):
        ctx.objective_grad_ex(g, dev(S), th, DR, 3, 2, mode="nope")


@pytest.mark.parametrize("dr", [0.05, 0.4, 1.5, 3.0])
def test_cranium_thickness_range(ctx, dr):
    # thin to thick shells: the rasterised map, J and both gradients with dJ/d(dR) against the oracle
    g, og = geom_pair(48, 20, 62, 48)
    S, _ = make_slice(og, seed=27)
    th = cands(28, 2)
    mu = ctx.rasterize_mu(g, dev(th), dr).cpu().numpy()
    J, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), dr, 3, 2, mode="unrolled")
    Je, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), dr, 3, 2, mode="envelope")
    J, G, Ge = J.cpu().numpy(), G.cpu().numpy(), Ge.cpu().numpy()
    for c in range(2):
        report(f"dR={dr} mu cand {c}", mu[c], oracle.rasterize_mu(og, th[c], dr), TOL)
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], dr, 3, with_delta_r=True)
        report(f"dR={dr} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"dR={dr} cand {c} dJ", G[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], dr, 3, with_delta_r=True)
        report(f"dR={dr} cand {c} envelope dJ", Ge[c], Gr, TOL_GRAD)


def test_candidates_outside_the_search_box(ctx):
    # no head (c0 = 0), a head past the field of view, harmonics large enough to make R negative in
    # places, no attenuation, and attenuation 13-30x the head's: maps, J, F^K and the gradient against
    # the oracle
    g, og = geom_pair(48, 20, 62, 48)
    S, _ = make_slice(og, seed=29)
    th = f32(np.array([[0.0, 0, 0, 0, 0, 0, 0.15, 0.25],
                       [30.0, 0, 0, 0, 0, 0, 0.15, 0.25],
                       [7.5, 6.0, -5.0, 4.0, -3.0, 2.0, 0.15, 0.25],
                       [7.5, 0, 1.2, 0, -0.3, 0, 0.0, 0.0],
                       [7.5, 0, 1.2, 0, -0.3, 0, 2.0, 5.0]]))
    mu = ctx.rasterize_mu(g, dev(th), DR).cpu().numpy()
    J, F, _ = ctx.objective(g, dev(S), dev(th), DR, 3, want_image=True)
    Jg, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 3, 2, mode="unrolled")
    J, F, G = J.cpu().numpy(), F.cpu().numpy(), G.cpu().numpy()
    for c in range(th.shape[0]):
        mr = oracle.rasterize_mu(og, th[c], DR)
        if np.abs(mr).max() > 0:
            report(f"outside cand {c} mu", mu[c], mr, TOL)
        else:
            assert np.all(mu[c] == 0)
        Jr, Fr, _ = oracle.evaluate(og, S, th[c], DR, 3)
        report(f"outside cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"outside cand {c} F^K", F[c], Fr, TOL)
        _, Gr = oracle.objective_and_grad(og, S, th[c], DR, 3, with_delta_r=True)
        report(f"outside cand {c} dJ", G[c], Gr, TOL_GRAD)


@pytest.mark.parametrize("counts", [5e5, 5e7, 5e9])
def test_objective_at_high_counts(ctx, counts):
    # up to ~4e6 counts per bin, 200 iterations, the true head first: where the model fits, J is a small
    # remainder of sums of S ln y; the library sums the misfit y - S - S ln(y/S) in FP32 and the
    # measurement-only part in FP64, so J keeps the parity gate (the plain per-bin y - S ln y in FP32 was
    # 1e-2 off at 5e9 counts)
    g, og = geom_pair(48, 20, 62, 48)
    S, _ = make_slice(og, seed=31, counts=counts)
    S = f32(S)
    th = cands(30, 2)
    J, _, _ = ctx.objective(g, dev(S), dev(th), DR, 200)
    _, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 200, 5, mode="envelope")
    _, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 50, 5, mode="unrolled")
    J, Ge, G = J.cpu().numpy(), Ge.cpu().numpy(), G.cpu().numpy()
    for c in range(2):
        Jr = oracle.evaluate(og, S, th[c], DR, 200)[0]
        report(f"counts {counts:.0e} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 200, with_delta_r=True)
        report(f"counts {counts:.0e} cand {c} envelope dJ (200 iterations)", Ge[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_grad(og, S, th[c], DR, 50, with_delta_r=True)
        report(f"counts {counts:.0e} cand {c} dJ (50 iterations)", G[c], Gr, TOL_GRAD)


@pytest.mark.parametrize("px", [0.01, 0.05, 2.0, 5.0])
def test_pixel_size_range(ctx, px):
    # a 32-pixel grid from 0.32 cm (the head far larger than the field: nearly uniform attenuation
    # everywhere) to 160 cm (the head a few pixels wide); J and both gradients against the oracle
    g, og = geom_pair(32, 16, 32, 32, pixel=px)
    S, _ = make_slice(og, seed=33)
    th = cands(34, 2)
    J, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 3, 2, mode="unrolled")
    _, Ge, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 3, 2, mode="envelope")
    J, G, Ge = J.cpu().numpy(), G.cpu().numpy(), Ge.cpu().numpy()
    for c in range(2):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 3, with_delta_r=True)
        report(f"pixel {px} cand {c} J", J[c:c + 1], np.array([Jr]), TOL)
        report(f"pixel {px} cand {c} dJ", G[c], Gr, TOL_GRAD)
        _, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 3, with_delta_r=True)
        report(f"pixel {px} cand {c} envelope dJ", Ge[c], Gr, TOL_GRAD)


def test_long_mlem_run(ctx):
    # 1000 iterations: the FP32 iterates stay within 2e-5 of the oracle's FP64 ones, J within 1e-6
    g, og = geom_pair(48, 20, 62, 48)
    S, _ = make_slice(og, seed=35)
    th = cands(36, 2)
    J, F, _ = ctx.objective(g, dev(S), dev(th), DR, 1000, want_image=True)
    J, F = J.cpu().numpy(), F.cpu().numpy()
    for c in range(2):
        Jr, Fr, _ = oracle.evaluate(og, S, th[c], DR, 1000)
        report(f"K=1000 cand {c} J", J[c:c + 1], np.array([Jr]), 1e-6)
        report(f"K=1000 cand {c} F^K", F[c], Fr, 1e-4)


def test_envelope_gradient_adjoint_config_samples(ctx, slice128):
    # 128 x 128, 128 angles, the 64-candidate draw, 20 iterations; two sampled candidates
    g, og = geom_pair(128, 128, pixel=0.2)
    S = slice128["meas"].astype(np.float64)
    import synth
    th = f32(synth.draw_candidates(synth.candidate_stream(1), 64))
    J, G, st = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 20, 5, mode="envelope")
    J = J.cpu().numpy()
    G = G.cpu().numpy()
    assert np.all(np.isfinite(G))
    for c in (3, 50):
        Jr, Gr = oracle.objective_and_envelope_grad(og, S, th[c], DR, 20, with_delta_r=True)
        report(f"envelope64 J cand {c}", J[c:c + 1], np.array([Jr]), TOL)
        report(f"envelope64 dJ cand {c}", G[c], Gr, TOL_GRAD)


def test_checkpoint_interval_does_not_change_results(ctx):
    g, og = geom_pair(40, 24)
    S, _ = make_slice(og, seed=19)
    th = dev(cands(20, 3))
    ref = None
    for ck in (1, 2, 3, 7, 100):
        J, G, _ = ctx.objective_grad(g, dev(S), th, DR, 7, ck)
        if ref is None:
            ref = (J.clone(), G.clone())
        else:
            assert torch.equal(J, ref[0]) and torch.equal(G, ref[1]), ck
    Jf, _, _ = ctx.objective(g, dev(S), th, DR, 7)
    assert torch.allclose(Jf, ref[0], rtol=2e-6, atol=0)  # opposed-ray pairing in the objective alone


def test_objective_grad_adjoint_config_samples(ctx, slice128):
    # 128 x 128, 128 angles, 64 candidates, 20 iterations, checkpoint every 5; two sampled candidates
    # against the oracle's reverse-mode gradient
    g, og = geom_pair(128, 128, pixel=0.2)
    S = slice128["meas"].astype(np.float64)
    import synth
    th = f32(synth.draw_candidates(synth.candidate_stream(1), 64))
    J, G, st = ctx.objective_grad(g, dev(S), dev(th), DR, 20, 5)
    J = J.cpu().numpy()
    G = G.cpu().numpy()
    assert np.all(np.isfinite(G))
    for c in (0, 41):
        Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 20)
        report(f"grad64 J cand {c}", J[c:c + 1], np.array([Jr]), TOL)
        print("   gpu   ", np.array2string(G[c], precision=5), "\n   oracle", np.array2string(Gr, precision=5))
        report(f"grad64 dJ cand {c}", G[c], Gr, TOL_GRAD)


def test_autograd_function(ctx, slice64):
    from paper_2109_11920_amd.api import objective
    g, og = geom_pair(64, 64, pixel=0.4)
    S = dev(slice64["meas"].astype(np.float64))
    th = dev(cands(21, 3)).requires_grad_(True)
    J = objective(ctx, g, S, th, DR, 4, 2)
    w = torch.tensor([1.0, -2.0, 0.5], device="cuda")
    (J * w).sum().backward()
    _, G, _ = ctx.objective_grad(g, S, th.detach(), DR, 4, 2)
    assert torch.allclose(th.grad, w[:, None] * G)


@pytest.mark.parametrize("lanes", ["1", "8"])
def test_evaluate_batch_random_slices_equal_eager(ctx, lanes, monkeypatch):
    # a batch of the second draw's geometries (objective only and with gradients alternating), on one
    # lane or on eight: every slice's J, gradient and status equal the eager entry points bit for bit,
    # on the eager pass and on a graph replay
    from paper_2109_11920_amd.api import SliceBatch
    monkeypatch.setenv("BOAC_BATCH_LANES", lanes)
    slices = []
    for i, (n, na, nb, nt, C, px) in enumerate(RANDOM_CASES):
        g, og = geom_pair(n, na, nb, nt, pixel=px)
        S, _ = make_slice(og, seed=96 + i)
        slices.append(SliceBatch.make(g, dev(S), dev(cands(97 + i, C)), with_grad=(i % 2 == 1)))
    stream = torch.cuda.Stream()
    for rep in range(2):
        for sb in slices:
            sb.obj.fill_(-1)
            if sb.grad is not None:
                sb.grad.fill_(-1)
        stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
        with torch.cuda.stream(stream):
            ctx.evaluate_batch(slices, DR, 3, 2)   # eager pass and capture, then a replay
        stream.synchronize()
        for i, sb in enumerate(slices):
            if sb.grad is None:
                J, _, st = ctx.objective(sb.geom, sb.meas, sb.cand, DR, 3)
                assert torch.equal(sb.obj, J) and torch.equal(sb.status, st), (rep, i)
            else:
                J, G, st = ctx.objective_grad(sb.geom, sb.meas, sb.cand, DR, 3, 2)
                assert torch.equal(sb.obj, J) and torch.equal(sb.grad, G) and torch.equal(sb.status, st), (rep, i)


def test_evaluate_batch_uneven_and_graph_replay(ctx):
    from paper_2109_11920_amd.api import SliceBatch
    shapes = [(96, 16), (128, 24), (192, 12), (256, 8)]
    slices, refs = [], []
    for i, (n, na) in enumerate(shapes):
        g, og = geom_pair(n, na)
        S, _ = make_slice(og, seed=30 + i, counts=2e4)
        th = cands(40 + i, 2 + i % 2)
        slices.append(SliceBatch.make(g, dev(S), dev(th), with_grad=(i % 2 == 0)))
        refs.append((og, S, th))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch(slices, DR, 4, 2)
    stream.synchronize()
    first = [(s.obj.clone(), None if s.grad is None else s.grad.clone()) for s in slices]
    for s in slices:
        s.obj.fill_(0)
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch(slices, DR, 4, 2)   # replays the captured graph
    stream.synchronize()
    for s, (J0, G0) in zip(slices, first):
        assert torch.equal(s.obj, J0)
        if G0 is not None:
            assert torch.equal(s.grad, G0)
    for i, (s, (og, S, th)) in enumerate(zip(slices, refs)):
        for c in range(th.shape[0]):
            if s.grad is not None:
                Jr, Gr = oracle.objective_and_grad(og, S, th[c], DR, 4)
                report(f"batch slice {i} n={og.n} dJ cand {c}", s.grad[c].cpu().numpy(), Gr, TOL_GRAD)
            else:
                Jr = oracle.evaluate(og, S, th[c], DR, 4)[0]
            report(f"batch slice {i} n={og.n} J cand {c}", s.obj[c:c + 1].cpu().numpy(), np.array([Jr]), TOL)


@pytest.mark.parametrize("split", ["1", "2"])
def test_evaluate_batch_split_slice_matches_eager(ctx, slice64, split, monkeypatch):
    # one slice of 130 candidates, whole on one lane (BOAC_BATCH_SPLIT=1, the default) or as two halves
    # on two lanes (130 = 64 + 66: the split point is rounded for alignment); objective, status and
    # gradient equal the eager entry points bit for bit
    from paper_2109_11920_amd.api import SliceBatch
    monkeypatch.setenv("BOAC_BATCH_SPLIT", split)
    g, og = geom_pair(64, 64, pixel=0.4)
    S = dev(slice64["meas"].astype(np.float64))
    th = dev(cands(50, 130))
    sb = SliceBatch.make(g, S, th, with_grad=True)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch([sb], DR, 3, 2)
    stream.synchronize()
    J, G, st = ctx.objective_grad(g, S, th, DR, 3, 2)
    assert torch.equal(sb.obj, J) and torch.equal(sb.grad, G) and torch.equal(sb.status, st)
    Jf, _, stf = ctx.objective(g, S, th, DR, 3)
    sf = SliceBatch.make(g, S, th, with_grad=False)
    stream.wait_stream(torch.cuda.current_stream())  # calls on one context do not overlap
    with torch.cuda.stream(stream):
        ctx.evaluate_batch([sf], DR, 3, 2)
    stream.synchronize()
    assert torch.equal(sf.obj, Jf) and torch.equal(sf.status, stf)
    Jr = oracle.evaluate(og, slice64["meas"].astype(np.float64), cands(50, 130)[129], DR, 3)[0]
    report("split slice J cand 129", sf.obj[129:130].cpu().numpy(), np.array([Jr]), TOL)


def test_launch_configurations_agree(slice64, tmp_path):
    # every tile shape / candidates-per-workgroup / ray blocking the autotuner may choose gives the
    # same objective and gradient within one backprojection kernel family (the per-candidate arithmetic
    # does not depend on the launch shape); the families (general, slot-staged and column-group-staged
    # slid block) round the window offsets or apply the ray weights differently and agree to FP32
    # rounding
    import json
    from paper_2109_11920_amd.api import Context
    from paper_2109_11920_amd.autotune import BACK_CONFIGS, RAY_CONFIGS, key
    g, og = geom_pair(64, 64, pixel=0.4)
    S = dev(slice64["meas"].astype(np.float64))
    C = 16
    th = dev(cands(22, C))
    results = []
    configs = [(r, b) for r in RAY_CONFIGS[:3] for b in BACK_CONFIGS] + [(r, BACK_CONFIGS[0]) for r in RAY_CONFIGS[3:]]
    for i, ((blk, rpt), (tw, th_, cg, slid)) in enumerate(configs):
        pair = i % 2  # the paired forward projection must give the same bits as one candidate per workgroup
        path = tmp_path / f"tune_{blk}_{rpt}_{tw}_{th_}_{cg}_{slid}.json"
        path.write_text(json.dumps({key("ray", g, C, 1): [blk, rpt, pair], key("ray", g, C, 2): [blk, rpt],
                                    key("back", g, C, 0): [tw, th_, cg, 1, slid]}))
        with Context(0, tune_cache=str(path)) as c2:
            J, G, _ = c2.objective_grad(g, S, th, DR, 3, 2)
            results.append(((blk, rpt, tw, th_, cg, slid), J.cpu().numpy(), G.cpu().numpy()))
    ref = {}
    for cfg, J, G in results:
        r = ref.setdefault(cfg[-1], (J, G))
        assert np.array_equal(J, r[0]) and np.array_equal(G, r[1]), cfg
    assert set(ref) == {0, 1, 2}
    J0, G0 = ref[0]
    for fam in (1, 2):
        J1, G1 = ref[fam]
        assert np.max(np.abs(J1 - J0) / np.abs(J0)) < 1e-6, fam
        assert np.linalg.norm(G1 - G0) / np.linalg.norm(G0) < 1e-5, fam
    ref = results[0]
    Jr, Gr = oracle.objective_and_grad(og, slice64["meas"].astype(np.float64), cands(22, C)[0], DR, 3)
    report("launch configs J cand 0", ref[1][:1], np.array([Jr]), TOL)
    report("launch configs dJ cand 0", ref[2][0], Gr, TOL_GRAD)


@pytest.mark.parametrize("shape,pixel", [((128, 128, 128, 128), 0.2), ((64, 64, 64, 64), 0.4), ((40, 24, 40, 40), None),
                                         ((70, 30, 70, 70), None)])
def test_few_candidate_plans_equal_the_unsplit_kernels(ctx, shape, pixel, monkeypatch):
    # few candidates: the projection splits each ray over 8 lanes and the column-group gather splits its
    # angles over workgroups (a second pass adds the 8-angle blocks in order); both reproduce the
    # one-thread-per-ray projection and the unsplit gather bit for bit, in every entry point
    g, og = geom_pair(*shape, pixel=pixel)
    S, _ = make_slice(og, seed=51)
    th = cands(52, 2)
    th[1] = f32(th[1] + np.array([0.3, 0.2, -0.2, 0.1, 0.1, -0.1, 0.01, -0.02]))
    runs = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BOAC_FWD_SPLIT", flag)
        monkeypatch.setenv("BOAC_GATHER_SPLIT", flag)
        J, F, _ = ctx.objective(g, dev(S), dev(th), DR, 7, want_image=True)
        J1, F1, _ = ctx.objective(g, dev(S), dev(th[1:]), DR, 7, want_image=True)
        mu = ctx.rasterize_mu(g, dev(th), DR)
        y = ctx.project(g, mu, F)
        x = ctx.backproject(g, mu, y)
        Jg, G, _ = ctx.objective_grad_ex(g, dev(S), dev(th), DR, 3, 2, mode="unrolled")
        runs[flag] = [t.cpu().numpy() for t in (J, F, J1, F1, y, x, Jg, G)]
    for name, a, b in zip(("J", "F^K", "J C=1", "F^K C=1", "A f", "A^T y", "J grad", "dJ"), runs["1"], runs["0"]):
        report(f"few-candidate plans {shape} {name}", a, b, 1e-6)
        assert np.array_equal(a, b), name
    # one candidate at a time equals the batch of two
    assert np.array_equal(runs["1"][2][0], runs["1"][0][1]) and np.array_equal(runs["1"][3][0], runs["1"][1][1])
    Jr, Fr, _ = oracle.evaluate(og, S, th[1], DR, 7)
    report(f"few-candidate plans {shape} J vs oracle", runs["1"][2], np.array([Jr]), TOL)
    report(f"few-candidate plans {shape} F^K vs oracle", runs["1"][3][0], Fr, TOL)


@pytest.mark.parametrize("shape,pixel", [((128, 128, 128, 128), 0.2), ((40, 24, 40, 40), None), ((36, 16, 36, 50), None),
                                         ((96, 64, 96, 96), None)])
def test_lane_parallel_attenuation_scan(ctx, shape, pixel, monkeypatch):
    # the attenuation scan spread over 8 lanes per ray against the one-thread-per-ray scan (same samples,
    # another compensated summation order) and against the oracle, through the projector
    g, og = geom_pair(*shape, pixel=pixel)
    th = cands(53, 3)
    mus = f32(np.stack([oracle.rasterize_mu(og, th[c], DR) for c in range(3)]))
    imgs = f32(np.random.default_rng(54).uniform(0.0, 2.0, (3, og.n, og.n)))
    out = {}
    for flag in ("1", "0"):
        monkeypatch.setenv("BOAC_ATT_SCAN", flag)
        out[flag] = ctx.project(g, dev(mus), dev(imgs)).cpu().numpy()
    report(f"att scan lanes vs thread {shape}", out["1"], out["0"], 2e-6)
    for c in range(3):
        ref = oracle.project(og, oracle.attenuation(og, mus[c]), imgs[c])
        report(f"att scan lanes {shape} cand {c} vs oracle", out["1"][c], ref, TOL)
