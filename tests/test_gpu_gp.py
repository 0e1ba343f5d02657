"""GPU parity of the surrogate acquisition (boac_gp_ei, FP64) against the oracle's GP posterior and
expected improvement on the same fitted observations. Query counts and observation counts are not
multiples of the 64-wide blocks; queries include the observations themselves (sigma near 0) and
points far outside the data (sigma near the prior)."""
import numpy as np
import pytest

import oracle.bo as obo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2109_11920_amd.api import Context
    c = Context(0)
    yield c
    c.close()


def _obs(n, d, seed):
    rng = np.random.default_rng(seed)
    U = rng.uniform(size=(n, d))
    y = 1e5 + 300 * np.sum((U - 0.4) ** 2, axis=1) + 20 * np.sin(5 * U[:, 0]) + rng.normal(scale=0.05, size=n)
    return U, y


@pytest.mark.parametrize("n,M,xi,d", [(1, 100, 0.0, 8), (37, 4999, 0.01, 8), (150, 2000, 0.0, 8), (300, 3001, 0.5, 8),
                                      (5, 777, 0.0, 1), (65, 1025, 0.02, 3), (200, 300, 0.0, 9), (129, 2048, 0.1, 64),
                                      (700, 20000, 0.0, 8)])
def test_gp_ei_matches_oracle(ctx, n, M, xi, d):
    # observation counts on both sides of the 64-row blocks, one to 64 dimensions
    from paper_2109_11920_amd.api import gp_fit
    U, y = _obs(n, d, 100 + n)
    m = gp_fit(U, y, obo.LENGTH_GRID, noise=obo.NOISE)
    ref = obo.fit_gp(U, y, obo.LENGTH_GRID, obo.NOISE)
    assert m.info.length == ref.length
    rng = np.random.default_rng(n)
    Q = np.vstack([rng.uniform(size=(M - n - 2, d)), U, np.full((2, d), 3.0)])
    best = float(y.min())
    q = torch.as_tensor(Q, device="cuda")
    ei, mu, sd = ctx.gp_ei(m, q, best, xi, want_mu_sigma=True)
    torch.cuda.synchronize()
    ei, mu, sd = ei.cpu().numpy(), mu.cpu().numpy(), sd.cpu().numpy()
    mu_r, sd_r = ref.predict(Q)
    ei_r = obo.expected_improvement(mu_r, sd_r, best, xi)
    e_mu = np.abs(mu - mu_r).max() / ref.s
    e_sd = np.abs(sd - sd_r).max() / ref.s
    e_ei = np.abs(ei - ei_r).max() / ref.s
    print(f"[parity] gp_ei n={n} d={d} M={M}: max|dmu|/s={e_mu:.2e} max|dsigma|/s={e_sd:.2e} max|dEI|/s={e_ei:.2e}",
          flush=True)
    assert e_mu < 1e-8 and e_sd < 1e-6 and e_ei < 1e-6
    assert np.all(ei >= 0) and np.all(sd >= 0)
    # far queries revert to the prior
    np.testing.assert_allclose(sd[-2:], ref.s, rtol=1e-12)
    # the argmax of EI (what the search uses) is the oracle's
    assert int(np.argmax(ei)) == int(np.argmax(ei_r))


def test_gp_ei_is_deterministic(ctx):
    from paper_2109_11920_amd.api import gp_fit
    U, y = _obs(90, 8, 7)
    m = gp_fit(U, y, obo.LENGTH_GRID)
    q = torch.rand((1000, 8), device="cuda", dtype=torch.float64, generator=torch.Generator("cuda").manual_seed(0))
    a = ctx.gp_ei(m, q, float(y.min()), 0.0)
    b = ctx.gp_ei(m, q, float(y.min()), 0.0)
    assert torch.equal(a, b)


@pytest.mark.parametrize("P,nc,n_local", [(512, 8, 10), (300, 7, 6), (4096, 8, 32)])
def test_device_local_search_equals_host_search(ctx, P, nc, n_local):
    # the acquisition search's local stage on the device (boac_gp_chaos_local) against the host loop of
    # the same search on the same surrogate: every round's points equal the host's bit for bit (FP64, same
    # operation order) and its EI values equal boac_gp_ei at those points; the proposals of the whole
    # search are the host search's
    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd.bo import chaotic_acquire
    d = 8
    U0, y = _obs(90, d, 7)
    m = gp_fit(U0, y, obo.LENGTH_GRID, noise=obo.NOISE)
    best = float(y.min())
    rng = np.random.default_rng(P + nc)
    z = rng.uniform(0.01, 0.99, size=(P, d))
    C = rng.uniform(size=(nc, d))
    f64 = torch.float64

    def ei_of(Q):
        return ctx.gp_ei(m, torch.as_tensor(np.ascontiguousarray(Q), device="cuda"), best, 0.0).cpu().numpy()

    Ce = ei_of(C)
    zt, Ct, Cet = (torch.tensor(a, dtype=f64, device="cuda") for a in (z, C, Ce))
    pts, vals = ctx.gp_chaos_local(m, best, 0.0, zt, Ct, Cet, 0.1, 0.85, n_local)
    torch.cuda.synchronize()
    pts, vals = pts.cpu().numpy(), vals.cpu().numpy()
    # the host loop
    per = P // nc
    zh, Ch, Ceh, r = z.copy(), C.copy(), Ce.copy(), 0.1
    for t in range(n_local):
        zz = zh[:per * nc].reshape(nc, per, d)
        Uh = np.clip(Ch[:, None, :] + r * (2.0 * zz - 1.0), 0.0, 1.0).reshape(-1, d)
        np.testing.assert_array_equal(pts[t], Uh)
        eh = ei_of(Uh)
        np.testing.assert_array_equal(vals[t], eh)
        e2 = eh.reshape(nc, per)
        j = np.argmax(e2, axis=1)
        better = e2[np.arange(nc), j] > Ceh
        Ch[better] = Uh.reshape(nc, per, d)[better, j[better]]
        Ceh[better] = e2[better, j[better]]
        zh = 4.0 * zh * (1.0 - zh)
        r *= 0.85
    np.testing.assert_array_equal(Ct.cpu().numpy(), Ch)
    np.testing.assert_array_equal(Cet.cpu().numpy(), Ceh)
    np.testing.assert_array_equal(zt.cpu().numpy(), zh)
    # the whole search, with and without the device stage
    def local(zl, Cl, Cel, r0):
        a, b = ctx.gp_chaos_local(m, best, 0.0, torch.tensor(zl, dtype=f64, device="cuda"),
                                  torch.tensor(Cl, dtype=f64, device="cuda"),
                                  torch.tensor(Cel, dtype=f64, device="cuda"), r0, 0.85, n_local)
        return a.cpu().numpy(), b.cpu().numpy()

    taken = rng.uniform(size=(20, d))
    kw = dict(n_global=4, n_local=n_local, centres=nc, radius0=0.1, shrink=0.85, exclusion=0.02, per_step=64)
    Ua, ba, na = chaotic_acquire(ei_of, z, 6, taken, **kw)
    Ub, bb, nb = chaotic_acquire(ei_of, z, 6, taken, local=local, **kw)
    np.testing.assert_array_equal(Ua, Ub)
    assert ba == bb and na == nb
    print(f"[parity] device local search P={P} centres={nc} rounds={n_local}: points, EI, centres and "
          f"proposals identical to the host search", flush=True)


def test_device_local_search_rejects_bad_sizes(ctx):
    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd._lib import BoacError
    U0, y = _obs(20, 8, 3)
    m = gp_fit(U0, y, obo.LENGTH_GRID, noise=obo.NOISE)
    f64 = torch.float64
    z = torch.full((4, 8), 0.3, dtype=f64, device="cuda")
    C = torch.full((5, 8), 0.5, dtype=f64, device="cuda")
    with pytest.raises(BoacError):
        ctx.gp_chaos_local(m, 0.0, 0.0, z, C, torch.zeros(5, dtype=f64, device="cuda"), 0.1, 0.85, 2)


@pytest.mark.parametrize("P,q,centres,n_global,n_local,exclusion,per_step,n_taken",
                         [(512, 12, 8, 6, 10, 0.02, 64, 40), (300, 3, 8, 4, 6, 0.2, 64, 0), (4096, 64, 8, 16, 32, 0.02, 256, 320),
                          (700, 20, 5, 3, 0, 0.05, 100, 10),
                          # every round's points kept (per_step > P), and an exclusion that leaves fewer than q
                          (200, 64, 8, 3, 4, 1.2, 256, 5),
                          # one chain; no exclusion (equal points may both be proposed); the most chains
                          (1, 1, 1, 1, 0, 0.0, 1, 0), (17, 5, 3, 2, 3, 0.0, 4, 2), (8192, 8, 8, 2, 2, 0.05, 8, 0)])
def test_device_search_equals_host_search(ctx, P, q, centres, n_global, n_local, exclusion, per_step, n_taken):
    # the whole acquisition search on the device (boac_gp_chaos_search) against the host search
    # (chaotic_acquire around boac_gp_ei) from the same chains: the same proposals in the same order, the
    # same largest EI and evaluation count
    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd.bo import chaotic_acquire
    d = 8
    U0, y = _obs(120, d, 17)
    m = gp_fit(U0, y, obo.LENGTH_GRID, noise=obo.NOISE)
    best = float(y.min())
    rng = np.random.default_rng(P + q)
    z = rng.uniform(0.01, 0.99, size=(P, d))
    taken = np.vstack([U0[:n_taken // 2], rng.uniform(size=(n_taken - n_taken // 2, d))]) if n_taken else None

    def ei_of(Q):
        return ctx.gp_ei(m, torch.as_tensor(np.ascontiguousarray(Q), device="cuda"), best, 0.0).cpu().numpy()

    kw = dict(n_global=n_global, n_local=n_local, centres=centres, radius0=0.1, shrink=0.85, exclusion=exclusion,
              per_step=per_step)
    Uh, vh, nh = chaotic_acquire(ei_of, z, q, taken, **kw)
    zt = torch.tensor(z, dtype=torch.float64, device="cuda")
    tk = None if taken is None else torch.tensor(taken, dtype=torch.float64, device="cuda")
    Ud, vd, nd = ctx.gp_chaos_search(m, best, 0.0, zt, tk, q, **kw)
    Ud = Ud.cpu().numpy()
    np.testing.assert_array_equal(zt.cpu().numpy(), z)  # the chains are not modified
    assert nd == nh and vd == vh, (nd, nh, vd, vh)
    np.testing.assert_array_equal(Ud, Uh)
    if exclusion >= 1.0:
        assert len(Ud) < q   # the case meant: the pool runs out before q proposals
    print(f"[parity] device search P={P} q={q} rounds {n_global}+{n_local}: {len(Ud)} proposals, largest EI and "
          f"{nd} evaluations identical to the host search", flush=True)


def test_device_search_many_tied_values(ctx):
    # with a length-scale far below the points' spacing, the posterior at almost every query is exactly
    # the prior, so most EI values are equal: the pools and the greedy choice then rest on the tie rule
    # (lower index first) throughout
    from paper_2109_11920_amd.api import gp_fit
    from paper_2109_11920_amd.bo import chaotic_acquire
    d = 8
    rng = np.random.default_rng(3)
    U0 = 0.5 + 0.01 * rng.uniform(size=(30, d))
    y = 1e5 + 1e4 * np.sum((U0 - 0.5) ** 2, axis=1)
    m = gp_fit(U0, y, np.array([0.01, 0.02]), noise=obo.NOISE)
    best = float(y.min())
    z = rng.uniform(0.01, 0.99, size=(1024, d))

    def ei_of(Q):
        return ctx.gp_ei(m, torch.as_tensor(np.ascontiguousarray(Q), device="cuda"), best, 0.0).cpu().numpy()

    e = ei_of(z)
    vals, counts = np.unique(e, return_counts=True)
    assert counts.max() > len(e) // 2   # the case this test is for: one value shared by most queries
    kw = dict(n_global=3, n_local=4, centres=8, radius0=0.1, shrink=0.85, exclusion=0.01, per_step=128)
    Uh, vh, nh = chaotic_acquire(ei_of, z, 16, None, **kw)
    Ud, vd, nd = ctx.gp_chaos_search(m, best, 0.0, torch.tensor(z, device="cuda"), None, 16, **kw)
    assert nd == nh and vd == vh
    np.testing.assert_array_equal(Ud.cpu().numpy(), Uh)
