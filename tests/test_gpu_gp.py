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


@pytest.mark.parametrize("n,M,xi", [(1, 100, 0.0), (37, 4999, 0.01), (150, 2000, 0.0), (300, 3001, 0.5)])
def test_gp_ei_matches_oracle(ctx, n, M, xi):
    from paper_2109_11920_amd.api import gp_fit
    d = 8
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
    print(f"[parity] gp_ei n={n} M={M}: max|dmu|/s={e_mu:.2e} max|dsigma|/s={e_sd:.2e} max|dEI|/s={e_ei:.2e}",
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
