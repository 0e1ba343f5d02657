"""The library's host surrogate fit (boac_gp_fit, native FP64) against the oracle's GP on the same
seeded observations. No GPU is involved."""
import numpy as np
import pytest

import oracle.bo as obo
from paper_2109_11920_amd.api import BoacError, gp_fit


def _obs(n, d, seed):
    rng = np.random.default_rng(seed)
    U = rng.uniform(size=(n, d))
    y = 1e5 + 300 * np.sum((U - 0.4) ** 2, axis=1) + 20 * np.sin(5 * U[:, 0]) + rng.normal(scale=0.05, size=n)
    return U, y


@pytest.mark.parametrize("n,d,n_select", [(1, 8, 0), (2, 8, 0), (37, 8, 0), (150, 8, 64), (300, 3, 0),
                                          (64, 1, 0), (65, 64, 0), (129, 9, 100), (520, 5, 0)])
def test_gp_fit_matches_oracle(n, d, n_select):
    U, y = _obs(n, d, n)
    m = gp_fit(U, y, obo.LENGTH_GRID, n_select=n_select, noise=obo.NOISE)
    ref = obo.fit_gp(U, y, obo.LENGTH_GRID, obo.NOISE, n_select=n_select or None)
    assert m.info.length == ref.length
    assert m.info.n == n and m.info.d == d
    assert m.info.m0 == pytest.approx(ref.m0, rel=1e-14)
    assert m.info.s == pytest.approx(ref.s, rel=1e-12)
    assert m.info.lml == pytest.approx(ref.log_marginal_likelihood(), rel=1e-9, abs=1e-9)
    np.testing.assert_allclose(m.alpha, ref.alpha, rtol=1e-7, atol=1e-9 * np.abs(ref.alpha).max())
    Linv_ref = np.linalg.inv(ref.L)
    err = np.linalg.norm(m.linv - Linv_ref) / np.linalg.norm(Linv_ref)
    print(f"[parity] gp_fit n={n} d={d}: length {m.info.length:.4g} L^-1 rel_l2={err:.2e}")
    # both inverses carry a forward error of order n eps cond(L); cond(L) = sqrt(cond(K)) ~ sqrt(n / noise)
    tol = 10 * n * np.finfo(float).eps * np.linalg.cond(ref.L)
    assert err < tol, (err, tol)
    assert np.all(np.triu(m.linv, 1) == 0)
    # the factor inverts the covariance: L^-1 K L^-T = I
    K = obo.rbf(U, U, 1.0, m.info.length) + obo.NOISE * np.eye(n)
    np.testing.assert_allclose(m.linv @ K @ m.linv.T, np.eye(n), atol=1e-6)


def test_gp_fit_rejects_bad_input():
    U, y = _obs(5, 2, 0)
    with pytest.raises(BoacError):
        gp_fit(U, y, [0.0])
    y2 = y.copy()
    y2[1] = np.nan
    with pytest.raises(BoacError):
        gp_fit(U, y2, obo.LENGTH_GRID)
    # duplicated inputs without a nugget: singular covariance for every length
    with pytest.raises(BoacError):
        gp_fit(np.vstack([U, U[:1]]), np.append(y, y[0]), obo.LENGTH_GRID, noise=0.0)
