"""Host logic of the BOAC outer loop (no GPU): batch selection with exclusion, line-search proposals,
and journal records."""
import numpy as np

from paper_2109_11920_amd.bo import Cycle, greedy_select, line_search_points


def test_greedy_select_orders_by_score_and_excludes_neighbours():
    U = np.array([[0.5, 0.5], [0.505, 0.5], [0.1, 0.1], [0.9, 0.9], [0.101, 0.1]])
    score = np.array([5.0, 4.0, 3.0, 1.0, 2.9])
    assert greedy_select(U, score, 3, 0.02) == [0, 2, 3]
    assert greedy_select(U, score, 10, 0.0) == [0, 1, 2, 4, 3]
    # points near what is already taken are skipped
    assert greedy_select(U, score, 2, 0.02, taken=np.array([[0.5, 0.51]])) == [2, 3]
    # ties keep the lower index first; non-finite scores end the selection
    assert greedy_select(U, np.array([1.0, 1.0, np.nan, 1.0, 0.5]), 5, 0.0)[:3] == [0, 1, 3]


def test_line_search_points_follow_the_negative_gradient():
    u0 = np.array([0.5, 0.5, 0.5])
    g = np.array([3.0, 0.0, -4.0])
    P = line_search_points(u0, g, steps=(0.1, 0.2))
    np.testing.assert_allclose(P, [[0.44, 0.5, 0.58], [0.38, 0.5, 0.66]])
    # clipped to the unit box; a zero gradient proposes nothing
    P = line_search_points(np.array([0.99, 0.5]), np.array([-1.0, 0.0]), steps=(0.5,))
    np.testing.assert_allclose(P, [[1.0, 0.5]])
    assert line_search_points(u0, np.zeros(3)).shape == (0, 3)


def test_cycle_journal_record_round_trips():
    c = Cycle(2, np.arange(16.0).reshape(2, 8), np.array([1.5, np.inf]), None, np.array([0, 1]), ["ei", "line"],
              0.25, 0.4, {"fit_ms": 1.0})
    import json
    r = Cycle.from_json(json.loads(json.dumps(c.to_json())))
    assert r.index == 2 and r.kind == ["ei", "line"] and r.grad is None
    np.testing.assert_array_equal(r.theta, c.theta)
    np.testing.assert_array_equal(r.J, c.J)


def test_acquisition_search_equals_the_oracle_search():
    # the library's chaotic search (step 5) and the oracle's reading of it, from the same chains, on a
    # closed-form acquisition with distinct values: identical proposals, largest value and evaluation count
    import oracle.bo as obo
    from paper_2109_11920_amd.bo import chaotic_acquire

    d = 8
    a = np.linspace(0.2, 0.8, d)
    b = np.full(d, 0.35)

    def acq(U):
        U = np.asarray(U, np.float64)
        return (np.exp(-np.sum((U - a) ** 2, axis=1) / 0.08) + 0.6 * np.exp(-np.sum((U - b) ** 2, axis=1) / 0.02)
                + 1e-3 * (1.0 + U[:, 0] + 0.37 * U[:, 3]))

    rng = np.random.default_rng(2024)
    for q, chains, exclusion in ((12, 512, 0.02), (3, 300, 0.2)):
        z = rng.uniform(0.01, 0.99, size=(chains, d))
        taken = rng.uniform(size=(40, d))
        kw = dict(n_global=6, n_local=10, centres=8, radius0=0.1, shrink=0.85, exclusion=exclusion,
                  per_step=max(4 * q, 64))
        U, best, m = chaotic_acquire(acq, z, q, taken, **kw)
        Ur, best_r, m_r = obo.chaotic_search(acq, z, q, taken, **kw)
        assert m == m_r and best == best_r
        np.testing.assert_array_equal(U, Ur)
        assert len(U) == q


def test_round_pool_keeps_the_best_with_ties_by_lower_index():
    # each round of the search keeps its per_step best points, ties by lower index: the same set as a
    # stable sort in decreasing value, also with many tied values
    from paper_2109_11920_amd.bo import chaotic_acquire
    rng = np.random.default_rng(5)
    for levels in (3, 40, 10 ** 6):
        vals = rng.integers(0, levels, size=512).astype(np.float64)
        z = rng.uniform(0.01, 0.99, size=(512, 2))
        seen = []

        def acq(U):
            seen.append(np.asarray(U, np.float64).copy())
            return vals[: len(U)] if len(U) == 512 else np.zeros(len(U))

        # one global round, no local rounds: the pool is that round's kept points; q = per_step picks with no
        # exclusion return exactly the kept set in decreasing value
        U, best, m = chaotic_acquire(acq, z, 48, None, n_global=1, n_local=0, centres=1, radius0=0.1, shrink=0.85,
                                     exclusion=0.0, per_step=48)
        ref = np.sort(np.argsort(-vals, kind="stable")[:48])
        order = ref[np.argsort(-vals[ref], kind="stable")]
        np.testing.assert_array_equal(U, z[order])
