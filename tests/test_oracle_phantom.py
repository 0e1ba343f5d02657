"""Pins for the oracle's phantom generator (the simulation study's numerical phantoms, read as: activity
1 in the true head's brain, three hot disks of radius 0.8-1.5 cm at 4x activity, overlaps by maximum,
centres rejection-sampled until 64 rim points lie inside the outline).

Each pin checks a property fixed by the geometry rather than by the code: the disk's area is pi rho^2,
its centroid is (cx, cy) with x along image columns, the accepted disks lie inside an outline computed
independently of the oracle (numpy's Legendre series), the plateaus are exactly 1 and 4, overlaps take
the maximum. Every pin is paired with a planted mistake that must make it fail."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import oracle.phantom as ph

G = oracle.Geometry(64, 8, 64, 64, 0.4)
TRUE_C = np.array([7.5, 0.0, 1.2, 0.0, -0.3, 0.0])


def _xy(g):
    x = (np.arange(g.n) - (g.n - 1) / 2.0) * g.pixel
    return x[None, :], x[:, None]        # column coordinate x_l, row coordinate y_i


def _outline(c, theta):
    """R(theta) = sum_k c_k P_k(cos theta) through numpy's Legendre series (independent of the oracle)."""
    return npleg.legval(np.cos(theta), np.asarray(c, np.float64))


# ---------------------------------------------------------------- disk coverage
DISKS = [(2.3, -1.1, 1.2), (-3.7, 4.05, 0.8), (0.13, 0.41, 1.5)]


def _pin_disk_coverage(fn, g=G):
    X, Y = _xy(g)
    for cx, cy, rho in DISKS:
        cov = fn(g, cx, cy, rho)
        assert cov.shape == (g.n, g.n)
        assert cov.min() >= 0.0 and cov.max() <= 1.0
        area = cov.sum() * g.pixel ** 2
        assert area == pytest.approx(math.pi * rho * rho, rel=3e-3), (cx, cy, rho, area)
        # centroid: x is the column coordinate, y the row coordinate
        w = cov.sum()
        assert (cov * X).sum() / w == pytest.approx(cx, abs=0.02 * g.pixel)
        assert (cov * Y).sum() / w == pytest.approx(cy, abs=0.02 * g.pixel)
        # exactly 1 well inside (distance + half the pixel diagonal below rho - h/2), exactly 0 well outside
        r = np.hypot(X - cx, Y - cy)
        half_diag = g.pixel / math.sqrt(2.0)
        h = g.pixel / 4
        assert np.all(cov[r + half_diag < rho - h / 2] == 1.0)
        assert np.all(cov[r - half_diag > rho + h / 2] == 0.0)


def test_disk_coverage_area_centroid_and_plateaus():
    _pin_disk_coverage(ph.disk_coverage)


@pytest.mark.parametrize("mistake", ["swapped_axes", "diameter_for_radius", "transposed", "hard_edge_shift"])
def test_planted_disk_coverage_mistakes_fail(mistake):
    real = ph.disk_coverage
    wrong = {
        "swapped_axes": lambda g, cx, cy, rho: real(g, cy, cx, rho),
        "diameter_for_radius": lambda g, cx, cy, rho: real(g, cx, cy, 0.5 * rho),
        "transposed": lambda g, cx, cy, rho: real(g, cx, cy, rho).T,
        # a half-pixel offset of the sampling grid
        "hard_edge_shift": lambda g, cx, cy, rho: real(g, cx + 0.5 * g.pixel, cy, rho),
    }[mistake]
    with pytest.raises(AssertionError):
        _pin_disk_coverage(wrong)


# ---------------------------------------------------------------- disk placement
def _pin_placement(c, disks, n, r_lo, r_hi):
    assert len(disks) == n
    th = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
    rmax = float(_outline(c, th).max())
    alpha = 2.0 * np.pi * np.arange(64) / 64
    for cx, cy, rho in disks:
        assert r_lo <= rho <= r_hi
        assert -rmax <= cx <= rmax and -rmax <= cy <= rmax
        px, py = cx + rho * np.cos(alpha), cy + rho * np.sin(alpha)
        # every one of the 64 rim points strictly inside the outline
        assert np.all(np.hypot(px, py) < _outline(c, np.arctan2(py, px))), (cx, cy, rho)


def _scripted(triples):
    for t in triples:
        yield t
    raise AssertionError("proposal stream exhausted")


def test_place_disks_accepts_only_disks_inside_the_outline():
    import synth
    rng = synth.streams(0)[0]
    disks = ph.place_disks(TRUE_C, synth.disk_proposals(rng), 3, 0.8, 1.5)
    _pin_placement(TRUE_C, disks, 3, 0.8, 1.5)


def _u_of(c, x):
    """Proposal coordinate mapping to centre coordinate x in the outline's bounding box."""
    th = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
    rmax = float(_outline(c, th).max())
    return (x + rmax) / (2.0 * rmax)


# R(90 deg) = 7.5 - 0.6 - 0.1125 = 6.7875 cm: a radius-1.5 disk centred at (0, 5.8) has its centre well
# inside but its top rim point at 7.3 cm, outside the outline (and inside the outline grown by 1 cm)
CROSSING = (1.0, 0.5, _u_of(TRUE_C, 5.8))


def test_place_disks_maps_and_rejects_proposals():
    th = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
    rmax = float(_outline(TRUE_C, th).max())
    props = [(0.5, 0.0, 0.0),      # centre at the bounding box's corner: outside, rejected
             (0.0, 0.5, 0.5),      # centre at the origin, radius 0.8: inside, accepted
             CROSSING,             # centre inside, rim crossing the outline: rejected
             (1.0, 0.6, 0.45)]     # radius 1.5 near the centre: accepted
    disks = ph.place_disks(TRUE_C, _scripted(props), 2, 0.8, 1.5)
    assert disks[0] == pytest.approx((0.0, 0.0, 0.8), abs=1e-15)
    assert disks[1] == pytest.approx((-rmax + 2 * rmax * 0.6, -rmax + 2 * rmax * 0.45, 1.5), rel=1e-12)
    _pin_placement(TRUE_C, disks, 2, 0.8, 1.5)


def test_planted_lenient_rim_test_fails(monkeypatch):
    # an outline test 1 cm too generous (its bounding box grows by 1 cm too) accepts a radius-1.5 disk
    # centred at (0, 5.8), whose top rim point lies outside the true outline
    real = ph.head_radius
    monkeypatch.setattr(ph, "head_radius", lambda c, cos_t: real(c, cos_t) + 1.0)
    lenient_c = TRUE_C + np.array([1.0, 0, 0, 0, 0, 0])   # P_0 = 1: the same outline grown by 1 cm
    props = [(1.0, 0.5, _u_of(lenient_c, 5.8)), (0.0, 0.5, 0.5)]
    disks = ph.place_disks(TRUE_C, _scripted(props), 1, 0.8, 1.5)
    with pytest.raises(AssertionError):
        _pin_placement(TRUE_C, disks, 1, 0.8, 1.5)


def test_planted_wrong_radius_range_fails():
    import synth
    real = ph.place_disks
    # radii drawn from [0.8, 3.0] instead of [0.8, 1.5]
    disks = real(TRUE_C, synth.disk_proposals(np.random.default_rng(7)), 6, 0.8, 3.0)
    with pytest.raises(AssertionError):
        _pin_placement(TRUE_C, disks, 6, 0.8, 1.5)


# ---------------------------------------------------------------- activity phantom
TWO_OVERLAPPING = [(1.0, 0.5, 1.4), (2.2, 0.5, 1.4)]   # centres 1.2 cm apart: a lens-shaped overlap


def _pin_activity(fn, g=G):
    f = fn(g, TRUE_C, 0.8, TWO_OVERLAPPING, 1.0, 4.0)
    X, Y = _xy(g)
    r = np.hypot(X, Y)
    R = _outline(TRUE_C, np.arctan2(Y, X))
    half_diag = g.pixel / math.sqrt(2.0)
    h = g.pixel / 4
    margin = half_diag + h
    d1 = np.hypot(X - 1.0, Y - 0.5)
    d2 = np.hypot(X - 2.2, Y - 0.5)
    inside_brain = r + margin < R
    outside_head = r - margin > R + 0.8 + h
    in_disk = (d1 + margin < 1.4) | (d2 + margin < 1.4)
    off_disks = (d1 - margin > 1.4) & (d2 - margin > 1.4)
    assert f.min() >= 0.0 and f.max() <= 4.0
    assert np.all(f[outside_head] == 0.0)
    assert np.all(f[inside_brain & off_disks] == 1.0)
    assert np.all(f[in_disk] == 4.0)
    # the overlap of both disks takes the maximum (4), not the sum
    both = (d1 + margin < 1.4) & (d2 + margin < 1.4)
    assert both.sum() >= 4 and np.all(f[both] == 4.0)
    # the hot part equals the per-disk coverage maximum exactly where the brain is full
    hot = np.maximum(ph.disk_coverage(g, 1.0, 0.5, 1.4), ph.disk_coverage(g, 2.2, 0.5, 1.4))
    np.testing.assert_allclose(f[inside_brain], 1.0 + 3.0 * hot[inside_brain], atol=1e-15)


def test_activity_plateaus_and_overlap_maximum():
    _pin_activity(ph.activity_phantom)


@pytest.mark.parametrize("mistake", ["sum_overlaps", "hot_absolute", "no_brain_mask"])
def test_planted_activity_mistakes_fail(mistake):
    from oracle.head import coverage_fractions

    def sum_overlaps(g, c, dr, disks, bg, hot):
        fb, _ = coverage_fractions(g, c, dr)
        return bg * fb + (hot - bg) * sum(ph.disk_coverage(g, *d) for d in disks)

    def hot_absolute(g, c, dr, disks, bg, hot):
        # the disks' activity added on top of the background: 1 + 4 inside a disk
        fb, _ = coverage_fractions(g, c, dr)
        m = np.maximum.reduce([ph.disk_coverage(g, *d) for d in disks])
        return bg * fb + hot * m

    def no_brain_mask(g, c, dr, disks, bg, hot):
        m = np.maximum.reduce([ph.disk_coverage(g, *d) for d in disks])
        return bg + (hot - bg) * m

    wrong = {"sum_overlaps": sum_overlaps, "hot_absolute": hot_absolute, "no_brain_mask": no_brain_mask}[mistake]
    with pytest.raises(AssertionError):
        _pin_activity(wrong)
