"""Pins for the oracle's continuous duration along the sun's actual path
(``oracle.continuous_true``; the definition of gross shadow, Sec. 3.1, with
the actual sun direction of Sec. 3.2 / Table 1): an independent 1-D root
find of a lone box's single transition and of a wall's back-face switch,
convergence of the accrual path model (great circles between knots) as the
knots close in (error falling as L^2), convergence of the sampled form as
the step shrinks (within transitions x step / 2), the equinox path being
nearly a great circle, a finer scan grid changing nothing, and invariants
(bounded by the span, empty scene, roof-covered points, monotone in height,
building order, a box split into two abutting boxes)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from workloads import Points, Scene, Span
from workloads.scenes import Day

LAT, LON = 40.7, -74.0


def box_scene(boxes):
    """boxes: list of (x0, y0, x1, y1, h)"""
    xy = np.array([[(b[0], b[1]), (b[2], b[1]), (b[2], b[3]), (b[0], b[3])] for b in boxes],
                  np.float32).reshape(-1, 2)
    return Scene(np.arange(0, 4 * len(boxes) + 1, 4, dtype=np.int32), xy,
                 np.array([b[4] for b in boxes], np.float32))


def pts(xyz, nrm=None, owner=None):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = len(xyz)
    nrm = np.zeros((n, 2), np.float32) if nrm is None else np.asarray(nrm, np.float32).reshape(-1, 2)
    own = np.full(n, -1, np.int32) if owner is None else np.asarray(owner, np.int32)
    return Points(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), nrm[:, 0].copy(), nrm[:, 1].copy(), own)


def window_span(month, day, tz, t0, t1, step=5.0):
    return Span(LAT, LON, [Day(2019, month, day, tz, (t0, t1))], step_min=step)


def test_lone_box_transition_matches_root_find():
    """A box 20 m deep, 2 km long north-south and 30 m tall; a ground point
    25 m east of its east face.  The point is lit until the afternoon sun,
    low in the west, is seen below the roof edge: the ray toward the sun
    (azimuth A, elevation e) meets the east face x = 0 at horizontal distance
    25 / (-sin A) and height 25 tan(e) / (-sin A), so the shadow starts at
    the root of tan e(t) = 30 (-sin A(t)) / 25 and lasts to the window's
    end.  The root comes from scipy's brentq on the solar position alone."""
    sc = box_scene([(-20.0, -1000.0, 0.0, 1000.0, 30.0)])
    P = pts([[25.0, 0.0, 0.0]])
    t0, t1 = 480.0, 1200.0                       # 08:00 .. 20:00 EDT, Jun 21

    def f(t):
        s = oracle.solar(2019, 6, 21, t, -4.0, LAT, LON)
        a = math.radians(s[4])
        return math.tan(math.radians(s[3])) - 30.0 * (-math.sin(a)) / 25.0

    grid = np.arange(780.0, t1, 1.0)             # after 13:00 the sun is in the west
    vals = np.array([f(t) for t in grid])
    k = int(np.flatnonzero(np.sign(vals[:-1]) != np.sign(vals[1:]))[0])
    t_star = brentq(f, grid[k], grid[k + 1], xtol=1e-11)
    D = oracle.continuous_true(sc, P, window_span(6, 21, -4.0, t0, t1))["minutes"][0, 0]
    assert D == pytest.approx(t1 - t_star, abs=1e-6)
    assert 60.0 < t1 - t_star < 400.0


def test_back_facing_wall_switch_matches_root_find():
    """A wall point facing east with nothing around it is in shadow exactly
    while its wall faces away from the sun (d_x <= 0): from the instant the
    sun crosses the meridian to the window's end."""
    sc = box_scene([(-10.0, -10.0, 0.0, 10.0, 15.0)])
    P = pts([[0.0, 0.0, 5.0]], nrm=[[1.0, 0.0]], owner=[0])
    t0, t1 = 480.0, 1080.0
    t_noon = brentq(lambda t: oracle.solar(2019, 3, 20, t, -4.0, LAT, LON)[0], 600.0, 900.0, xtol=1e-11)
    D = oracle.continuous_true(sc, P, window_span(3, 20, -4.0, t0, t1))["minutes"][0, 0]
    assert D == pytest.approx(t1 - t_noon, abs=1e-6)


def test_accrual_path_model_converges_as_L_squared(c1):
    """The great-circle path between knots (the accrual form's model,
    ``oracle.continuous``) approaches the actual path as the knots close in;
    its deviation, and so the duration error, falls as L^2 (Sec. 3.2 and
    Table 1: the linear motion is accurate over short intervals)."""
    sub = c1.points.take(np.arange(3, c1.points.n, 97))
    D = oracle.continuous_true(c1.scene, sub, c1.span)["minutes"]
    err = {}
    for L in (60.0, 30.0, 15.0, 1.0):
        m = oracle.continuous(c1.scene, sub, oracle.sun_path(c1.span, L))["minutes"]
        err[L] = np.abs(m - D).mean()
    assert 3.0 < err[60.0] / err[30.0] < 5.5
    assert 3.0 < err[30.0] / err[15.0] < 5.5
    assert err[1.0] < 1e-3
    assert err[30.0] > 0.01                     # the knots matter at 30 min: not a trivial pass


def test_equinox_path_is_nearly_a_great_circle(c1):
    """On the equinox the sun's daily circle is (nearly) a great circle, so
    even hour-long knots barely move the duration; at the solstice the same
    knots cost far more."""
    sub = c1.points.take(np.arange(11, c1.points.n, 211))
    res = {}
    for md in ((3, 20), (6, 21)):
        span = window_span(*md, -4.0, 480.0, 1080.0)
        D = oracle.continuous_true(c1.scene, sub, span)["minutes"]
        m = oracle.continuous(c1.scene, sub, oracle.sun_path(span, 60.0))["minutes"]
        res[md] = np.abs(m - D).mean()
    assert res[(3, 20)] < 0.02
    assert res[(6, 21)] > 10 * res[(3, 20)]


def test_sampled_form_converges_within_transition_bound(c1):
    """The sampled form with instants every 15 s differs from the continuous
    duration by at most half a step per transition: each instant stands for
    the part of the window nearer to it than to any other, and only a cell
    holding a switch can be credited wrongly, by at most half its width."""
    sub = c1.points.take(np.arange(5, c1.points.n, 331))
    t0, t1, dt = 480.0, 1080.0, 0.25
    t = np.arange(t0, t1 + 1e-9, dt)
    w = np.full(len(t), dt)
    w[0] = w[-1] = dt / 2
    dirs = np.array([oracle.solar(2019, 6, 21, tk, -4.0, LAT, LON)[:3] for tk in t])
    z = np.zeros(len(t), np.int32)
    path = oracle.OraclePath(dirs, w, t, z, z, np.zeros((0, 2)), np.zeros((0, 2, 3)), np.zeros(0, np.int32),
                             np.zeros(1, np.int32), 1, np.array([[t0, t1]]))
    S = oracle.sampled(c1.scene, sub, path, bits=True)
    bits = np.unpackbits(S["bits"].view(np.uint8), axis=1, bitorder="little")[:, :len(t)]
    trans = np.abs(np.diff(bits.astype(int), axis=1)).sum(1)
    D = oracle.continuous_true(c1.scene, sub, window_span(6, 21, -4.0, t0, t1))["minutes"][0]
    err = np.abs(S["minutes"][0] - D)
    assert np.all(err <= trans * dt / 2 + 1e-6), (err - trans * dt / 2).max()
    assert trans.sum() > 0 and (err > 1e-3).any()


def test_finer_scan_grid_changes_nothing(c1):
    """A 1-second scan grid gives the 5-second grid's durations: the default
    grid (with its finer rescans near each prism) misses no run."""
    sub = c1.points.take(np.arange(0, c1.points.n, 173))
    a = oracle.continuous_true(c1.scene, sub, c1.span)["minutes"]
    b = oracle.continuous_true(c1.scene, sub, c1.span, grid_min=1.0 / 60.0)["minutes"]
    assert np.abs(a - b).max() < 1e-6


def test_true_path_invariants(c1):
    """Bounded by the span; zero for an empty scene; the whole span under a
    roof; never less after a building grows; independent of the order of the
    buildings; unchanged when a box is cut into two abutting boxes."""
    sc = c1.scene
    span = c1.span
    T = 1080.0 - 480.0
    sub = c1.points.take(np.arange(2, c1.points.n, 151))
    D = oracle.continuous_true(sc, sub, span)["minutes"][0]
    assert np.all(D >= 0) and np.all(D <= T + 1e-9)
    empty = Scene(np.zeros(1, np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))
    assert np.all(oracle.continuous_true(empty, sub, span)["minutes"] == 0)
    # roof-covered: centres of the first few footprints
    cen = sc.centroids()[:5]
    roof = pts(np.c_[cen, np.zeros(5)])
    assert np.allclose(oracle.continuous_true(sc, roof, span)["minutes"], T, atol=1e-9)
    # monotone in height
    taller = Scene(sc.vert_off, sc.xy, sc.height.copy())
    taller.height[::5] += np.float32(15.0)
    D2 = oracle.continuous_true(taller, sub, span)["minutes"][0]
    assert np.all(D2 >= D - 1e-7) and (D2 > D + 1e-3).any()
    # building order
    perm = np.random.default_rng(0).permutation(sc.n_b)
    D3 = oracle.continuous_true(sc.subset(perm), sub, span)["minutes"][0]
    assert np.abs(D3 - D).max() < 1e-7
    # one box cut into two abutting boxes (the union of two closed prisms is
    # the original closed prism)
    f = sc.footprint(0).astype(np.float64)
    x0, y0, x1, y1 = f[:, 0].min(), f[:, 1].min(), f[:, 0].max(), f[:, 1].max()
    xm = np.float32(0.5 * (x0 + x1))
    h = float(sc.height[0])
    parts = [(x0, y0, xm, y1, h), (xm, y0, x1, y1, h)]
    rest = [tuple(list(sc.footprint(b).min(0)) + list(sc.footprint(b).max(0)) + [float(sc.height[b])])
            for b in range(1, sc.n_b)]
    split = box_scene(parts + rest)
    D4 = oracle.continuous_true(split, sub, span)["minutes"][0]
    assert np.abs(D4 - D).max() < 1e-6


def test_catches_runs_shorter_than_the_grid():
    """A thin pole 200 m away shadows a ground point for a few seconds; the
    5-second scan must find that run and agree with a 0.05-second scan."""
    span = window_span(6, 21, -4.0, 480.0, 1080.0)
    s = oracle.solar(2019, 6, 21, 607.0 + 2.5 / 60.0, -4.0, LAT, LON)   # between two scan instants
    u = s[:2] / np.linalg.norm(s[:2])
    c = u * 200.0
    h = 200.0 * math.tan(math.radians(s[3])) + 20.0
    sc = box_scene([(c[0] - 0.01, c[1] - 0.01, c[0] + 0.01, c[1] + 0.01, h)])
    P = pts([[0.0, 0.0, 0.0]])
    coarse = oracle.continuous_true(sc, P, span)["minutes"][0, 0]
    fine = oracle.continuous_true(sc, P, span, grid_min=1.0 / 1200.0)["minutes"][0, 0]
    assert 0.0 < fine < 5.0 / 60.0
    assert coarse == pytest.approx(fine, abs=1e-6)


@pytest.mark.parametrize("level", [60.0, 5.0])
def test_box_between_chord_plane_and_actual_path(level):
    """The sun's actual path bulges off the great circle through the ends of
    a stretch.  A 4 mm pole 1.5 km away whose roof lies between that great
    circle's plane and the actual ray at the stretch's middle is met by the
    actual path although it lies wholly on one side of the plane: a prism
    may be skipped only with the bulge taken into account.  The box's shadow
    time is checked against the predicate sampled every 0.05 s around it."""
    t0, t1 = 480.0, 1080.0
    span = window_span(6, 21, -4.0, t0, t1)
    ta = t0 + 3 * level if level == 60.0 else t0 + 60.0 + 4 * level   # a stretch the oracle walks
    tb, tm = ta + level, ta + level / 2
    da, db, dm = (oracle.solar(2019, 6, 21, t, -4.0, LAT, LON)[:3] for t in (ta, tb, tm))
    N = np.cross(da, db)
    N /= np.linalg.norm(N)
    r = 1500.0
    q = dm * r / np.linalg.norm(dm[:2])          # the actual ray at the middle, 1.5 km out
    # height of the chord plane above the box's footprint centre: N . (x, y, z) = 0
    zc = -(N[0] * q[0] + N[1] * q[1]) / N[2]
    zt = q[2]
    assert abs(zc - zt) > 0.02                  # the bulge is resolvable here
    w = 0.002
    if zt < zc:
        # roof between the ray (below) and the plane (above): the whole box is below the plane
        H = 0.5 * (zt + zc)
        plane_side = lambda x, y, z: N @ np.array([x, y, z])
        corners = [plane_side(q[0] + sx * w, q[1] + sy * w, z) for sx in (-1, 1) for sy in (-1, 1) for z in (0.0, H)]
        assert max(corners) < 0 or min(corners) > 0
    else:
        pytest.skip("the path bulges upward here")
    sc = box_scene([(q[0] - w, q[1] - w, q[0] + w, q[1] + w, H)])
    P = pts([[0.0, 0.0, 0.0]])
    D = oracle.continuous_true(sc, P, span)["minutes"][0, 0]
    tt = np.arange(tm - 10.0, tm + 10.0, 1.0 / 1200.0)
    hit = np.array([oracle.shadow(sc, (0.0, 0.0, 0.0), oracle.solar(2019, 6, 21, t, -4.0, LAT, LON)[:3]) for t in tt])
    assert hit.any() and not hit[0] and not hit[-1]
    assert D == pytest.approx(hit.sum() / 1200.0, abs=2.0 / 1200.0)


def test_thin_pole_run_matches_azimuth_root_find():
    """A 2 cm square pole 200 m from a ground point, tall enough to block
    the sun at any elevation it has then, shadows the point for about a
    second: exactly while the sun's azimuth lies between the azimuths of the
    pole's two silhouette corners as seen from the point.  Both ends come
    from brentq on the solar azimuth alone; the 5-second scan must find the
    run and match them."""
    t_mid = 607.0 + 2.5 / 60.0                      # between two scan instants
    s = oracle.solar(2019, 6, 21, t_mid, -4.0, LAT, LON)
    az = math.radians(s[4])
    c = 200.0 * np.array([math.sin(az), math.cos(az)])
    h = 200.0 * math.tan(math.radians(s[3])) + 40.0
    half = 0.01
    sc = box_scene([(c[0] - half, c[1] - half, c[0] + half, c[1] + half, h)])
    corners = np.array(sc.footprint(0), np.float64)
    az_c = np.arctan2(corners[:, 0], corners[:, 1])          # azimuths of the corners from the point
    lo, hi = az_c.min(), az_c.max()

    def sun_az(t):
        return math.radians(oracle.solar(2019, 6, 21, t, -4.0, LAT, LON)[4])
    t_in = brentq(lambda t: sun_az(t) - lo, t_mid - 1.0, t_mid + 1.0, xtol=1e-12)
    t_out = brentq(lambda t: sun_az(t) - hi, t_mid - 1.0, t_mid + 1.0, xtol=1e-12)
    expect = abs(t_out - t_in)
    span = window_span(6, 21, -4.0, 480.0, 1080.0)
    D = oracle.continuous_true(sc, pts([[0.0, 0.0, 0.0]]), span)["minutes"][0, 0]
    assert 0.0 < expect < 5.0 / 60.0
    assert D == pytest.approx(expect, abs=1e-6)
