"""Pins of the oracle's direction-graph reading (Sec. 6, Eq. (1)): the
hemisphere cells are bounded and about as few as the bound allows, and the
graph form reduces to the plain continuous form wherever merging loses
nothing (cells too small to merge, members that share their directions)."""
import datetime as dt

import numpy as np

import oracle
from workloads import Span, make_c1, subset_points
from workloads.scenes import Day, _nyc_tz


def _dirs(n, seed):
    """Uniform directions on the upper hemisphere."""
    v = np.random.default_rng(seed).normal(size=(n, 3))
    v[:, 2] = np.abs(v[:, 2])
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_cells_are_bounded():
    """Any two directions in one cell lie within the cell's diagonal,
    sqrt(2) * bound, of each other (brute force over every pair of a
    sample that shares a cell)."""
    for bound in (5.0, 1.0):
        d = _dirs(40_000 if bound == 5.0 else 200_000, 3)
        key = oracle.hemisphere_cell(d, bound)
        order = np.argsort(key, kind="stable")
        ks, ds = key[order], d[order]
        starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
        worst = 0.0
        for a, b in zip(starts, np.r_[starts[1:], len(ks)]):
            if b - a < 2:
                continue
            c = np.clip(ds[a:b] @ ds[a:b].T, -1.0, 1.0)
            worst = max(worst, float(np.degrees(np.arccos(c.min()))))
        assert worst <= np.sqrt(2.0) * bound * 1.001, (bound, worst)
        assert worst >= 0.9 * bound                    # cells are not needlessly small


def test_cell_count_matches_the_bound():
    """The hemisphere (2 pi sr) cut into cells of about bound x bound: the
    number of cells a dense sample meets is within a few percent of
    2 pi / bound^2 (cells of full width bound at the equator of each ring)."""
    bound = 5.0
    n_cells = len(np.unique(oracle.hemisphere_cell(_dirs(400_000, 4), bound)))
    ideal = 2.0 * np.pi / np.radians(bound) ** 2
    assert 0.98 < n_cells / ideal < 1.1, n_cells / ideal


def test_cells_split_by_azimuth_and_elevation():
    """Directions one bound apart in azimuth at the horizon, or in
    elevation, fall in different cells; a tiny step does not move across
    the middle of a cell."""
    b = 2.0
    def d(el, az):
        el, az = np.radians(el), np.radians(az)
        return np.array([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az), np.sin(el)])
    c = oracle.hemisphere_cell
    assert c(d(1.0, 11.0), b) != c(d(1.0, 13.0), b)
    assert c(d(1.0, 11.0), b) != c(d(3.0, 11.0), b)
    assert c(d(1.0, 11.0), b) == c(d(1.0 + 1e-6, 11.0 + 1e-6), b)


def test_cell_keys_of_adjacent_rings_differ_at_the_smallest_bound():
    """At 1e-6 degrees a ring holds about 3.6e8 sectors: sector 4,000,005 of
    one ring and sector 5 of the next must still have different keys (a
    key of ring * 4,000,000 + sector would make them equal)."""
    bd = 1e-6
    b = np.radians(bd)
    r = 1000
    n_sec = int(np.ceil(2 * np.pi * np.cos(r * b) / b))
    def d(ring, sec, n):
        el = (ring + 0.5) * b
        az = (sec + 0.5) / n * 2 * np.pi - np.pi
        return np.array([np.cos(el) * np.sin(az), np.cos(el) * np.cos(az), np.sin(el)])
    n2 = int(np.ceil(2 * np.pi * np.cos((r + 1) * b) / b))
    k1 = oracle.hemisphere_cell(d(r, 4_000_005, n_sec), bd)
    k2 = oracle.hemisphere_cell(d(r + 1, 5, n2), bd)
    assert k1 // (1 << 32) == r and k2 // (1 << 32) == r + 1
    assert k1 != k2


def _small():
    w = make_c1()
    return w, w.points.take(subset_points(w.points, 200, 7))


def _span(dates, bins):
    return Span(40.7, -74.0, [Day(x.year, x.month, x.day, _nyc_tz(x)) for x in dates], 5.0, bins)


def test_tiny_cells_give_the_continuous_form():
    w, pts = _small()
    path = oracle.sun_path(_span([dt.date(2019, 3, 20), dt.date(2019, 6, 21)], [0, 1]), 30.0)
    g, groups = oracle.graph_continuous(w.scene, pts, path, 1e-6)
    assert len(groups) == len(path.seg_t)
    np.testing.assert_allclose(g, oracle.continuous(w.scene, pts, path)["minutes"], rtol=1e-12, atol=1e-9)


def test_members_count_with_their_own_duration():
    """Two segments with the same directions but durations of 30 and 45
    minutes form one edge; each keeps its own duration, so the edge's
    minutes equal the plain form over both (the occluded share of the arc
    is the same, the minutes scale with each duration)."""
    w, pts = _small()
    p = oracle.sun_path(_span([dt.date(2019, 6, 21)], [0]), 30.0)
    j = len(p.seg_t) // 2
    path = oracle.OraclePath(p.dirs[:0], p.w[:0], p.t[:0], p.sample_day[:0], p.sample_bin[:0],
                             np.array([[600.0, 630.0], [700.0, 745.0]]), np.stack([p.seg_dir[j], p.seg_dir[j]]),
                             np.array([0, 1], np.int32), np.array([0, 0], np.int32), 1, p.spans)
    g, groups = oracle.graph_continuous(w.scene, pts, path, 0.5)
    assert [len(x) for x in groups] == [2]
    plain = oracle.continuous(w.scene, pts, path)["minutes"]
    assert plain.max() > 0
    np.testing.assert_allclose(g, plain, rtol=1e-9, atol=1e-9)
    one = oracle.continuous(w.scene, pts, oracle.OraclePath(
        path.dirs, path.w, path.t, path.sample_day, path.sample_bin, path.seg_t[:1], path.seg_dir[:1],
        path.seg_day[:1], path.day_bin[:1], 1, path.spans))["minutes"]
    np.testing.assert_allclose(g, one * 75.0 / 30.0, rtol=1e-9, atol=1e-9)


def test_repeated_days_merge_without_loss():
    w, pts = _small()
    path = oracle.sun_path(_span([dt.date(2019, 6, 21)] * 3, [0, 0, 0]), 30.0)
    g, groups = oracle.graph_continuous(w.scene, pts, path, 0.5)
    assert 3 * len(groups) == len(path.seg_t)
    np.testing.assert_allclose(g, oracle.continuous(w.scene, pts, path)["minutes"], rtol=1e-9, atol=1e-9)


def test_coarse_cells_merge_days_with_a_bounded_region_error():
    """Ten days around the June solstice at the paper's 5-degree cells:
    many fewer edges, per-point minutes no longer those of each day, but
    the region total stays within a few percent (each edge's
    representative arc lies within the cells of its members)."""
    w, pts = _small()
    dates = [dt.date(2019, 6, 16) + dt.timedelta(days=i) for i in range(10)]
    path = oracle.sun_path(_span(dates, [0] * 10), 30.0)
    g, groups = oracle.graph_continuous(w.scene, pts, path, 5.0)
    plain = oracle.continuous(w.scene, pts, path)["minutes"]
    assert len(groups) <= len(path.seg_t) / 4
    assert abs(g.sum() - plain.sum()) / plain.sum() < 0.05
    assert np.abs(g - plain).max() > 1.0        # but points do move


def test_edge_of_mirrored_members_is_the_arc_between_them():
    """Two members whose knots are a base arc's knots turned by +-eps about
    an axis perpendicular to each: their mean directions are the base
    knots, so the edge is the base arc, and the graph's minutes are the
    continuous form's on the base arc weighted by the members' durations
    (30 and 45 minutes, over the first member's 30)."""
    w, pts = _small()
    p = oracle.sun_path(_span([dt.date(2019, 6, 21)], [0]), 30.0)
    j = len(p.seg_t) // 2
    a, b = p.seg_dir[j]
    eps = 2e-4

    def turn(x, s):
        k = np.cross(x, [0.0, 0.0, 1.0])
        k /= np.linalg.norm(k)
        return np.cos(eps) * x + s * np.sin(eps) * np.cross(k, x)
    seg_dir = np.stack([[turn(a, 1), turn(b, 1)], [turn(a, -1), turn(b, -1)]])
    seg_t = np.array([[600.0, 630.0], [700.0, 745.0]])
    path = oracle.OraclePath(p.dirs[:0], p.w[:0], p.t[:0], p.sample_day[:0], p.sample_bin[:0], seg_t, seg_dir,
                             np.array([0, 1], np.int32), np.array([0, 0], np.int32), 1, p.spans)
    arc, times = oracle.edge_arc(path, [0, 1])
    np.testing.assert_allclose(arc, [a, b], atol=1e-12)
    g, groups = oracle.graph_continuous(w.scene, pts, path, 1.0)
    assert [len(x) for x in groups] == [2]
    base = oracle.OraclePath(path.dirs, path.w, path.t, path.sample_day, path.sample_bin, seg_t[:1],
                             np.array([[a, b]]), path.seg_day[:1], path.day_bin[:1], 1, path.spans)
    one = oracle.continuous(w.scene, pts, base)["minutes"]
    assert one.max() > 0
    np.testing.assert_allclose(g, one * 75.0 / 30.0, rtol=1e-9, atol=1e-9)
