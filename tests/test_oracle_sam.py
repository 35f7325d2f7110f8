"""Pins of the oracle's raster shadow accrual map (Sec. 4): the tan law of
the shadow's motion on the plane, the grid's cover of the scene, agreement
with the exact shadow predicate away from shadow edges at fine texels,
convergence as texels shrink, and the cases whose answer is known."""
import numpy as np

import oracle
from workloads import Scene, Span, make_c1, subset_points
from workloads.scenes import Day, _pts


def _box_scene(H=40.0):
    xy = np.array([[0, 0], [20, 0], [20, 30], [0, 30]], np.float32)
    return Scene(np.array([0, 4], np.int32), xy, np.array([H], np.float32))


def _day(window=(7 * 60, 17 * 60)):
    # June 21 at the small scene's site, whole minutes, every 30 min
    return Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, window)], 30.0)


def test_projection_follows_the_tan_law():
    """Sec. 4: with the plane normal to the start direction a, the shadow of
    a point at the fraction f of a segment of angle theta lies at
    p1 + (pn - p1) tan(f theta) / tan(theta)."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        a = rng.normal(size=3); a[2] = abs(a[2]) + 0.2; a /= np.linalg.norm(a)
        b = a + rng.normal(scale=0.15, size=3); b[2] = abs(b[2]); b /= np.linalg.norm(b)
        theta = np.arccos(np.clip(a @ b, -1, 1))
        s = rng.uniform(-100, 100, size=(5, 3))
        c = float((s @ a).min()) - 50.0
        p1, pn = oracle.sam_project(s, a, c, a), oracle.sam_project(s, a, c, b)
        for f in (0.1, 0.5, 0.9):
            p = oracle.sam_project(s, a, c, oracle.slerp(a, b, f))
            np.testing.assert_allclose(p, p1 + (pn - p1) * np.tan(f * theta) / np.tan(theta), atol=1e-9)
            np.testing.assert_allclose((p - s) @ a, (c - s @ a) * np.ones(5), atol=1e-9)  # on the plane


def test_grid_covers_the_scene_for_every_instant():
    """Every prism corner's shadow, at every instant of every segment, falls
    at least one texel inside the grid (the margin)."""
    w = make_c1()
    path = oracle.sun_path(w.span, 30.0)
    box = (w.scene.xy[:, 0].min(), w.scene.xy[:, 1].min(), 0.0,
           w.scene.xy[:, 0].max(), w.scene.xy[:, 1].max(), w.scene.height.max())
    V = np.concatenate([np.c_[w.scene.xy, np.zeros(len(w.scene.xy))],
                        np.c_[w.scene.xy, np.repeat(w.scene.height, np.diff(w.scene.vert_off))]]).astype(np.float64)
    for j, ks in enumerate(oracle.sam_segments(path)):
        a, b = path.seg_dir[j]
        G = oracle.sam_grid(box, a, b, 2.0)
        for f in np.linspace(0, 1, 7):
            P = oracle.sam_project(V, G["a"], G["c"], oracle.slerp(a, b, f))
            fu, fv = (P @ G["u"] - G["u0"]) / G["h"], (P @ G["v"] - G["v0"]) / G["h"]
            assert fu.min() >= 1 and fv.min() >= 1 and fu.max() <= G["nu"] - 1 and fv.max() <= G["nv"] - 1
            assert (P @ G["a"] - G["c"]).max() < 1e-6 and (V @ G["a"] - G["c"]).min() >= 1.0 - 1e-9


def test_fine_texels_agree_with_the_exact_predicate():
    """A lone 20 x 30 x 40 m box, ground points on a 4 m lattice around it,
    10 cm texels: wherever the exact predicate (the instant's great-circle
    direction) is the same at the point and at 16 points around it, out to
    the reach of a texel on the ground, the map decides the same."""
    sc = _box_scene()
    g = np.arange(-90.0, 111.0, 4.0) + 0.37
    X, Y = np.meshgrid(g, g)
    pts = _pts(X.ravel(), Y.ravel())
    path = oracle.sun_path(_day(), 60.0)
    h = 0.1
    r = oracle.sam(sc, pts, path, h)
    checked = agree = 0
    for j, ks in enumerate(oracle.sam_segments(path)):
        a, b = path.seg_dir[j]
        ta, tb = path.seg_t[j]
        for k in ks:
            d = oracle.slerp(a, b, (path.t[k] - ta) / (tb - ta))
            reach = 2.0 * h / max(d[2], 1e-3) + h
            ring = [(reach * np.cos(t), reach * np.sin(t)) for t in np.linspace(0, 2 * np.pi, 8, endpoint=False)]
            ring += [(x / 2, y / 2) for x, y in ring]
            for i in range(pts.n):
                p = (pts.x[i], pts.y[i], 0.0)
                e = oracle.shadow(sc, p, d)
                if any(oracle.shadow(sc, (p[0] + dx, p[1] + dy, 0.0), d) != e for dx, dy in ring):
                    continue
                checked += 1
                agree += int(r["shadowed"][i, k] == e)
    assert checked > 0.9 * pts.n * len(path.t)
    assert agree == checked


def test_roof_covered_and_empty():
    sc = _box_scene()
    pts = _pts([10.0, 5.0], [15.0, 25.0])            # both under the roof
    path = oracle.sun_path(_day(), 60.0)
    r = oracle.sam(sc, pts, path, 0.5)
    assert r["shadowed"].all()
    empty = Scene(np.array([0], np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))
    r = oracle.sam(empty, pts, path, 0.5, box=(0, 0, 0, 1, 1, 1))
    assert not r["shadowed"].any() and r["counts"].sum() == 0


def test_taller_never_shades_less():
    sc, tall = _box_scene(40.0), _box_scene(60.0)
    g = np.arange(-60.0, 81.0, 3.0) + 0.41
    X, Y = np.meshgrid(g, g)
    pts = _pts(X.ravel(), Y.ravel())
    path = oracle.sun_path(_day(), 60.0)
    box = (0, 0, 0, 20, 30, 60)
    lo = oracle.sam(sc, pts, path, 0.5, box=box)["shadowed"]
    hi = oracle.sam(tall, pts, path, 0.5, box=box)["shadowed"]
    assert np.all(hi >= lo) and hi.sum() > lo.sum()


def test_error_falls_as_texels_shrink():
    """On the small scene, the share of (point, instant) decisions that
    differ from the exact predicate along the same directions falls as the
    texel shrinks (4 m, 1 m, 0.25 m), and the counts' mean error with it."""
    w = make_c1()
    sub = w.points.take(subset_points(w.points, 256, 17))
    path = oracle.sun_path(w.span, 30.0)
    exact = np.zeros((sub.n, len(path.t)), np.uint8)
    for j, ks in enumerate(oracle.sam_segments(path)):
        a, b = path.seg_dir[j]
        ta, tb = path.seg_t[j]
        for k in ks:
            d = oracle.slerp(a, b, (path.t[k] - ta) / (tb - ta))
            exact[:, k] = [oracle.shadow(w.scene, (sub.x[i], sub.y[i], sub.z[i]), d) for i in range(sub.n)]
    miss = [float((oracle.sam(w.scene, sub, path, h)["shadowed"] != exact).mean()) for h in (4.0, 1.0, 0.25)]
    assert miss[0] > miss[1] > miss[2] and miss[2] < 0.01, miss


def test_exit_depths_c_equals_numpy():
    """The C brute force and the numpy statement of the map depth agree on
    random rays through the small scene, grown, shrunk and as is."""
    w = make_c1()
    rng = np.random.default_rng(5)
    X = np.c_[rng.uniform(-50, 560, 3000), rng.uniform(-50, 560, 3000), rng.uniform(-200, 0, 3000)]
    for d in ([0.3, -0.2, 0.9], [-0.8, 0.1, 0.3]):
        d = np.array(d) / np.linalg.norm(d)
        for g in (0.0, 0.005, -0.005):
            a, b = oracle.exit_depths(w.scene, X, d, g), oracle.exit_depths_np(w.scene, X, d, g)
            assert np.isfinite(a).sum() > 100
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-9)
