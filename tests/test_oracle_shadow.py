"""Pins for the oracle's shadow predicate and its sampled / continuous
accumulation: closed forms, hand-computed cases, an independent predicate
(Moller-Trumbore on the triangulated prisms, and a shadow-polygon test on
the ground), invariants, and convergence between the two forms."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads import Points, Scene, Span
from workloads.scenes import Day

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def box_scene(boxes):
    """boxes: list of (x0, y0, x1, y1, h)"""
    xy = np.array([[(b[0], b[1]), (b[2], b[1]), (b[2], b[3]), (b[0], b[3])] for b in boxes],
                  np.float32).reshape(-1, 2)
    return Scene(np.arange(0, 4 * len(boxes) + 1, 4, dtype=np.int32), xy,
                 np.array([b[4] for b in boxes], np.float32))


def empty_scene():
    return Scene(np.zeros(1, np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))


def sundir(az_deg, el_deg):
    a, e = math.radians(az_deg), math.radians(el_deg)
    return np.array([math.sin(a) * math.cos(e), math.cos(a) * math.cos(e), math.sin(e)])


def pts(xyz, nrm=None, owner=None):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = len(xyz)
    nrm = np.zeros((n, 2), np.float32) if nrm is None else np.asarray(nrm, np.float32).reshape(-1, 2)
    own = np.full(n, -1, np.int32) if owner is None else np.asarray(owner, np.int32)
    return Points(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), nrm[:, 0].copy(), nrm[:, 1].copy(), own)


# --------------------------------------------------------------------------
# predicate: closed forms and hand-computed cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("az", [0.0, 90.0, 180.0, 270.0])
@pytest.mark.parametrize("el", [10.0, 30.0, 60.0])
def test_lone_box_shadow_length(az, el):
    """A lone box of height h casts a shadow of length h / tan(e) beyond its
    far face, pointing away from the sun's azimuth."""
    a, h = 0.5, 30.0
    sc = box_scene([(-a, -a, a, a, h)])
    d = sundir(az, el)
    u = -d[:2] / np.linalg.norm(d[:2])            # shadow direction on the ground
    L = a + h / math.tan(math.radians(el))
    for r, expect in ((L - 1e-3, 1), (L + 1e-3, 0), (0.5 * L + 0.25, 1), (a + 0.01, 1)):
        p = (u[0] * r, u[1] * r, 0.0)
        assert oracle.shadow(sc, p, d) == expect, (r, L)
        assert oracle.shadow(sc, p, d, mt=True) == expect
    # and nothing on the sunward side
    p = (-u[0] * (a + 1.0), -u[1] * (a + 1.0), 0.0)
    assert oracle.shadow(sc, p, d) == 0


def test_noon_shadow_points_north():
    """At local apparent noon on Jun 21 at 40.7 N the sun is due south: a box
    shades the ground north of it and nothing to its south, east or west."""
    lat, lon, tz = 40.7, -74.0, -4.0
    eot = oracle.solar(2019, 6, 21, 720.0, tz, lat, lon)[6]
    s = oracle.solar(2019, 6, 21, 720.0 - 4 * lon - eot + 60 * tz, tz, lat, lon)
    d = s[:3]
    h = 40.0
    sc = box_scene([(-5, -5, 5, 5, h)])
    L = h / math.tan(math.radians(s[3]))
    assert oracle.shadow(sc, (0, 5 + 0.5 * L, 0), d) == 1
    assert oracle.shadow(sc, (0, 5 + L + 0.05, 0), d) == 0
    for p in ((0, -5.5, 0), (5.5, 0, 0), (-5.5, 0, 0), (5.5, 5 + 0.5 * L, 0)):
        assert oracle.shadow(sc, p, d) == 0


def test_empty_scene_gives_zero():
    sc = empty_scene()
    rng = np.random.default_rng(0)
    for _ in range(100):
        d = sundir(rng.uniform(0, 360), rng.uniform(1, 89))
        assert oracle.shadow(sc, rng.uniform(-50, 50, 3) * [1, 1, 0], d) == 0
    # a facade point with nothing around is shadowed exactly when its wall faces away
    d = sundir(90.0, 30.0)     # sun in the east
    assert oracle.shadow(sc, (0, 0, 1), d, nrm=(1, 0), owner=0) == 0
    assert oracle.shadow(sc, (0, 0, 1), d, nrm=(-1, 0), owner=0) == 1


def test_roof_covered_points_always_shadowed():
    sc = box_scene([(0, 0, 10, 10, 3.0)])
    rng = np.random.default_rng(1)
    for _ in range(200):
        d = sundir(rng.uniform(0, 360), rng.uniform(0.5, 89.5))
        p = (rng.uniform(0.01, 9.99), rng.uniform(0.01, 9.99), 0.0)
        assert oracle.shadow(sc, p, d) == 1


def test_hand_computed_two_boxes():
    """Box A [0,10]x[0,10] h=20, box B [20,30]x[0,10] h=5, sun due west at
    45 deg: a ray from (x, 5, 0) rises 1 m per metre travelled west."""
    sc = box_scene([(0, 0, 10, 10, 20.0), (20, 0, 30, 10, 5.0)])
    d = sundir(270.0, 45.0)
    cases = [((35, 5, 0), 1),    # reaches B's east face at height 5 = H (closed prism)
             ((36, 5, 0), 0),    # over B (6 > 5), then A at 26 > 20
             ((25, 5, 0), 1),    # under B's roof
             ((15, 5, 0), 1),    # A at 5 <= 20
             ((31, 5, 0), 1),    # B at 1
             ((5, 15, 0), 0),    # north of both, sun from the west
             ((45, 5, 0), 0)]    # B at 15 > 5, A at 35 > 20
    for p, e in cases:
        assert oracle.shadow(sc, p, d) == e, p
        assert oracle.shadow(sc, p, d, mt=True) == e, p
    # facade points on B (owner 1): west wall faces the sun, A hides it at 10 + 2 <= 20
    assert oracle.shadow(sc, (20, 5, 2), d, nrm=(-1, 0), owner=1) == 1
    assert oracle.shadow(sc, (20, 5, 19), d, nrm=(-1, 0), owner=1) == 0   # 19 + 10 > 20
    assert oracle.shadow(sc, (30, 5, 2), d, nrm=(1, 0), owner=1) == 1     # east wall faces away


def test_cyrus_beck_agrees_with_moller_trumbore(c1):
    from workloads import make_c2
    w = make_c2(n_ground=0, n_facade=0)
    sc = w.scene.subset(np.arange(400))
    rng = np.random.default_rng(7)
    lo, hi = sc.xy.min(0), sc.xy.max(0)
    bad = 0
    for _ in range(3000):
        p = (rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), 0.0)
        d = sundir(rng.uniform(0, 360), rng.uniform(0.5, 80))
        bad += oracle.shadow(sc, p, d) != oracle.shadow(sc, p, d, mt=True)
    assert bad == 0


def test_shadow_monotone_in_height():
    from workloads import make_c2
    w = make_c2(n_ground=0, n_facade=0)
    sc = w.scene.subset(np.arange(300))
    sc2 = Scene(sc.vert_off, sc.xy, (sc.height * 1.5).astype(np.float32))
    rng = np.random.default_rng(8)
    lo, hi = sc.xy.min(0), sc.xy.max(0)
    for _ in range(1500):
        p = (rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]), 0.0)
        d = sundir(rng.uniform(0, 360), rng.uniform(1, 80))
        assert oracle.shadow(sc, p, d) <= oracle.shadow(sc2, p, d)


# --------------------------------------------------------------------------
# sampled accumulation
# --------------------------------------------------------------------------
def _longest_run(bits):
    best = cur = 0
    for b in bits:
        cur = cur + 1 if b else 0
        best = max(best, cur)
    return best


def test_paper_fig2_semantics():
    """Gross shadow counts shadowed instants and continuous shadow is the
    longest run (Sec. 3.1, Sec. 5).  The bit patterns of the paper's example
    are produced by two towers and a three-instant sweep of the sun; the
    oracle's count must equal the example's gross minutes (1-minute
    instants)."""
    with open(os.path.join(GOLD, "paper_fig2_shadow_types.json")) as f:
        g = json.load(f)["points"]
    # sun sweeping from south-west to south-east at 30 deg elevation; two
    # 20 m towers; search the ground for each of the example's patterns
    sc = box_scene([(0, 0, 4, 4, 20.0), (14, 0, 18, 4, 20.0)])
    dirs = np.array([sundir(az, 30.0) for az in (150.0, 180.0, 210.0)])
    path = oracle.OraclePath(dirs, np.ones(3), np.arange(3.0), np.zeros(3, np.int32), np.zeros(3, np.int32),
                             np.zeros((0, 2)), np.zeros((0, 2, 3)), np.zeros(0, np.int32),
                             np.zeros(1, np.int32), 1, np.array([[0.0, 2.0]]))
    gx, gy = np.meshgrid(np.arange(-20, 40, 0.5) + 0.25, np.arange(4.5, 40, 0.5) + 0.25)
    grid = pts(np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], 1))
    r = oracle.sampled(sc, grid, path, bits=True)
    bitv = [[(int(r["bits"][i, 0]) >> k) & 1 for k in range(3)] for i in range(grid.n)]
    for name, e in g.items():
        idx = [i for i, b in enumerate(bitv) if b == e["bits"]]
        assert idx, f"pattern {e['bits']} not produced"
        i = idx[0]
        assert r["counts"][0, i] == e["gross_min"]
        assert r["minutes"][0, i] == e["gross_min"]
        assert _longest_run(bitv[i]) == e["continuous_min"]
        # the independent predicate agrees on the three instants
        for k in range(3):
            p = (grid.x[i], grid.y[i], 0.0)
            assert oracle.shadow(sc, p, dirs[k], mt=True) == e["bits"][k]


def test_c1_always_shadowed_points(c1):
    path = oracle.sun_path(c1.span)
    r = oracle.sampled(c1.scene, c1.points, path)
    K = len(path.w)
    full = r["counts"][0] == K
    assert full.mean() > 0.2
    np.testing.assert_allclose(r["minutes"][0][full], 600.0)
    assert np.all(r["minutes"][0] <= 600.0 + 1e-9)
    # every roof-covered lattice point is among them
    inside = np.zeros(c1.points.n, bool)
    for b in range(c1.scene.n_b):
        f = c1.scene.footprint(b)
        inside |= (c1.points.x > f[:, 0].min()) & (c1.points.x < f[:, 0].max()) & \
                  (c1.points.y > f[:, 1].min()) & (c1.points.y < f[:, 1].max())
    assert np.all(full[inside])


def test_c1_ambiguous_fraction_small(c1):
    """The silhouette band (1e-5 rad) holds at most 1e-4 of the point-step
    pairs of the small scene."""
    path = oracle.sun_path(c1.span)
    sub = c1.points.take(np.arange(0, c1.points.n, 4))
    r = oracle.sampled(c1.scene, sub, path, amb=True)
    assert r["amb"].mean() <= 1e-4


# --------------------------------------------------------------------------
# continuous accumulation
# --------------------------------------------------------------------------
def test_theorem1_tan_projection():
    """Theorem 1 (Sec. 4): with the light direction turning at a constant
    angular rate from d1 to dn, the shadow of a source point on the plane
    orthogonal to d1 lies at p1 + (pn - p1) tan(i theta / n) / tan(theta).
    Checks the oracle's great-circle interpolation against that formula."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        d1 = rng.normal(size=3); d1 /= np.linalg.norm(d1)
        dn = d1 + rng.normal(size=3) * 0.3; dn /= np.linalg.norm(dn)
        theta = math.acos(np.clip(d1 @ dn, -1, 1))
        s = rng.normal(size=3) * 10
        plane_pt = s - 50 * d1          # plane orthogonal to d1, beyond s

        def proj(d):                    # shadow of s along direction -d on the plane
            lam = ((s - plane_pt) @ d1) / (d @ d1)
            return s - lam * d
        p1, pn = proj(d1), proj(dn)
        n = 7
        for i in range(n + 1):
            d = oracle.slerp(d1, dn, i / n)
            np.testing.assert_allclose(proj(d), p1 + (pn - p1) * math.tan(i * theta / n) / math.tan(theta),
                                       atol=1e-9)


def _ground_shadow_np(scene, px, py, D):
    """Independent predicate for ground points: p is shadowed iff the
    horizontal segment from p toward the sun, of length H |d_xy| / d_z,
    meets the footprint (the prism's ground shadow is the footprint swept
    along the shadow direction).  Separating-axis test, vectorised over
    directions D [T, 3]."""
    out = np.zeros(len(D), bool)
    for b in range(scene.n_b):
        f = scene.footprint(b).astype(np.float64)
        H = float(scene.height[b])
        ex = (D[:, 0] / D[:, 2]) * H
        ey = (D[:, 1] / D[:, 2]) * H
        q0 = np.stack([np.full(len(D), px), np.full(len(D), py)], 1)
        q1 = q0 + np.stack([ex, ey], 1)
        sep = np.zeros(len(D), bool)
        e = np.roll(f, -1, 0) - f
        for k in range(len(f)):        # footprint edge normals
            n = np.array([e[k, 1], -e[k, 0]])
            pmax = (f @ n).max()
            sep |= np.minimum(q0 @ n, q1 @ n) > pmax
            pmin = (f @ n).min()
            sep |= np.maximum(q0 @ n, q1 @ n) < pmin
        n2 = np.stack([-ey, ex], 1)    # segment normal
        proj = f @ n2.T                # [m, T]
        s0 = np.sum(q0 * n2, 1)
        sep |= (proj.min(0) > s0) | (proj.max(0) < s0)
        out |= ~sep
    return out


def _np_slerp(a, b, f):
    th = math.acos(np.clip(a @ b, -1, 1))
    return (np.sin((1 - f) * th)[:, None] * a + np.sin(f * th)[:, None] * b) / math.sin(th)


def test_continuous_vs_independent_fine_grid(c1):
    """D_L on C1 points vs a 1-second integration of the shadow-polygon
    predicate along the same great-circle path."""
    path = oracle.sun_path(c1.span, seg_min=30.0)
    rng = np.random.default_rng(11)
    idx = rng.choice(c1.points.n, 24, replace=False)
    sub = c1.points.take(idx)
    r = oracle.continuous(c1.scene, sub, path)
    for i in range(sub.n):
        tot = 0.0
        for j in range(len(path.seg_t)):
            ta, tb = path.seg_t[j]
            G = int(round((tb - ta) * 60))
            f = (np.arange(G) + 0.5) / G
            D = _np_slerp(path.seg_dir[j, 0], path.seg_dir[j, 1], f)
            tot += _ground_shadow_np(c1.scene, float(sub.x[i]), float(sub.y[i]), D).sum() * (tb - ta) / G
        # midpoint rule on 1 s cells: each transition costs at most half a cell
        assert r["minutes"][0, i] == pytest.approx(tot, abs=0.1), i


def test_continuous_bounded_and_monotone(c1):
    path = oracle.sun_path(c1.span, seg_min=60.0)
    sub = c1.points.take(np.arange(0, c1.points.n, 97))
    r0 = oracle.continuous(c1.scene, sub, path)["minutes"][0]
    assert np.all(r0 >= 0) and np.all(r0 <= 600.0 + 1e-9)
    sc2 = Scene(c1.scene.vert_off, c1.scene.xy, (c1.scene.height + 7.0).astype(np.float32))
    r1 = oracle.continuous(sc2, sub, path)["minutes"][0]
    assert np.all(r1 >= r0 - 1e-7)
    assert np.any(r1 > r0 + 1.0)


def test_continuous_permutation_and_split_invariance():
    boxes = [(0, 0, 10, 10, 20.0), (20, 0, 30, 10, 35.0), (5, 20, 25, 30, 12.0)]
    sc = box_scene(boxes)
    perm = box_scene(boxes[::-1])
    split = box_scene([boxes[0], (20, 0, 25, 10, 35.0), (25, 0, 30, 10, 35.0), boxes[2]])
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=5.0)
    path = oracle.sun_path(span, seg_min=30.0)
    g = np.stack(np.meshgrid(np.arange(-30, 60, 7.3), np.arange(-30, 60, 6.1)), -1).reshape(-1, 2)
    P = pts(np.concatenate([g, np.zeros((len(g), 1))], 1))
    a = oracle.continuous(sc, P, path)["minutes"]
    b = oracle.continuous(perm, P, path)["minutes"]
    c = oracle.continuous(split, P, path)["minutes"]
    np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(a, c, atol=1e-6)


def test_sampled_converges_to_continuous(c1):
    """Sampled minutes approach the continuous duration as the step shrinks;
    each shadow transition costs at most half a step."""
    sub = c1.points.take(np.arange(5, c1.points.n, 211))
    errs = []
    for step in (5.0, 1.0):
        span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=step)
        path = oracle.sun_path(span, seg_min=step)   # knots at every instant: same path
        s = oracle.sampled(c1.scene, sub, path, bits=True)
        d = oracle.continuous(c1.scene, sub, path)
        K = len(path.w)
        bits = np.unpackbits(s["bits"].view(np.uint8), axis=1, bitorder="little")[:, :K].astype(int)
        trans = np.abs(np.diff(bits, axis=1)).sum(1)
        err = np.abs(s["minutes"][0] - d["minutes"][0])
        assert np.all(err <= trans * step / 2 + 1e-6)
        errs.append(err.mean())
    assert errs[1] < errs[0]


def test_counts_of_instants_inside_continuous_set(c1):
    """With knots at every instant, an instant lies in the continuous
    shadowed set exactly when the sampled predicate holds there."""
    path = oracle.sun_path(c1.span)
    sub = c1.points.take(np.arange(3, c1.points.n, 173))
    s = oracle.sampled(c1.scene, sub, path)
    d = oracle.continuous(c1.scene, sub, path)
    np.testing.assert_array_equal(s["counts"], d["counts"])


def test_equinox_path_is_nearly_great_circle(c1):
    """At the equinox the sun's daily path is (nearly) a great circle at a
    constant rate, so hour-long knots lose almost nothing; at the solstice
    the same knots deviate more, and the error falls roughly as L^2."""
    sub = c1.points.take(np.arange(7, c1.points.n, 257))
    res = {}
    for md, tz in (((3, 20), -4.0), ((6, 21), -4.0)):
        span = Span(40.7, -74.0, [Day(2019, *md, tz, (480.0, 1080.0))], step_min=5.0)
        ref = oracle.continuous(c1.scene, sub, oracle.sun_path(span, seg_min=1.0))["minutes"][0]
        for L in (30.0, 60.0):
            m = oracle.continuous(c1.scene, sub, oracle.sun_path(span, seg_min=L))["minutes"][0]
            res[(md, L)] = np.abs(m - ref).mean()
    assert res[((3, 20), 60.0)] < 0.02
    assert res[((6, 21), 60.0)] > 3 * res[((3, 20), 60.0)]
    assert res[((6, 21), 30.0)] < 0.5 * res[((6, 21), 60.0)]


def test_continuous_catches_runs_shorter_than_the_grid():
    """A thin pole 200 m away shadows a ground point for a few seconds; the
    default 5-second scan must find that run (gross shadow is the measure of
    the whole shadowed set, Sec. 3.1) and agree with a 0.05-second scan."""
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=5.0)
    path = oracle.sun_path(span, seg_min=30.0)
    # place the pole on the shadow line of the sun at 10:07 local, 200 m out
    s = oracle.solar(2019, 6, 21, 607.0, -4.0, 40.7, -74.0)
    d = s[:3]
    u = d[:2] / np.linalg.norm(d[:2])
    r = 200.0
    c = u * r
    h = r * math.tan(math.radians(s[3])) + 20.0
    sc = box_scene([(c[0] - 0.01, c[1] - 0.01, c[0] + 0.01, c[1] + 0.01, h)])
    P = pts([[0.0, 0.0, 0.0]])
    coarse = oracle.continuous(sc, P, path)["minutes"][0, 0]
    fine = oracle.continuous(sc, P, path, grid_min=1.0 / 1200.0)["minutes"][0, 0]
    assert 0.0 < fine < 5.0 / 60.0
    assert coarse == pytest.approx(fine, abs=1e-6)


# --------------------------------------------------------------------------
# gradient with respect to heights
# --------------------------------------------------------------------------
def test_gradient_implicit_matches_central_differences(c1):
    """The oracle's implicit-differentiation gradient against FP64 central
    differences of its own continuous duration (heights rounded to float32,
    so the difference quotient uses the actual step)."""
    sub = c1.points.take(np.arange(5, c1.points.n, 331))
    path = oracle.sun_path(c1.span, 30.0)
    g = oracle.grad_implicit(c1.scene, sub, path)
    assert np.all(g >= 0.0)                      # a taller building never shades less
    for b in list(np.argsort(-g)[:4]) + [int(np.flatnonzero(g == 0)[0])]:
        H = float(c1.scene.height[b])
        hp, hm = np.float32(H + 0.01), np.float32(H - 0.01)
        lp = oracle.continuous(oracle.with_height(c1.scene, b, hp), sub, path)["minutes"].sum()
        lm = oracle.continuous(oracle.with_height(c1.scene, b, hm), sub, path)["minutes"].sum()
        fd = (lp - lm) / float(hp - hm)
        if g[b] == 0:
            assert abs(fd) < 1e-6
        else:
            assert fd == pytest.approx(g[b], rel=2e-4)


def test_gradient_lone_box_roof_crossings():
    """A lone box on a winter morning: ground points where the tip of its
    shadow (the roof edge) passes have a positive height derivative equal to
    the central difference; a building far from every sun path owns no
    boundary (zero)."""
    span = Span(40.7, -74.0, [Day(2019, 12, 21, -5.0, (540.0, 720.0))], step_min=5.0)
    path = oracle.sun_path(span, seg_min=30.0)
    sc = box_scene([(-5, -5, 5, 5, 40.0), (900, 900, 910, 910, 20.0)])
    gx, gy = np.meshgrid(np.arange(-80.0, 0.0, 8.0) + 0.5, np.arange(40.0, 140.0, 8.0) + 0.5)
    P = pts(np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], 1))
    per_point = np.array([oracle.grad_implicit(sc, P.take([i]), path) for i in range(P.n)])
    assert np.all(per_point >= 0) and np.all(per_point[:, 1] == 0)
    i = int(np.argmax(per_point[:, 0]))
    assert per_point[i, 0] > 0
    one = P.take([i])
    hp, hm = np.float32(40.01), np.float32(39.99)
    lp = oracle.continuous(oracle.with_height(sc, 0, hp), one, path)["minutes"].sum()
    lm = oracle.continuous(oracle.with_height(sc, 0, hm), one, path)["minutes"].sum()
    assert (lp - lm) / float(hp - hm) == pytest.approx(per_point[i, 0], rel=2e-4)


def test_continuous_matches_unculled_fine_sampling():
    """Low boxes (0.3..3 m) a few metres from ground and wall points under a
    low morning sun, where the continuous form's box culls (the segment's
    plane, the half-space behind the arc, the rays' lowest elevation) sit
    close to the geometry: its duration along one hour-long great circle
    equals the predicate -- tested against every building, no cull --
    sampled every 0.6 s along the same circle, within half a sample per
    transition."""
    rng = np.random.default_rng(12)
    boxes = []
    for k in range(24):
        cx, cy = rng.uniform(-25, 25, 2)
        w, d = rng.uniform(0.5, 4.0, 2)
        boxes.append((cx - w, cy - d, cx + w, cy + d, rng.uniform(0.3, 3.0)))
    sc = box_scene(boxes)
    P = pts(np.c_[rng.uniform(-30, 30, (40, 2)), rng.uniform(0.0, 0.4, 40)])
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (340.0, 400.0))], step_min=5.0)
    path = oracle.sun_path(span, seg_min=60.0)
    assert len(path.seg_t) == 1
    D = oracle.continuous(sc, P, path)["minutes"][0]
    ta, tb = path.seg_t[0]
    dt = 0.01
    t = np.arange(ta, tb + 1e-9, dt)
    dirs = np.array([oracle.slerp(path.seg_dir[0, 0], path.seg_dir[0, 1], (x - ta) / (tb - ta)) for x in t])
    w_ = np.full(len(t), dt)
    w_[0] = w_[-1] = dt / 2
    z = np.zeros(len(t), np.int32)
    fine = oracle.OraclePath(dirs, w_, t, z, z, np.zeros((0, 2)), np.zeros((0, 2, 3)), np.zeros(0, np.int32),
                             np.zeros(1, np.int32), 1, np.array([[ta, tb]]))
    S = oracle.sampled(sc, P, fine, bits=True)
    bits = np.unpackbits(S["bits"].view(np.uint8), axis=1, bitorder="little")[:, :len(t)]
    trans = np.abs(np.diff(bits.astype(int), axis=1)).sum(1)
    assert (D > 0).sum() >= 10 and trans.sum() > 0
    assert np.all(np.abs(S["minutes"][0] - D) <= trans * dt / 2 + 1e-6)


def test_thin_pole_run_matches_great_circle_root_find():
    """The great-circle form's short-run detection against an analytic
    crossing: a 2 cm pole 200 m away shadows the point while the azimuth of
    the path's direction (slerp between the segment's knots) lies between
    the azimuths of the pole's silhouette corners; both ends by brentq on
    that azimuth."""
    from scipy.optimize import brentq
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=5.0)
    path = oracle.sun_path(span, seg_min=30.0)
    t_mid = 607.0 + 2.5 / 60.0
    j = int(np.searchsorted(path.seg_t[:, 0], t_mid, side="right") - 1)
    ta, tb = path.seg_t[j]
    on_arc = lambda t: oracle.slerp(path.seg_dir[j, 0], path.seg_dir[j, 1], (t - ta) / (tb - ta))
    d = on_arc(t_mid)
    az = math.atan2(d[0], d[1])
    c = 200.0 * np.array([math.sin(az), math.cos(az)])
    h = 200.0 * d[2] / math.hypot(d[0], d[1]) + 40.0
    sc = box_scene([(c[0] - 0.01, c[1] - 0.01, c[0] + 0.01, c[1] + 0.01, h)])
    corners = np.array(sc.footprint(0), np.float64)
    az_c = np.arctan2(corners[:, 0], corners[:, 1])
    arc_az = lambda t: math.atan2(on_arc(t)[0], on_arc(t)[1])
    t_in = brentq(lambda t: arc_az(t) - az_c.min(), t_mid - 1.0, t_mid + 1.0, xtol=1e-12)
    t_out = brentq(lambda t: arc_az(t) - az_c.max(), t_mid - 1.0, t_mid + 1.0, xtol=1e-12)
    D = oracle.continuous(sc, pts([[0.0, 0.0, 0.0]]), path)["minutes"][0, 0]
    assert 0.0 < abs(t_out - t_in) < 5.0 / 60.0
    assert D == pytest.approx(abs(t_out - t_in), abs=1e-6)
