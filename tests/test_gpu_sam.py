"""GPU raster shadow accrual maps (Sec. 4, sa_sam_accumulate) against the
oracle's raster form, decision by decision where the oracle says a float32
evaluation cannot go either way, and within the ambiguous instants'
weight elsewhere; error paths."""
import datetime as dt

import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Scene, Span, make_c1, make_c2, subset_points
from workloads.scenes import Day, _nyc_tz, _pts

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def box_of(scene):
    return (float(scene.xy[:, 0].min()), float(scene.xy[:, 1].min()), 0.0,
            float(scene.xy[:, 0].max()), float(scene.xy[:, 1].max()), float(scene.height.max()))


def gpu_sam(ctx, scene, pts, span, seg, texel, bias=0.01, box=None):
    path = sa.Path(ctx, sa.sunpath_for_span(span, seg))
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.ground_from_workload(pts)
    c, m = sa.sam_accumulate(ctx, sc, dp, path, texel, bias=bias, box=box)
    ctx.sync()
    return c.cpu().numpy(), m.cpu().numpy().astype(np.float64)


def check(ctx, scene, pts, span, seg, texel, box, label):
    say(f"sam parity: {label}, {pts.n} points, texel {texel} m")
    c, m = gpu_sam(ctx, scene, pts, span, seg, texel, box=box)
    path = oracle.sun_path(span, seg)
    o = oracle.sam(scene, pts, path, texel, box=box)
    amb = o["amb"].astype(bool)
    n_amb = np.zeros((path.n_bins, pts.n), np.int64)
    w_amb = np.zeros((path.n_bins, pts.n))
    for b in range(path.n_bins):
        sel = path.sample_bin == b
        n_amb[b] = amb[:, sel].sum(1)
        w_amb[b] = (amb[:, sel] * path.w[sel]).sum(1)
    dc = np.abs(c.astype(np.int64) - o["counts"])
    clean = n_amb == 0
    say(f"  {amb.mean():.2%} ambiguous decisions; counts differ at {(dc > 0).mean():.2%} of point-bins "
        f"(clean ones {(dc[clean] > 0).mean() if clean.any() else 0:.2%}); mean count {c.mean():.2f} "
        f"oracle {o['counts'].mean():.2f}")
    assert np.array_equal(c[clean], o["counts"][clean])
    assert np.all(dc <= n_amb)
    assert np.all(np.abs(m - o["minutes"]) <= w_amb + 1e-3 * (1 + o["minutes"]))
    return c, o


@pytest.mark.parametrize("texel", [1.0, 0.5])
def test_sam_small_scene_matches_oracle(ctx, texel):
    w = make_c1()
    sub = w.points.take(subset_points(w.points, 1024, 81))
    c, o = check(ctx, w.scene, sub, w.span, 30.0, texel, box_of(w.scene), "small scene, June 21")
    assert o["counts"].sum() > 0


def test_sam_two_days_ragged_tail(ctx):
    """Two days in two bins, 45-minute knots (ragged last segments), 777
    points (a ragged final block)."""
    w = make_c1()
    sub = w.points.take(subset_points(w.points, 777, 82))
    days = [Day(x.year, x.month, x.day, _nyc_tz(x), (9 * 60, 15 * 60)) for x in (dt.date(2019, 3, 20), dt.date(2019, 12, 21))]
    span = Span(40.7, -74.0, days, 5.0, [0, 1])
    check(ctx, w.scene, sub, span, 45.0, 1.0, box_of(w.scene), "equinox + winter solstice")


def test_sam_block_scene_subset(ctx):
    """The block scene (20,000 prisms), 256 of its ground points, an hour
    at 1-minute instants: the map spans the whole scene at 2 m texels."""
    w = make_c2(n_ground=20_000, n_facade=0)
    sub = w.points.take(subset_points(w.points, 256, 83))
    day = w.span.days[0]
    span = Span(w.span.lat, w.span.lon, [Day(day.year, day.month, day.day, day.tz_h, (15 * 60, 16 * 60))], 1.0)
    check(ctx, w.scene, sub, span, 30.0, 2.0, box_of(w.scene), "block scene, 15:00-16:00")


def test_sam_lone_box_against_exact(ctx):
    """A lone box at 0.1 m texels, points on a 5 m lattice around it,
    against the oracle's map (which its pins tie to the exact predicate
    away from shadow edges at such texels)."""
    xy = np.array([[0, 0], [20, 0], [20, 30], [0, 30]], np.float32)
    sc = Scene(np.array([0, 4], np.int32), xy, np.array([40.0], np.float32))
    g = np.arange(-60.0, 81.0, 5.0) + 0.37
    X, Y = np.meshgrid(g, g)
    pts = _pts(X.ravel(), Y.ravel())
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (7 * 60, 17 * 60))], 30.0)
    check(ctx, sc, pts, span, 60.0, 0.1, (0, 0, 0, 20, 30, 40), "lone box")


def test_sam_edge_cases(ctx):
    w = make_c1()
    span = w.span
    path = sa.Path(ctx, sa.sunpath_for_span(span, 30.0))
    sc = sa.Scene.from_workload(ctx, w.scene)
    say("sam edge cases: empty points, empty scene, errors")
    import torch
    empty = sa.DevicePoints(*(torch.zeros(0, device="cuda") for _ in range(3)))
    c, m = sa.sam_accumulate(ctx, sc, empty, path, 1.0)
    assert c.numel() == 0
    none = Scene(np.array([0], np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))
    pts = w.points.take(np.arange(100))
    c, m = sa.sam_accumulate(ctx, sa.Scene.from_workload(ctx, none), sa.DevicePoints.ground_from_workload(pts),
                             path, 1.0, box=(0, 0, 0, 1, 1, 1))
    ctx.sync()
    assert int(c.sum()) == 0 and float(m.sum()) == 0.0
    dp = sa.DevicePoints.ground_from_workload(pts)
    with pytest.raises(sa.SAError) as e:
        sa.sam_accumulate(ctx, sc, dp, path, 0.0)
    assert e.value.code == -1
    with pytest.raises(sa.SAError) as e:                       # facade arrays given
        sa.sam_accumulate(ctx, sc, sa.DevicePoints.from_workload(pts), path, 1.0)
    assert e.value.code == -1
    with pytest.raises(sa.SAError) as e:                       # graph paths have no per-segment instants
        sa.sam_accumulate(ctx, sc, dp, sa.Path(ctx, sa.sunpath_for_span(span, 30.0), graph_bound_deg=1.0), 1.0)
    assert e.value.code == -1
    with pytest.raises(sa.SAError) as e:                       # a map above the cap
        sa.sa_sam_accumulate(ctx, sc, dp, path, 1.0, torch.empty((1, 100), dtype=torch.int32, device="cuda"),
                             max_texels=1000)
    assert e.value.code == -3
    with pytest.raises(ValueError):
        sa.DevicePoints.ground_from_workload(make_c2(n_ground=0, n_facade=100).points)


def test_sam_repeated_calls_reuse_the_map(ctx):
    """One context, three calls: 1 m texels, then 0.5 m (a larger map, a
    new buffer), then 1 m again over the stale words of both: the last call
    equals the first exactly (words of earlier segments carry older stamps
    and read as empty); then enough calls to wrap the stamp twice."""
    w = make_c1()
    sub = w.points.take(subset_points(w.points, 512, 84))
    say("sam repeated calls on one context: 1 m, 0.5 m, 1 m")
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.ground_from_workload(sub)
    c1, m1 = sa.sam_accumulate(ctx, sc, dp, path, 1.0)
    c2, m2 = sa.sam_accumulate(ctx, sc, dp, path, 0.5)
    c3, m3 = sa.sam_accumulate(ctx, sc, dp, path, 1.0)
    ctx.sync()
    assert int(c1.sum()) > 0
    assert np.array_equal(c1.cpu().numpy(), c3.cpu().numpy())
    assert np.array_equal(m1.cpu().numpy(), m3.cpu().numpy())
    assert not np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    # past the 8-bit segment stamp's wrap (a map clear every 255 segments):
    # 27 more calls of this path's segments, every one equal to the first
    for _ in range(27):
        c4, m4 = sa.sam_accumulate(ctx, sc, dp, path, 1.0)
        ctx.sync()
        assert np.array_equal(c1.cpu().numpy(), c4.cpu().numpy())
    assert 30 * path.n_segments > 2 * 255


def test_sam_bench_configuration_sampled_points(ctx):
    """The configuration the raster bench times (the block scene's 2M
    ground points, June 21 at 1-minute instants, 30-minute knots, 2 m
    texels, the scene's own box), run on every point; 32 seeded points
    checked against the oracle's map one by one."""
    w = make_c2(n_facade=0)
    span = Span(w.span.lat, w.span.lon, [w.span.days[1]], w.span.step_min)
    say(f"sam at the bench configuration: {w.points.n} points, 2 m texels")
    path = sa.Path(ctx, sa.sunpath_for_span(span, 30.0))
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.ground_from_workload(w.points)
    c, m = sa.sam_accumulate(ctx, sc, dp, path, 2.0)
    ctx.sync()
    idx = subset_points(w.points, 32, 85)
    c, m = c.cpu().numpy()[:, idx], m.cpu().numpy()[:, idx].astype(np.float64)
    sub = w.points.take(idx)
    opath = oracle.sun_path(span, 30.0)
    o = oracle.sam(w.scene, sub, opath, 2.0, box=box_of(w.scene))
    n_amb = o["amb"].sum(1)[None, :]
    w_amb = (o["amb"] * opath.w[None, :]).sum(1)[None, :]
    dc = np.abs(c.astype(np.int64) - o["counts"])
    say(f"  {o['amb'].mean():.2%} ambiguous; counts differ at {(dc > 0).sum()} of {dc.size} points; "
        f"mean count {c.mean():.1f} oracle {o['counts'].mean():.1f}")
    assert o["counts"].sum() > 0
    assert np.array_equal(c[n_amb == 0], o["counts"][n_amb == 0])
    assert np.all(dc <= n_amb)
    assert np.all(np.abs(m - o["minutes"]) <= w_amb + 1e-3 * (1 + o["minutes"]))
