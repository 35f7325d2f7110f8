"""GPU parity: the HIP library against the FP64 CPU oracle on the same
seeded inputs, through the C ABI.

Bars:
 * sampled form: per (point, instant) predicate bit-exact except for rays
   within 1e-5 rad of a silhouette (the oracle's ambiguity mask), which
   must be at most 1e-4 of all pairs;
 * accrual form vs the oracle's continuous duration along the same
   great-circle path: |GPU - oracle| <= 0.01 min for 99.9% of points,
   mean <= 1e-3 min (float32 geometry against FP64 bisection), and never
   more than 0.5 min.
"""
import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Scene, Span, make_c1, make_c2, subset_points
from workloads.scenes import Day

from gpu_util import check_sampled, run_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


@pytest.fixture(scope="module")
def c2small():
    return make_c2(n_ground=100_000, n_facade=100_000)


def accrual_bar(g, o, label):
    d = np.abs(g["minutes"] - o["minutes"]).ravel()
    q999, mean, mx = np.quantile(d, 0.999), d.mean(), d.max()
    say(f"{label}: |A-D_L| mean {mean:.2e} p99.9 {q999:.2e} max {mx:.2e} min")
    assert q999 <= 0.01 and mean <= 1e-3 and mx <= 0.5


def test_sampled_c1_full(ctx, c1):
    say("sampled C1 full")
    g = run_lib(ctx, c1.scene, c1.points, c1.span, sa.SA_SAMPLED, bits=True)
    o = oracle.sampled(c1.scene, c1.points, oracle.sun_path(c1.span), bits=True, amb=True)
    frac, nm = check_sampled(g, o, oracle.sun_path(c1.span).w)
    say(f"  ambiguous fraction {frac:.2e}, mismatched pairs {nm}")
    assert frac <= 1e-4


@pytest.mark.parametrize("seg", [30.0, 60.0])
def test_accrual_c1(ctx, c1, seg):
    say(f"accrual C1 seg {seg}")
    idx = subset_points(c1.points, 2048, seed=5)
    sub = c1.points.take(idx)
    g = run_lib(ctx, c1.scene, sub, c1.span, sa.SA_ACCRUAL, seg_min=seg)
    o = oracle.continuous(c1.scene, sub, oracle.sun_path(c1.span, seg))
    accrual_bar(g, o, f"C1 L={seg}")
    # sample instants inside the occluded set: equal except where an end of
    # the set sits on an instant
    dc = np.abs(g["counts"] - o["counts"])
    assert (dc > 0).mean() <= 2e-3 and dc.max() <= 1


def test_sampled_c2_subset(ctx, c2small):
    w = c2small
    idx = np.concatenate([subset_points(w.points.take(np.arange(100_000)), 192, 1),
                          100_000 + subset_points(w.points.take(np.arange(100_000, 200_000)), 192, 2)])
    sub = w.points.take(idx)
    say("sampled C2 subset", sub.n)
    g = run_lib(ctx, w.scene, sub, w.span, sa.SA_SAMPLED, bits=True)
    op = oracle.sun_path(w.span)
    o = oracle.sampled(w.scene, sub, op, bits=True, amb=True)
    frac, nm = check_sampled(g, o, op.w)
    say(f"  ambiguous fraction {frac:.2e}, mismatched pairs {nm}")
    assert frac <= 1e-4


def test_accrual_c2_subset(ctx, c2small):
    w = c2small
    idx = np.concatenate([subset_points(w.points.take(np.arange(100_000)), 96, 3),
                          100_000 + subset_points(w.points.take(np.arange(100_000, 200_000)), 96, 4)])
    sub = w.points.take(idx)
    say("accrual C2 subset", sub.n)
    g = run_lib(ctx, w.scene, sub, w.span, sa.SA_ACCRUAL, seg_min=30.0)
    o = oracle.continuous(w.scene, sub, oracle.sun_path(w.span, 30.0))
    accrual_bar(g, o, "C2 L=30")


def test_ragged_and_tiny_point_sets(ctx, c1):
    for n in (1, 63, 65, 200):
        sub = c1.points.take(np.arange(7, 7 + n * 13, 13))
        g = run_lib(ctx, c1.scene, sub, c1.span, sa.SA_SAMPLED, bits=True)
        o = oracle.sampled(c1.scene, sub, oracle.sun_path(c1.span), bits=True, amb=True)
        check_sampled(g, o, oracle.sun_path(c1.span).w)
        ga = run_lib(ctx, c1.scene, sub, c1.span, sa.SA_ACCRUAL)
        oa = oracle.continuous(c1.scene, sub, oracle.sun_path(c1.span, 30.0))
        assert np.abs(ga["minutes"] - oa["minutes"]).max() <= 0.05


def test_zero_points(ctx, c1):
    sub = c1.points.take(np.arange(0))
    g = run_lib(ctx, c1.scene, sub, c1.span, sa.SA_SAMPLED)
    assert g["minutes"].size == 0


def test_empty_and_single_building_scenes(ctx, c1):
    empty = Scene(np.zeros(1, np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))
    sub = c1.points.take(np.arange(0, c1.points.n, 101))
    for mode in (sa.SA_SAMPLED, sa.SA_ACCRUAL):
        g = run_lib(ctx, empty, sub, c1.span, mode)
        assert np.all(g["minutes"] == 0) and np.all(g["counts"] == 0)
    one = c1.scene.subset(np.array([5]))
    g = run_lib(ctx, one, sub, c1.span, sa.SA_SAMPLED, bits=True)
    o = oracle.sampled(one, sub, oracle.sun_path(c1.span), bits=True, amb=True)
    check_sampled(g, o, oracle.sun_path(c1.span).w)
    ga = run_lib(ctx, one, sub, c1.span, sa.SA_ACCRUAL)
    oa = oracle.continuous(one, sub, oracle.sun_path(c1.span, 30.0))
    assert np.abs(ga["minutes"] - oa["minutes"]).max() <= 0.05


def test_bvh_structure(ctx, c2small):
    w = c2small
    sc = sa.Scene.from_workload(ctx, w.scene)
    info = sc.info()
    nodes, order = sc.read_bvh()
    say("bvh", info)
    assert info["n_nodes"] == w.scene.n_b - 1 and 1 <= info["depth"] <= 63
    assert np.array_equal(np.sort(order), np.arange(w.scene.n_b))
    f = nodes.view(np.float32)
    # every prism box lies in every box on its path from the root
    lo = np.minimum.reduceat(w.scene.xy, w.scene.vert_off[:-1], axis=0)
    hi = np.maximum.reduceat(w.scene.xy, w.scene.vert_off[:-1], axis=0)
    seen = np.zeros(w.scene.n_b, int)
    stack = [0]
    boxes = {0: None}
    while stack:
        i = stack.pop()
        for side, ref in ((0, nodes[i, 10]), (1, nodes[i, 11])):
            b = f[i, side * 4: side * 4 + 4]
            z1 = f[i, 8 + side]
            if ref < 0:
                prim = order[~ref]
                assert b[0] <= lo[prim, 0] and b[1] <= lo[prim, 1] and b[2] >= hi[prim, 0] and b[3] >= hi[prim, 1]
                assert z1 >= w.scene.height[prim]
                seen[prim] += 1
            else:
                stack.append(ref)
    assert np.all(seen == 1)


def test_set_heights_matches_fresh_upload(ctx, c1):
    """Refit after a height edit gives the same result as uploading the
    edited scene."""
    sub = c1.points.take(np.arange(0, c1.points.n, 37))
    ids = np.array([3, 17, 40])
    newh = np.array([140.0, 12.0, 99.0], np.float32)
    edited = Scene(c1.scene.vert_off, c1.scene.xy, c1.scene.height.copy())
    edited.height[ids] = newh
    sp = sa.sunpath_for_span(c1.span, 30.0)
    path = sa.Path(ctx, sp)
    dp = sa.DevicePoints.from_workload(sub)
    s1 = sa.Scene.from_workload(ctx, c1.scene)
    s1.set_heights(ids, newh)
    s2 = sa.Scene.from_workload(ctx, edited)
    for mode in (sa.SA_SAMPLED, sa.SA_ACCRUAL):
        a = sa.accumulate(ctx, s1, dp, path, mode)
        b = sa.accumulate(ctx, s2, dp, path, mode)
        ctx.sync()
        assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
        assert np.array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())


def test_invalid_geometry_rejected(ctx):
    cw = np.array([[0, 0], [0, 10], [10, 10], [10, 0]], np.float32)   # clockwise
    with pytest.raises(sa.SAError) as e:
        sa.Scene(ctx, np.array([0, 4], np.int32), cw, np.array([10.0], np.float32))
    assert e.value.code == -2
    with pytest.raises(sa.SAError):
        sa.Scene(ctx, np.array([0, 4], np.int32), cw[::-1].copy(), np.array([-1.0], np.float32))


def test_region_sums(ctx):
    import torch
    rng = np.random.default_rng(9)
    v = rng.uniform(0, 600, 1_000_003).astype(np.float32)
    a = rng.uniform(0.5, 2.0, v.size).astype(np.float32)
    cuts = np.sort(rng.choice(np.arange(1, v.size), 7, replace=False))
    off = np.concatenate([[0], cuts, [v.size]]).astype(np.int64)
    out = torch.empty(len(off) - 1, dtype=torch.float64, device="cuda")
    sa.sa_region_sum(ctx, torch.from_numpy(v).cuda(), torch.from_numpy(off).cuda(), out, torch.from_numpy(a).cuda())
    ctx.sync()
    ref = np.array([np.sum(v[off[r]:off[r + 1]].astype(np.float64) * a[off[r]:off[r + 1]]) for r in range(len(off) - 1)])
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-12)


def test_full_size_c2_sampled_outputs(ctx):
    """The benchmark's workload at full size (20k prisms, 4M points, 3 days):
    both forms in the benchmark's launch configuration; sampled points
    checked against the oracle one by one."""
    import torch
    w = make_c2()
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    cs, ms, _ = sa.accumulate(ctx, sc, dp, path, sa.SA_SAMPLED)
    ca, ma, _ = sa.accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL)
    ctx.sync()
    idx = np.concatenate([subset_points(w.points.take(np.arange(2_000_000)), 64, 51),
                          2_000_000 + subset_points(w.points.take(np.arange(2_000_000, 4_000_000)), 64, 52)])
    sub = w.points.take(idx)
    op = oracle.sun_path(w.span)
    o = oracle.sampled(w.scene, sub, op, amb=True)
    na = o["amb"].sum(1)
    dc = np.abs(cs.cpu().numpy()[:, idx].sum(0) - o["counts"].sum(0))
    assert np.all(dc <= na)
    oc = oracle.continuous(w.scene, sub, oracle.sun_path(w.span, 30.0))
    d = np.abs(ma.cpu().numpy()[:, idx] - oc["minutes"])
    say(f"full C2 sampled points: ambiguous {na.sum()}, accrual |A-D_L| max {d.max():.2e}")
    assert np.quantile(d, 0.999) <= 0.01 and d.max() <= 0.5


@pytest.mark.parametrize("site", ["sydney_winter", "oslo_summer", "quito_equinox"])
def test_other_sites_and_seasons(ctx, c1, site):
    """The small scene under other skies: southern hemisphere in June (low
    northern sun), 60 N at midsummer (an 18-hour day, sun low in the north
    at both ends) and the equator at the equinox (the sun path through the
    zenith's neighbourhood: segment planes within a fraction of a degree of
    vertical).  Both forms against the oracle, sunrise to sunset at
    5-minute instants."""
    lat, lon, tz, day = {"sydney_winter": (-33.9, 151.2, 10.0, (2019, 6, 21)),
                         "oslo_summer": (59.9, 10.7, 2.0, (2019, 6, 21)),
                         "quito_equinox": (-0.2, -78.5, -5.0, (2019, 3, 20))}[site]
    span = Span(lat, lon, [Day(day[0], day[1], day[2], tz)], 5.0)
    sub = c1.points.take(subset_points(c1.points, 1024, seed=17))
    # planes of the noon segments near the zenith: their vertical part
    sp = sa.sunpath_for_span(span, 30.0)
    kd = sp.knot_dir.reshape(-1, 3)
    nz = np.abs(np.cross(kd[:-1], kd[1:])[:, 2]) / np.linalg.norm(np.cross(kd[:-1], kd[1:]), axis=1)
    say(f"{site}: smallest |nz| of a segment plane {nz.min():.2e}")
    if site == "quito_equinox":
        assert nz.min() < np.sin(np.radians(1.0))     # the steep-plane path is exercised
    g = run_lib(ctx, c1.scene, sub, span, sa.SA_SAMPLED, bits=True)
    o = oracle.sampled(c1.scene, sub, oracle.sun_path(span), bits=True, amb=True)
    frac, n_mism = check_sampled(g, o, oracle.sun_path(span).w)
    say(f"{site}: {g['K']} instants, ambiguous {frac:.2e}, mismatched bits {n_mism}")
    assert frac <= 1e-4
    for seg in (30.0, 60.0):
        ga = run_lib(ctx, c1.scene, sub, span, sa.SA_ACCRUAL, seg_min=seg)
        oa = oracle.continuous(c1.scene, sub, oracle.sun_path(span, seg))
        accrual_bar(ga, oa, f"  {site} L={seg}")
