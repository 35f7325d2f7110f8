"""GPU parity of the continuous shadow (Sec. 3.1: the longest time a point
stays in shadow without interruption within a day, maximum over a bin's
days) against the oracle, in both forms, through the C ABI."""
import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Span, make_c2, subset_points
from workloads.scenes import Day

from gpu_util import say, unpack_words
from test_gpu_spill import SPAN as RING_SPAN, centre_points, ring_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def run(ctx, scene, pts, span, mode, seg_min=30.0, bits=False, flags=0, longest=None, minutes=None):
    import torch
    sp = sa.sunpath_for_span(span, seg_min)
    path = sa.Path(ctx, sp)
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    dev = "cuda"
    c = torch.empty((path.n_bins, dp.n), dtype=torch.int32, device=dev)
    m = minutes if minutes is not None else torch.empty((path.n_bins, dp.n), dtype=torch.float32, device=dev)
    L = longest if longest is not None else torch.empty((path.n_bins, dp.n), dtype=torch.float32, device=dev)
    b = torch.empty(((sp.n_samples + 31) // 32, dp.n), dtype=torch.int32, device=dev) if bits else None
    sa.sa_accumulate(ctx, sc, dp, path, mode, c, m, b, flags, 1.0, longest=L)
    ctx.sync()
    out = dict(counts=c.cpu().numpy(), minutes=m.cpu().numpy().astype(np.float64),
               longest=L.cpu().numpy().astype(np.float64), L=L, m=m)
    if bits:
        out["bits"] = unpack_words(b.cpu().numpy().view(np.uint32).T, sp.n_samples)
    return out


def test_sampled_longest_is_the_longest_run_of_its_bits(ctx, c1):
    """The sampled form's continuous shadow is the definition applied to its
    own predicate (whose bits match the oracle's, tested elsewhere), and
    within the ambiguous instants' weight of the oracle's."""
    say("sampled continuous shadow, small scene")
    g = run(ctx, c1.scene, c1.points, c1.span, sa.SA_SAMPLED, bits=True)
    op = oracle.sun_path(c1.span)
    ref = oracle.longest_sampled(g["bits"].astype(bool), op)
    np.testing.assert_allclose(g["longest"], ref, rtol=1e-6, atol=1e-4)
    sub = c1.points.take(np.arange(0, c1.points.n, 7))
    o = oracle.sampled(c1.scene, sub, op, bits=True, amb=True)
    ob = unpack_words(o["bits"], len(op.w)).astype(bool)
    lo = oracle.longest_sampled(ob, op)
    slack = (o["amb"].astype(bool) * op.w[None, :]).sum(1)
    d = np.abs(g["longest"][:, ::7] - lo)
    assert np.all(d <= slack[None, :] + 1e-3)
    assert (g["longest"] > 0).mean() > 0.3


@pytest.mark.parametrize("seg", [30.0, 60.0])
def test_accrual_longest_small_scene(ctx, c1, seg):
    idx = subset_points(c1.points, 2048, seed=7)
    sub = c1.points.take(idx)
    say(f"accrual continuous shadow, small scene, L={seg}")
    g = run(ctx, c1.scene, sub, c1.span, sa.SA_ACCRUAL, seg_min=seg)
    o = oracle.continuous(c1.scene, sub, oracle.sun_path(c1.span, seg))
    for k in ("minutes", "longest"):
        d = np.abs(g[k] - o[k]).ravel()
        say(f"  {k}: |GPU - oracle| mean {d.mean():.2e} p99.9 {np.quantile(d, 0.999):.2e} max {d.max():.2e}")
        assert np.quantile(d, 0.999) <= 0.01 and d.mean() <= 1e-3
    assert (g["longest"] < g["minutes"] - 1.0).any()     # some points have broken shadow


def test_accrual_longest_block_scene_three_days(ctx):
    w = make_c2(n_ground=50_000, n_facade=50_000)
    idx = np.concatenate([subset_points(w.points.take(np.arange(50_000)), 96, 8),
                          50_000 + subset_points(w.points.take(np.arange(50_000, 100_000)), 96, 9)])
    sub = w.points.take(idx)
    say("accrual continuous shadow, block scene subset", sub.n)
    g = run(ctx, w.scene, sub, w.span, sa.SA_ACCRUAL)
    o = oracle.continuous(w.scene, sub, oracle.sun_path(w.span, 30.0))
    d = np.abs(g["longest"] - o["longest"]).ravel()
    say(f"  longest: mean {d.mean():.2e} p99.9 {np.quantile(d, 0.999):.2e} max {d.max():.2e}")
    assert np.quantile(d, 0.999) <= 0.01 and d.mean() <= 1e-3


def test_one_bin_over_two_days_is_the_maximum(ctx, c1):
    sub = c1.points.take(np.arange(0, c1.points.n, 11))
    days = [Day(2019, 3, 20, -4.0, (480.0, 1080.0)), Day(2019, 6, 21, -4.0, (480.0, 1080.0))]
    for mode in (sa.SA_SAMPLED, sa.SA_ACCRUAL):
        sep = run(ctx, c1.scene, sub, Span(40.7, -74.0, days, 5.0), mode)
        one = run(ctx, c1.scene, sub, Span(40.7, -74.0, days, 5.0, day_bin=[0, 0]), mode)
        np.testing.assert_array_equal(one["longest"][0], sep["longest"].max(0))
        np.testing.assert_allclose(one["minutes"][0], sep["minutes"].sum(0), rtol=1e-6, atol=1e-3)


def test_add_flag_keeps_the_larger(ctx, c1):
    import torch
    sub = c1.points.take(np.arange(0, c1.points.n, 13))
    g = run(ctx, c1.scene, sub, c1.span, sa.SA_ACCRUAL)
    L = torch.zeros_like(g["L"])
    L[:, ::2] = 1e4
    g2 = run(ctx, c1.scene, sub, c1.span, sa.SA_ACCRUAL, flags=sa.SA_FLAG_ADD, longest=L, minutes=g["m"].clone())
    expect = g["longest"].copy()
    expect[:, ::2] = 1e4
    np.testing.assert_array_equal(g2["longest"], expect)
    np.testing.assert_allclose(g2["minutes"], 2 * g["minutes"], rtol=1e-6)


def test_overflowing_sets_walked_in_order(ctx):
    """The ring of poles: sets of more than four pieces are walked window by
    window inside the kernel; minutes and longest runs match the oracle."""
    scene, pts = ring_scene(), centre_points()
    g = run(ctx, scene, pts, RING_SPAN, sa.SA_ACCRUAL)
    o = oracle.continuous(scene, pts, oracle.sun_path(RING_SPAN, 30.0))
    say(f"ring: longest {g['longest'].ravel()[:4]}, oracle {o['longest'].ravel()[:4]}")
    assert np.abs(g["minutes"] - o["minutes"]).max() <= 0.01
    assert np.abs(g["longest"] - o["longest"]).max() <= 0.01


def test_accrual_longest_over_several_view_launches(ctx):
    """Twelve days on the block scene (20k prisms): about 300 segments, more
    than one launch's budget of per-segment node views (256 MiB, ~209
    segments here), so the continuous-shadow kernel runs in two launches of
    whole days.  Against the oracle, one bin per day."""
    import datetime as dt
    from workloads.scenes import _nyc_tz
    w = make_c2(n_ground=20_000, n_facade=20_000)
    idx = np.concatenate([subset_points(w.points.take(np.arange(20_000)), 48, 21),
                          20_000 + subset_points(w.points.take(np.arange(20_000, 40_000)), 48, 22)])
    sub = w.points.take(idx)
    days = [dt.date(2019, m, 21) for m in range(1, 13)]
    span = Span(40.7, -74.0, [Day(d.year, d.month, d.day, _nyc_tz(d)) for d in days], 1.0)
    sp = sa.sunpath_for_span(span, 30.0)
    n_segs = len(sp.knot_t) - sp.n_days
    assert n_segs * (w.scene.n_b - 1) * 64 > 256 << 20
    say(f"continuous shadow, 12 days, {n_segs} segments")
    g = run(ctx, w.scene, sub, span, sa.SA_ACCRUAL)
    o = oracle.continuous(w.scene, sub, oracle.sun_path(span, 30.0))
    for k in ("minutes", "longest"):
        d = np.abs(g[k] - o[k]).ravel()
        say(f"  {k}: |GPU - oracle| mean {d.mean():.2e} p99.9 {np.quantile(d, 0.999):.2e} max {d.max():.2e}")
        assert np.quantile(d, 0.999) <= 0.01 and d.mean() <= 1e-3


def test_sampled_longest_block_scene(ctx):
    """Block scene (20k prisms), three days at 1-minute instants: the
    sampled form's longest run must be the definition applied to its own
    predicate bits (whose parity with the oracle is tested elsewhere)."""
    w = make_c2(n_ground=20_000, n_facade=20_000)
    idx = np.concatenate([subset_points(w.points.take(np.arange(20_000)), 64, 31),
                          20_000 + subset_points(w.points.take(np.arange(20_000, 40_000)), 64, 32)])
    sub = w.points.take(idx)
    g = run(ctx, w.scene, sub, w.span, sa.SA_SAMPLED, bits=True)
    ref = oracle.longest_sampled(g["bits"].astype(bool), oracle.sun_path(w.span))
    d = np.abs(g["longest"] - ref)
    say(f"sampled longest, block scene: max |GPU - definition| {d.max():.2e}, mean longest {ref.mean():.1f}")
    np.testing.assert_allclose(g["longest"], ref, rtol=1e-6, atol=1e-3)
    assert (ref > 60).mean() > 0.2
