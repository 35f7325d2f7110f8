"""GPU parity of the building contribution and the region shadow score
(Sec. 7.2) against the oracle, through the C ABI."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Span, make_c2, subset_points
from workloads.scenes import Day

from gpu_util import say

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def gpu_contrib(ctx, scene, pts, span, seg_min=30.0, weight=None):
    import torch
    path = sa.Path(ctx, sa.sunpath_for_span(span, seg_min))
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    w = None if weight is None else torch.from_numpy(weight.astype(np.float32)).cuda()
    out = sa.building_contribution(ctx, sc, dp, path, w)
    ctx.sync()
    return out.cpu().numpy()


def test_contribution_small_scene(ctx, c1):
    idx = subset_points(c1.points, 2048, seed=11)
    sub = c1.points.take(idx)
    wt = np.random.default_rng(3).uniform(0.5, 2.0, sub.n)
    g = gpu_contrib(ctx, c1.scene, sub, c1.span, weight=wt)
    o = oracle.contribution(c1.scene, sub, oracle.sun_path(c1.span, 30.0), weight=wt.astype(np.float32))
    d = np.abs(g - o)
    say(f"contribution small scene: total {o.sum():.4e}, max |GPU - oracle| {d.max():.3e}")
    assert d.max() <= 1e-5 * o.sum() + 0.05
    # every shadowed moment counts at least once
    tot = oracle.continuous(c1.scene, sub, oracle.sun_path(c1.span, 30.0))["minutes"]
    assert g.sum() >= (tot[0] * wt).sum() - 1e-3 * g.sum()


def test_contribution_block_scene_facades(ctx):
    w = make_c2(n_ground=20_000, n_facade=20_000)
    idx = np.concatenate([subset_points(w.points.take(np.arange(20_000)), 48, 12),
                          20_000 + subset_points(w.points.take(np.arange(20_000, 40_000)), 48, 13)])
    sub = w.points.take(idx)
    g = gpu_contrib(ctx, w.scene, sub, w.span)
    o = oracle.contribution(w.scene, sub, oracle.sun_path(w.span, 30.0))
    d = np.abs(g - o)
    say(f"contribution block scene: buildings with shadow {int((o > 0).sum())}, max |GPU - oracle| {d.max():.3e}")
    assert d.max() <= 1e-5 * o.sum() + 0.05
    own = np.unique(sub.owner[sub.owner >= 0])
    assert (o[:, own] > 0).any()       # back-facing walls counted for their buildings


def test_bin_span_and_score(ctx):
    """Daylight per bin from the library equals the oracle's spans; the
    score reduction equals an FP64 numpy sum with the paper's month weights."""
    import torch
    days = [Day(2019, m, 21, -5.0 if m in (1, 2, 11, 12) else -4.0, None) for m in range(1, 13)]
    span = Span(40.7, -74.0, days, 1.0)
    path = sa.Path(ctx, sa.sunpath_for_span(span, 30.0))
    op = oracle.sun_path(span, 30.0)
    osp = np.zeros(op.n_bins)
    np.add.at(osp, op.day_bin, op.spans[:, 1] - op.spans[:, 0])
    np.testing.assert_allclose(path.bin_span(), osp, rtol=1e-12, atol=1e-9)
    with open(os.path.join(GOLD, "paper_table_month_weights.json")) as f:
        wt = json.load(f)["weights"]
    w12 = np.array([wt[k] for k in ("Jan", "Feb", "Mar", "Apr", "May", "Jun", "Jul", "Aug", "Sep", "Oct",
                                    "Nov", "Dec")])
    rng = np.random.default_rng(5)
    n = 300_001
    vals = (rng.uniform(0, 1, (12, n)) * osp[:, None]).astype(np.float32)
    area = rng.uniform(0.5, 2.0, n).astype(np.float32)
    cuts = np.sort(rng.choice(np.arange(1, n), 4, replace=False))
    off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    got = sa.shadow_score(ctx, path, torch.from_numpy(vals).cuda(), w12, torch.from_numpy(off).cuda(),
                          torch.from_numpy(area).cuda())
    ctx.sync()
    ref = [oracle.shadow_score(vals[:, off[r]:off[r + 1]], w12, osp, area[off[r]:off[r + 1]])
           for r in range(len(off) - 1)]
    np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-10, atol=1e-6)


def test_contribution_over_several_view_launches(ctx):
    """Twelve days on the block scene: more segments than one launch's budget
    of per-segment node views, so the contribution kernel runs in several
    launches.  Against the oracle, one bin per day."""
    import datetime as dt
    from workloads.scenes import _nyc_tz
    w = make_c2(n_ground=20_000, n_facade=20_000)
    idx = np.concatenate([subset_points(w.points.take(np.arange(20_000)), 24, 23),
                          20_000 + subset_points(w.points.take(np.arange(20_000, 40_000)), 24, 24)])
    sub = w.points.take(idx)
    days = [dt.date(2019, m, 21) for m in range(1, 13)]
    span = Span(40.7, -74.0, [Day(d.year, d.month, d.day, _nyc_tz(d)) for d in days], 1.0)
    sp = sa.sunpath_for_span(span, 30.0)
    assert (len(sp.knot_t) - sp.n_days) * (w.scene.n_b - 1) * 64 > 256 << 20
    g = gpu_contrib(ctx, w.scene, sub, span)
    o = oracle.contribution(w.scene, sub, oracle.sun_path(span, 30.0))
    d = np.abs(g - o)
    say(f"contribution, 12 days: max |GPU - oracle| {d.max():.3e} of total {o.sum():.4e}")
    assert g.shape == o.shape == (12, w.scene.n_b)
    assert d.max() <= 1e-5 * o.sum() + 0.05
