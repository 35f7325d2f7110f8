"""Output handling of the accrual form and the height edits, through the C
ABI: outputs pre-filled with garbage are fully written (each bin stored
once when the path's bins are contiguous, cleared first when they
interleave), SA_FLAG_ADD adds, the FP64 minutes are the float minutes
before rounding, a device-array height edit equals the host one and flags
bad entries for sa_sync, and the gradient honours out_scale and
SA_FLAG_ADD."""
import numpy as np
import pytest

import paper_1907_04435_amd as sa
from workloads import Span, make_c1, subset_points
from workloads.scenes import Day

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


@pytest.fixture(scope="module")
def small(ctx):
    w = make_c1()
    sub = w.points.take(subset_points(w.points, 3000, 41))
    return w, sub, sa.Scene.from_workload(ctx, w.scene), sa.DevicePoints.from_workload(sub)


def _run(ctx, sc, dp, path, fill=float("nan"), flags=0, m64=False):
    torch = ctx.torch
    c = torch.full((path.n_bins, dp.n), -5, dtype=torch.int32, device="cuda")
    m = torch.full((path.n_bins, dp.n), fill, dtype=torch.float32, device="cuda")
    d = torch.full((path.n_bins, dp.n), fill, dtype=torch.float64, device="cuda") if m64 else None
    sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, c, m, flags=flags, minutes64=d)
    ctx.sync()
    return c.cpu().numpy(), m.cpu().numpy(), (d.cpu().numpy() if m64 else None)


def test_outputs_overwritten_and_added(ctx, small):
    w, sub, sc, dp = small
    days = [Day(2019, 6, 21, -4.0, (480.0, 1080.0)), Day(2019, 6, 22, -4.0, (480.0, 1080.0)),
            Day(2019, 12, 21, -5.0, (540.0, 900.0))]
    contiguous = sa.Path(ctx, sa.sunpath_for_span(Span(40.7, -74.0, days, 5.0, [0, 0, 1]), 30.0))
    interleaved = sa.Path(ctx, sa.sunpath_for_span(Span(40.7, -74.0, days, 5.0, [0, 1, 0]), 30.0))
    c1, m1, d1 = _run(ctx, sc, dp, contiguous, m64=True)
    assert (c1 >= 0).all() and np.isfinite(m1).all() and np.isfinite(d1).all()
    # FP64 minutes: the float minutes before their rounding
    np.testing.assert_array_equal(m1, d1.astype(np.float32))
    c2, m2, _ = _run(ctx, sc, dp, interleaved)
    assert (c2 >= 0).all() and np.isfinite(m2).all()
    # bins [0, 0, 1] vs [0, 1, 0]: day 1 and day 2 swap bins
    per_day = []
    for d in days:
        p = sa.Path(ctx, sa.sunpath_for_span(Span(40.7, -74.0, [d], 5.0), 30.0))
        per_day.append(_run(ctx, sc, dp, p)[:2])
    np.testing.assert_array_equal(c1[0], per_day[0][0][0] + per_day[1][0][0])
    np.testing.assert_array_equal(c2[0], per_day[0][0][0] + per_day[2][0][0])
    np.testing.assert_allclose(m2[1], per_day[1][1][0], atol=1e-3)
    # SA_FLAG_ADD adds to what is there
    c3, m3, _ = _run(ctx, sc, dp, contiguous, fill=1.5, flags=sa.SA_FLAG_ADD)
    np.testing.assert_array_equal(c3, c1 - 5)
    np.testing.assert_allclose(m3, m1 + 1.5, atol=1e-3)
    say(f"  store-once and clear paths agree; mean minutes {m1.mean():.2f}")


def test_device_height_edit(ctx, small):
    import torch
    w, sub, _, dp = small
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    ids = np.array([3, 17, 40, 63], np.int32)
    hh = np.array([120.0, 5.0, 77.5, 200.0], np.float32)
    a = sa.Scene.from_workload(ctx, w.scene)
    a.set_heights(ids, hh)
    b = sa.Scene.from_workload(ctx, w.scene)
    b.set_heights(torch.from_numpy(ids).cuda(), torch.from_numpy(hh).cuda())
    ma = _run(ctx, a, dp, path)[1]
    mb = _run(ctx, b, dp, path)[1]
    np.testing.assert_array_equal(ma, mb)
    assert abs(b.info()["max_height"] - max(float(w.scene.height.max()), 200.0)) < 1e-3
    # a bad entry is skipped and reported by sync; the good ones apply
    b.set_heights(torch.tensor([5, 999], dtype=torch.int32, device="cuda"),
                  torch.tensor([60.0, 10.0], dtype=torch.float32, device="cuda"))
    with pytest.raises(sa.SAError) as e:
        ctx.sync()
    assert e.value.code == -1
    a.set_heights(np.array([5], np.int32), np.array([60.0], np.float32))
    np.testing.assert_array_equal(_run(ctx, a, dp, path)[1], _run(ctx, b, dp, path)[1])


def test_grad_scale_and_add(ctx, small):
    import torch
    w, sub, sc, dp = small
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    g1 = torch.empty(w.scene.n_b, dtype=torch.float32, device="cuda")
    sa.sa_grad_heights(ctx, sc, dp, path, None, g1)
    g2 = torch.full_like(g1, 7.0)
    sa.sa_grad_heights(ctx, sc, dp, path, None, g2, flags=sa.SA_FLAG_ADD, out_scale=1.0 / 60.0)
    g3 = torch.empty_like(g1)
    sa.sa_grad_heights(ctx, sc, dp, path, None, g3)
    ctx.sync()
    a, b, c = (x.cpu().numpy().astype(np.float64) for x in (g1, g2, g3))
    assert (a > 0).sum() > 10
    np.testing.assert_allclose(b, 7.0 + a / 60.0, rtol=1e-6, atol=1e-6)
    # FP64 accumulation with per-wave sums: the same inputs give the same
    # float gradient (the FP64 atomics' order can only move a sum that sits
    # on a float rounding boundary by one unit)
    np.testing.assert_allclose(a, c, rtol=2.5e-7, atol=0)
    assert np.mean(a == c) >= 0.99
