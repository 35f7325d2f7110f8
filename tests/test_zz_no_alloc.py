"""sa_accumulate_noalloc (the entry point for callers that cannot allocate)
against sa_accumulate, through the C ABI: two calls in a row, the second
on a smaller input, with outputs pre-filled with garbage.  Counts and bit
vectors must be equal; minutes and the continuous shadow within 1e-3 min
(the fixed scratch splits the block scene's path into more launches, whose
float partial sums are added in another grouping).  A path one of whose
days does not fit the fixed scratch is refused before any work."""
import numpy as np
import pytest

import paper_1907_04435_amd as sa
from workloads import make_c1, make_c2, subset_points

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def outputs(ctx, path, n, bits=False, longest=False):
    torch = ctx.torch
    o = {"counts": torch.full((path.n_bins, n), -7, dtype=torch.int32, device="cuda"),
         "minutes": torch.full((path.n_bins, n), float("nan"), dtype=torch.float32, device="cuda")}
    o["bits"] = torch.full(((path.n_samples + 31) // 32, n), -1, dtype=torch.int32, device="cuda") if bits else None
    o["longest"] = torch.full((path.n_bins, n), float("nan"), dtype=torch.float32, device="cuda") if longest else None
    return o


def call(fn, ctx, scene, dp, path, mode, o):
    fn(ctx, scene, dp, path, mode, o["counts"], o["minutes"], o["bits"], longest=o["longest"])


def host(o):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in o.items()}


def compare(a, b, label):
    np.testing.assert_array_equal(a["counts"], b["counts"])
    assert np.isfinite(b["minutes"]).all()
    d = np.abs(a["minutes"] - b["minutes"]).max()
    say(f"  {label}: counts equal, max |minutes diff| {d:.2e}")
    assert d <= 1e-3
    if a["bits"] is not None:
        np.testing.assert_array_equal(a["bits"], b["bits"])
    if a["longest"] is not None:
        assert np.isfinite(b["longest"]).all()
        assert np.abs(a["longest"] - b["longest"]).max() <= 1e-3


def test_noalloc_matches_accumulate_two_calls(ctx):
    # first input: the block scene (20,000 prisms: the fixed scratch holds
    # the views of 52 of its 73 segments, so the call runs two launches),
    # 30,000 points over three days, accrual form with the continuous shadow
    w = make_c2(n_ground=15_000, n_facade=15_000)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    dp = sa.DevicePoints.from_workload(w.points)
    # second, smaller input: the small scene, 2,000 points, both forms
    w1 = make_c1()
    sub1 = w1.points.take(subset_points(w1.points, 2000, 3))
    sc1 = sa.Scene.from_workload(ctx, w1.scene)
    path1 = sa.Path(ctx, sa.sunpath_for_span(w1.span, 30.0))
    dp1 = sa.DevicePoints.from_workload(sub1)
    say("no-alloc: references with sa_accumulate")
    ref_a = outputs(ctx, path, dp.n, longest=True)
    call(sa.sa_accumulate, ctx, sc, dp, path, sa.SA_ACCRUAL, ref_a)
    ref_b = outputs(ctx, path1, dp1.n)
    call(sa.sa_accumulate, ctx, sc1, dp1, path1, sa.SA_ACCRUAL, ref_b)
    ref_c = outputs(ctx, path1, dp1.n, bits=True)
    call(sa.sa_accumulate, ctx, sc1, dp1, path1, sa.SA_SAMPLED, ref_c)
    ref_d = outputs(ctx, path, dp.n)
    call(sa.sa_accumulate, ctx, sc, dp, path, sa.SA_ACCRUAL, ref_d)
    ctx.sync()
    say("no-alloc: two calls in a row, the second smaller")
    got_a = outputs(ctx, path, dp.n, longest=True)
    call(sa.sa_accumulate_noalloc, ctx, sc, dp, path, sa.SA_ACCRUAL, got_a)
    got_b = outputs(ctx, path1, dp1.n)
    call(sa.sa_accumulate_noalloc, ctx, sc1, dp1, path1, sa.SA_ACCRUAL, got_b)
    got_c = outputs(ctx, path1, dp1.n, bits=True)
    call(sa.sa_accumulate_noalloc, ctx, sc1, dp1, path1, sa.SA_SAMPLED, got_c)
    ctx.sync()
    compare(host(ref_a), host(got_a), "block scene, accrual + continuous shadow")
    compare(host(ref_b), host(got_b), "small scene, accrual")
    compare(host(ref_c), host(got_c), "small scene, sampled")
    # and again on the first input, after the smaller call changed the
    # scratch: without the continuous shadow the 73 segments run as 52 + 21,
    # splitting Jun 21's bin over two launches
    got_a2 = outputs(ctx, path, dp.n, longest=True)
    call(sa.sa_accumulate_noalloc, ctx, sc, dp, path, sa.SA_ACCRUAL, got_a2)
    got_d = outputs(ctx, path, dp.n)
    call(sa.sa_accumulate_noalloc, ctx, sc, dp, path, sa.SA_ACCRUAL, got_d)
    ctx.sync()
    compare(host(ref_a), host(got_a2), "block scene again")
    compare(host(ref_d), host(got_d), "block scene, accrual in two launches")


def test_noalloc_refuses_a_day_beyond_the_fixed_scratch(ctx):
    """With the continuous shadow a launch must hold a whole day: 1-minute
    knots on the block scene need 895 segments of views for Jun 21, more
    than the fixed array holds, so the call is refused (CAPACITY) and the
    outputs are left untouched."""
    w = make_c2(n_ground=1000, n_facade=0)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 1.0))
    dp = sa.DevicePoints.from_workload(w.points)
    o = outputs(ctx, path, dp.n, longest=True)
    with pytest.raises(sa.SAError) as e:
        call(sa.sa_accumulate_noalloc, ctx, sc, dp, path, sa.SA_ACCRUAL, o)
    assert e.value.code == -3
    ctx.sync()
    assert (o["counts"].cpu().numpy() == -7).all()
