"""The sampled form's two queue kernels compute the same predicate per
(point, instant) for every packet shape (64 / k points x k consecutive
instants, k = 1 ... 16): the one that adds a walk's hits to per-point sums
(counts and minutes of units in one bin) and the one that sets them in a
bitmap replayed in time order (bit vectors, the continuous shadow, bins
that interleave), whether its units are bin runs or whole tiles.  Counts
are equal, minutes equal to float rounding (the sums are grouped
differently), the continuous shadow equals the definition applied to the
bit vectors; and the counts agree with the oracle outside the silhouette
band."""
import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Span, make_c2, subset_points

from gpu_util import say, unpack_words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def layouts(ctx, scene, pts, span, inst=8):
    """Per call, with packets of ``inst`` instants: "sums" (counts and
    minutes only: per-point sums where units lie in one bin), "runs" (with
    the continuous shadow: the replayed bitmap, units of one bin run) and
    "bits" (with bit vectors: the replayed bitmap, a whole tile per unit),
    each a dict of numpy arrays."""
    import torch
    ctx.set_launch(sampled_instants_per_packet=inst)
    sp = sa.sunpath_for_span(span, 30.0)   # knots do not matter to the sampled form
    path = sa.Path(ctx, sp)
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    B, K = path.n_bins, sp.n_samples
    out = {}
    for name, runs, bits in (("sums", False, False), ("runs", True, False), ("bits", True, True)):
        c = torch.empty((B, dp.n), dtype=torch.int32, device="cuda")
        m = torch.empty((B, dp.n), dtype=torch.float32, device="cuda")
        L = torch.empty((B, dp.n), dtype=torch.float32, device="cuda") if runs else None
        b = torch.empty(((K + 31) // 32, dp.n), dtype=torch.int32, device="cuda") if bits else None
        sa.sa_accumulate(ctx, sc, dp, path, sa.SA_SAMPLED, c, m, b, longest=L)
        ctx.sync()
        r = {"counts": c.cpu().numpy(), "minutes": m.cpu().numpy().astype(np.float64)}
        if runs:
            r["longest"] = L.cpu().numpy().astype(np.float64)
        if bits:
            r["bits"] = unpack_words(b.cpu().numpy().view(np.uint32).T, K)
        out[name] = r
    ctx.set_launch()
    return out, sp


CASES = {
    # three days, a bin each (the block scene's own span)
    "days": lambda w: w.span,
    # one bin over three days: a single run of instants
    "one_bin": lambda w: Span(w.span.lat, w.span.lon, w.span.days, w.span.step_min, [0, 0, 0]),
    # bins that interleave: units span bins (the bitmap kernel for every call)
    "interleaved": lambda w: Span(w.span.lat, w.span.lon, w.span.days, w.span.step_min, [0, 1, 0]),
}


@pytest.mark.parametrize("inst", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("case", sorted(CASES))
def test_layouts_agree(ctx, case, inst):
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sub = w.points.take(subset_points(w.points, 1001, 17))   # ragged: not a multiple of 4, 8, 16 or 64
    span = CASES[case](w)
    r, sp = layouts(ctx, w.scene, sub, span, inst)
    ref = r["bits"]
    for name in ("sums", "runs"):
        np.testing.assert_array_equal(r[name]["counts"], ref["counts"])
        dm = np.abs(r[name]["minutes"] - ref["minutes"])
        say(f"{case}, {inst} instants per packet, {name}: counts equal over {sub.n} points x {sp.n_samples} "
            f"instants; max |minutes diff| {dm.max():.2e}")
        assert np.all(dm <= 1e-5 * np.abs(ref["minutes"]) + 1e-3)
    runs = oracle.longest_sampled(ref["bits"].astype(bool), oracle.sun_path(span))
    np.testing.assert_allclose(r["runs"]["longest"], runs, rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(ref["longest"], runs, rtol=1e-5, atol=1e-3)
    assert (ref["counts"] > 0).mean() > 0.3


def test_layouts_against_oracle(ctx):
    """The block scene over two days (a bin each) against the oracle:
    counts of every layout exact wherever no instant is in the silhouette
    band, and otherwise within the band's count."""
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sub = w.points.take(subset_points(w.points, 257, 23))
    days = [w.span.days[1], w.span.days[2]]
    span = Span(w.span.lat, w.span.lon, days, w.span.step_min)
    r, sp = layouts(ctx, w.scene, sub, span)
    op = oracle.sun_path(span)
    o = oracle.sampled(w.scene, sub, op, bits=True, amb=True)
    amb = o["amb"].astype(bool)
    ob = unpack_words(o["bits"], len(op.w)).astype(bool)
    na = np.stack([amb[:, op.sample_day == d].sum(1) for d in range(len(days))])
    oc = np.stack([ob[:, op.sample_day == d].sum(1) for d in range(len(days))])
    for name in ("sums", "runs", "bits"):
        dc = np.abs(r[name]["counts"] - oc)
        say(f"{name} vs oracle: {int((na > 0).sum())} of {na.size} point-days touch the band; "
            f"max |count diff| {int(dc.max())}")
        assert np.all(dc <= na)
        np.testing.assert_array_equal(r[name]["counts"][na == 0], oc[na == 0])


@pytest.mark.parametrize("inst", [1, 4, 16])
def test_queue_on_tiny_and_ragged_sets(ctx, c1, inst):
    """Both queue kernels on point sets of 1, 3, 63, 65 and 200 points of
    the small scene (a single partial group, partial tiles, several tiles),
    on one building and on an empty scene: equal counts in every call, equal
    to the oracle's outside the silhouette band, and no shadow (no bit set)
    without buildings."""
    from workloads import Scene
    op = oracle.sun_path(c1.span)
    one = c1.scene.subset(np.array([5]))
    empty = Scene(np.zeros(1, np.int32), np.zeros((0, 2), np.float32), np.zeros(0, np.float32))
    for n in (1, 3, 63, 65, 200):
        sub = c1.points.take(np.arange(7, 7 + n * 13, 13))
        for scene in (c1.scene, one):
            r, _ = layouts(ctx, scene, sub, c1.span, inst)
            for name in ("sums", "runs"):
                np.testing.assert_array_equal(r[name]["counts"], r["bits"]["counts"])
                assert np.abs(r[name]["minutes"] - r["bits"]["minutes"]).max() <= 1e-3
            np.testing.assert_array_equal(r["bits"]["bits"].sum(1), r["bits"]["counts"].sum(0))
        o = oracle.sampled(c1.scene, sub, op, amb=True)
        r, _ = layouts(ctx, c1.scene, sub, c1.span, inst)
        dc = np.abs(r["sums"]["counts"].sum(0) - o["counts"].sum(0))
        assert np.all(dc <= o["amb"].sum(1))
        r, _ = layouts(ctx, empty, sub, c1.span, inst)
        for name in ("sums", "runs", "bits"):
            assert np.all(r[name]["counts"] == 0) and np.all(r[name]["minutes"] == 0)
        assert not r["bits"]["bits"].any() and np.all(r["runs"]["longest"] == 0)
