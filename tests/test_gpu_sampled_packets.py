"""The sampled form's packet layouts compute the same predicate per (point,
instant): 64 / k points x k consecutive instants for k = 4, 8, 16 (counts,
minutes and the continuous shadow, whenever every work unit lies in one bin)
and 64 points x 1 instant (with bit vectors, or when bins interleave).
Counts are equal, minutes equal to float rounding (the sums are grouped
differently), the continuous shadow equals the definition applied to the
other layout's bits; and the counts of the 8 x 8 layout agree with the
oracle outside the silhouette band."""
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


def both_layouts(ctx, scene, pts, span, inst=8):
    """(counts, minutes, longest) without bit vectors (packets of ``inst``
    instants where units lie in one bin) and (counts, minutes, longest,
    bits) with them (64 x 1 packets)."""
    import torch
    ctx.set_launch(sampled_instants_per_packet=inst)
    sp = sa.sunpath_for_span(span, 30.0)   # knots do not matter to the sampled form
    path = sa.Path(ctx, sp)
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    B, K = path.n_bins, sp.n_samples
    out = []
    for bits in (False, True):
        c = torch.empty((B, dp.n), dtype=torch.int32, device="cuda")
        m = torch.empty((B, dp.n), dtype=torch.float32, device="cuda")
        L = torch.empty((B, dp.n), dtype=torch.float32, device="cuda")
        b = torch.empty(((K + 31) // 32, dp.n), dtype=torch.int32, device="cuda") if bits else None
        sa.sa_accumulate(ctx, sc, dp, path, sa.SA_SAMPLED, c, m, b, longest=L)
        ctx.sync()
        r = [c.cpu().numpy(), m.cpu().numpy().astype(np.float64), L.cpu().numpy().astype(np.float64)]
        if bits:
            r.append(unpack_words(b.cpu().numpy().view(np.uint32).T, K))
        out.append(r)
    ctx.set_launch()
    return out, sp


CASES = {
    # three days, a bin each (the block scene's own span)
    "days": lambda w: w.span,
    # one bin over three days: a single run of instants
    "one_bin": lambda w: Span(w.span.lat, w.span.lon, w.span.days, w.span.step_min, [0, 0, 0]),
    # bins that interleave: the 64 x 1 layout for both calls
    "interleaved": lambda w: Span(w.span.lat, w.span.lon, w.span.days, w.span.step_min, [0, 1, 0]),
}


@pytest.mark.parametrize("inst", [4, 8, 16])
@pytest.mark.parametrize("case", sorted(CASES))
def test_layouts_agree(ctx, case, inst):
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sub = w.points.take(subset_points(w.points, 1001, 17))   # ragged: not a multiple of 4, 8, 16 or 64
    span = CASES[case](w)
    ((c8, m8, l8), (c1, m1, l1, bits)), sp = both_layouts(ctx, w.scene, sub, span, inst)
    np.testing.assert_array_equal(c8, c1)
    dm = np.abs(m8 - m1)
    say(f"{case}, {inst} instants per packet: counts equal over {sub.n} points x {sp.n_samples} instants; "
        f"max |minutes diff| {dm.max():.2e}")
    assert np.all(dm <= 1e-5 * np.abs(m1) + 1e-3)
    ref = oracle.longest_sampled(bits.astype(bool), oracle.sun_path(span))
    np.testing.assert_allclose(l8, ref, rtol=1e-5, atol=1e-3)
    np.testing.assert_allclose(l1, ref, rtol=1e-5, atol=1e-3)
    assert (c8 > 0).mean() > 0.3


def test_packets_against_oracle(ctx):
    """8 x 8 packets on the block scene (two days, a bin each) against the
    oracle: counts exact wherever no instant is in the silhouette band, and
    otherwise within the band's count."""
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sub = w.points.take(subset_points(w.points, 257, 23))
    days = [w.span.days[1], w.span.days[2]]
    span = Span(w.span.lat, w.span.lon, days, w.span.step_min)
    ((c8, m8, l8), _), sp = both_layouts(ctx, w.scene, sub, span)
    op = oracle.sun_path(span)
    o = oracle.sampled(w.scene, sub, op, bits=True, amb=True)
    amb = o["amb"].astype(bool)
    ob = unpack_words(o["bits"], len(op.w)).astype(bool)
    na = np.stack([amb[:, op.sample_day == d].sum(1) for d in range(len(days))])
    oc = np.stack([ob[:, op.sample_day == d].sum(1) for d in range(len(days))])
    dc = np.abs(c8 - oc)
    say(f"8 x 8 packets vs oracle: {int((na > 0).sum())} of {na.size} point-days touch the band; "
        f"max |count diff| {int(dc.max())}")
    assert np.all(dc <= na)
    np.testing.assert_array_equal(c8[na == 0], oc[na == 0])
