"""GPU adjoint of the accrual form with respect to building heights,
against the oracle's implicit-differentiation gradient, against central
finite differences of the GPU forward, and through torch.autograd."""
import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Scene, Span, make_c1, make_c4, subset_points

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def gpu_grad(ctx, scene, pts, span, seg, dl=None):
    path = sa.Path(ctx, sa.sunpath_for_span(span, seg))
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    import torch
    g = torch.empty(scene.n_b, dtype=torch.float32, device="cuda")
    sa.sa_grad_heights(ctx, sc, dp, path, dl, g)
    ctx.sync()
    return g.cpu().numpy().astype(np.float64)


def test_grad_c1_matches_oracle(ctx, c1):
    sub = c1.points.take(subset_points(c1.points, 512, 31))
    g = gpu_grad(ctx, c1.scene, sub, c1.span, 30.0)
    o = oracle.grad_implicit(c1.scene, sub, oracle.sun_path(c1.span, 30.0))
    say("c1 grad gpu", g[:6].round(4), "oracle", o[:6].round(4))
    big = np.abs(o) > 0.05 * np.abs(o).max()
    rel = np.abs(g - o)[big] / np.abs(o)[big]
    say(f"  rel err max {rel.max():.2e} median {np.median(rel):.2e}; abs err small {np.abs(g - o)[~big].max():.2e}")
    assert rel.max() <= 1e-3
    assert np.abs(g - o)[~big].max() <= 1e-3 * np.abs(o).max()
    assert np.all(g >= -1e-4 * np.abs(o).max())          # taller never shades less


def test_grad_near_vertical_planes(ctx, c1):
    """The small scene at the equator on the equinox: every segment plane is
    within 0.2 degrees of vertical (the steep-plane extreme search, clip
    crossings formed directly in the plane).  Against the oracle."""
    from workloads.scenes import Day
    span = Span(-0.2, -78.5, [Day(2019, 3, 20, -5.0)], 5.0)
    sub = c1.points.take(subset_points(c1.points, 512, 33))
    g = gpu_grad(ctx, c1.scene, sub, span, 30.0)
    o = oracle.grad_implicit(c1.scene, sub, oracle.sun_path(span, 30.0))
    big = np.abs(o) > 0.05 * np.abs(o).max()
    rel = np.abs(g - o)[big] / np.abs(o)[big]
    say(f"equator grad: {big.sum()} buildings, rel err max {rel.max():.2e} median {np.median(rel):.2e}")
    assert big.sum() >= 5
    assert rel.max() <= 1e-3
    assert np.abs(g - o)[~big].max() <= 1e-3 * np.abs(o).max()


def test_grad_weighted_by_upstream(ctx, c1):
    """dl_dmin scales each point-day's contribution linearly."""
    import torch
    sub = c1.points.take(subset_points(c1.points, 256, 32))
    w = np.random.default_rng(3).uniform(0.0, 2.0, (1, sub.n)).astype(np.float32)
    g = gpu_grad(ctx, c1.scene, sub, c1.span, 30.0, torch.from_numpy(w).cuda())
    o = oracle.grad_implicit(c1.scene, sub, oracle.sun_path(c1.span, 30.0), dl=w.astype(np.float64))
    big = np.abs(o) > 0.05 * np.abs(o).max()
    assert (np.abs(g - o)[big] / np.abs(o)[big]).max() <= 1e-3


def test_grad_c4_subset_matches_oracle(ctx):
    """Differentiation scene (5,000 buildings around the park, Mar 20,
    1-minute knots), a 512-point subset of the park: adjoint against the
    oracle's implicit-differentiation gradient for every building."""
    w = make_c4()
    sub = w.points.take(subset_points(w.points, 512, 61))
    g = gpu_grad(ctx, w.scene, sub, w.span, 1.0)
    o = oracle.grad_implicit(w.scene, sub, oracle.sun_path(w.span, 1.0))
    big = np.abs(o) > 1e-3 * np.abs(o).max()
    rel = np.abs(g - o)[big] / np.abs(o)[big]
    k = np.flatnonzero(big)[np.argmax(rel)]
    say(f"c4 subset: {big.sum()} buildings with gradient; rel err max {rel.max():.2e} (building {k}: "
        f"gpu {g[k]:.6g} oracle {o[k]:.6g}, |grad| max {np.abs(o).max():.4g}) median {np.median(rel):.2e} "
        f"p99 {np.quantile(rel, 0.99):.2e}")
    assert np.quantile(rel, 0.99) <= 1e-3 and rel.max() <= 5e-3
    assert np.abs(g - o)[~big].max() <= 1e-3 * np.abs(o).max()


def test_grad_c4_vs_fp64_central_differences(ctx):
    """The GPU adjoint against FP64 central differences of the oracle's
    continuous duration (dh = 0.01 m, heights rounded to float32 so the
    quotient uses the actual step) on a 128-point subset of the park, for
    the six buildings with the largest gradient there: relative agreement
    within 1e-3.  FP64 removes the float32 summation noise that limits
    difference quotients of the GPU forward itself."""
    w = make_c4()
    sub = w.points.take(subset_points(w.points, 128, 63))
    g = gpu_grad(ctx, w.scene, sub, w.span, 1.0)
    path = oracle.sun_path(w.span, 1.0)
    rel = []
    for b in np.argsort(-np.abs(g))[:6]:
        H = float(w.scene.height[b])
        hp, hm = np.float32(H + 0.01), np.float32(H - 0.01)
        lp = oracle.continuous(oracle.with_height(w.scene, int(b), hp), sub, path)["minutes"].sum()
        lm = oracle.continuous(oracle.with_height(w.scene, int(b), hm), sub, path)["minutes"].sum()
        fd = (lp - lm) / float(hp - hm)
        rel.append(abs(fd - g[b]) / abs(g[b]))
        say(f"  building {b}: adjoint {g[b]:.6g}, FP64 central difference {fd:.6g}")
    say(f"c4 adjoint vs FP64 central differences: max rel {max(rel):.2e}")
    assert max(rel) <= 1e-3


def test_grad_c4_vs_finite_differences(ctx):
    """Full differentiation scene (200k park points, 5,000 buildings, Mar
    20, 1-minute knots): central differences with dh = 0.5 m on 64 random
    buildings with a gradient and 8 without, from the forward's FP64
    per-point minutes.

    The loss is a sum over points of piecewise smooth functions of a
    height; a point's function has a kink where a roof edge's crossing
    meets a vertex or another occluder's interval end.  Over +-0.5 m some
    points of every building kink, so the total's quotient is the mean of a
    derivative that changes across the bracket (by ~2 %), not the
    derivative at H.  Kinks are therefore separated per point: a point is
    smooth over the bracket when its own central differences at 0.5, 0.25
    and 0.125 m agree (within 2e-3 relative, or 1e-6 min/m) and its forward
    and backward differences at 0.125 m agree within 5 % (central
    differences cannot see a kink right at H: they average its two sides
    at every step, while the adjoint gives the current side); the adjoint
    is taken with dl_dmin = 1 on the smooth points and 0 elsewhere, and
    must agree with the smooth points' summed quotient within 1e-3 relative
    for every building that has smooth points (at least 48 of the 64).
    Buildings whose every affected point kinks within the bracket, the
    kinked points' share and their part of the total quotient are
    reported.  As a whole-loss check, the quotient equals the adjoint
    averaged over the bracket (midpoint rule, 32 heights): median relative
    difference <= 5e-4.  Zero-gradient buildings give zero quotients."""
    import torch
    w = make_c4()
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 1.0))
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    g = torch.empty(w.scene.n_b, dtype=torch.float32, device="cuda")
    sa.sa_grad_heights(ctx, sc, dp, path, None, g)
    ctx.sync()
    gh = g.cpu().numpy().astype(np.float64)

    def minutes(b, h):
        sc.set_heights(np.array([b], np.int32), np.array([h], np.float32))
        m = torch.empty((1, w.points.n), dtype=torch.float64, device="cuda")
        sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, minutes64=m)
        return m[0]

    def adjoint(b, h, dl=None):
        sc.set_heights(np.array([b], np.int32), np.array([h], np.float32))
        sa.sa_grad_heights(ctx, sc, dp, path, dl, g)
        return float(g[b].item())

    rng = np.random.default_rng(44)
    pos = np.flatnonzero(gh > 1e-3 * gh.max())
    zero = np.flatnonzero(gh == 0)
    dh, nq = 0.5, 32
    rows = []
    for b in list(rng.choice(pos, 64, replace=False)) + list(rng.choice(zero, 8, replace=False)):
        H = float(w.scene.height[b])
        fd = {}
        for step in (dh, dh / 2, dh / 4):
            hp, hm = np.float32(H + step), np.float32(H - step)
            fd[step] = (minutes(b, hp) - minutes(b, hm)) / float(hp - hm)
        total = float(fd[dh].sum())
        if gh[b] == 0:
            minutes(b, np.float32(H))
            assert abs(total) <= 1e-4 * gh.max(), (b, total)
            continue
        a, m2, m4 = fd[dh], fd[dh / 2], fd[dh / 4]
        tol = lambda x, y, r: (x - y).abs() <= r * torch.maximum(x.abs(), y.abs()) + 1e-6
        mid = minutes(b, np.float32(H))
        hq, hr = np.float32(H + dh / 4), np.float32(H - dh / 4)
        fwd = (minutes(b, hq) - mid) / float(hq - np.float32(H))
        bwd = (mid - minutes(b, hr)) / float(np.float32(H) - hr)
        smooth = tol(a, m2, 2e-3) & tol(a, m4, 2e-3) & tol(m2, m4, 2e-3) & tol(fwd, bwd, 5e-2)
        fd_s = float((a * smooth).sum())
        g_s = adjoint(b, np.float32(H), smooth.float().reshape(1, -1).contiguous())
        hp, hm = np.float32(H + dh), np.float32(H - dh)
        nodes = [np.float32(float(hm) + (float(hp) - float(hm)) * (k + 0.5) / nq) for k in range(nq)]
        g_mean = float(np.mean([adjoint(b, h) for h in nodes]))
        minutes(b, np.float32(H))
        affected = int((a != 0).sum())
        rows.append((b, gh[b], total, fd_s, g_s, g_mean, affected, int(((a != 0) & ~smooth).sum()),
                     int(((a != 0) & smooth).sum())))
    r = np.array(rows, dtype=np.float64)
    has = r[:, 8] > 0                      # buildings with smooth affected points
    rel_smooth = np.abs(r[has, 3] - r[has, 4]) / np.abs(r[has, 4])
    rel_mean = np.abs(r[:, 2] - r[:, 5]) / np.abs(r[:, 2])
    rel_at_h = np.abs(r[:, 2] - r[:, 1]) / np.abs(r[:, 1])
    kink_pts = r[:, 7] / np.maximum(r[:, 6], 1)
    kink_fd = np.abs(r[:, 2] - r[:, 3]) / np.abs(r[:, 2])
    say(f"c4 dh=0.5 on {len(r)} buildings: {int(has.sum())} with smooth points, their FD vs adjoint: max rel "
        f"{rel_smooth.max():.2e}, median {np.median(rel_smooth):.2e}, share within 1e-3 "
        f"{np.mean(rel_smooth <= 1e-3):.0%}; {int((~has).sum())} with every affected point kinked; kinked "
        f"points per building: median {np.median(kink_pts):.1%} of affected points, {np.median(kink_fd):.1%} "
        f"of the quotient; whole loss: FD vs bracket-mean adjoint median {np.median(rel_mean):.2e} (max "
        f"{rel_mean.max():.2e}), FD vs adjoint at H median {np.median(rel_at_h):.2e}")
    assert has.sum() >= 48
    assert np.all(rel_smooth <= 1e-3)
    assert np.median(rel_mean) <= 5e-4


def test_autograd_function(ctx, c1):
    import torch
    sub = c1.points.take(subset_points(c1.points, 300, 33))
    path = sa.Path(ctx, sa.sunpath_for_span(c1.span, 30.0))
    sc = sa.Scene.from_workload(ctx, c1.scene)
    dp = sa.DevicePoints.from_workload(sub)
    H = torch.tensor(c1.scene.height, dtype=torch.float32, device="cuda", requires_grad=True)
    fn = sa.shadow_minutes_fn()
    m = fn.apply(H, ctx, sc, dp, path)
    (m * 2.0).sum().backward()
    o = oracle.grad_implicit(c1.scene, sub, oracle.sun_path(c1.span, 30.0))
    big = np.abs(o) > 0.05 * np.abs(o).max()
    gh = H.grad.cpu().numpy()
    assert (np.abs(gh - 2 * o)[big] / np.abs(2 * o)[big]).max() <= 1e-3


def test_grad_over_several_view_launches(ctx):
    """Mar 20 and Jun 21 at 1-minute knots on the differentiation scene:
    about 1,600 segments, more than one launch's budget of per-segment node
    views (~840 segments for 5,000 buildings), so the adjoint runs in two
    launches, the second starting inside Jun 21.  The loss sums over days,
    so its gradient equals the sum of the single-day gradients."""
    from workloads.scenes import Day, _nyc_tz
    import datetime as dt
    w = make_c4()
    sub = w.points.take(subset_points(w.points, 20_000, 62))
    days = [Day(d.year, d.month, d.day, _nyc_tz(d)) for d in (dt.date(2019, 3, 20), dt.date(2019, 6, 21))]
    both = Span(w.span.lat, w.span.lon, days, 1.0, [0, 0])
    sp = sa.sunpath_for_span(both, 1.0)
    assert (len(sp.knot_t) - sp.n_days) * (w.scene.n_b - 1) * 64 > 256 << 20
    g = gpu_grad(ctx, w.scene, sub, both, 1.0)
    parts = [gpu_grad(ctx, w.scene, sub, Span(w.span.lat, w.span.lon, [d], 1.0), 1.0) for d in days]
    ref = parts[0] + parts[1]
    d = np.abs(g - ref)
    say(f"two-day gradient: max |both - sum of days| {d.max():.3e} of max |grad| {np.abs(ref).max():.4g}")
    assert (np.abs(ref) > 0).sum() > 50
    assert d.max() <= 1e-4 * np.abs(ref).max()
