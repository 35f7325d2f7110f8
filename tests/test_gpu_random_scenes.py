"""GPU parity on seeded random scenes: convex footprints of 3 to 12
vertices at random orientations and aspect ratios (one per cell of a
jittered grid, so footprints never overlap), heights from 5 to 200 m,
ground points anywhere (some under roofs) and facade points on random
walls, at random sites (60 S to 60 N) and dates.  Both forms against the
oracle with the bars of the other parity tests, and the height adjoint
against the oracle's implicit derivative."""
import datetime as dt

import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import Points, Scene, Span
from workloads.scenes import Day

from gpu_util import check_sampled, run_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def random_workload(seed, cells=6, cell=60.0, n_ground=384, n_facade=192):
    rng = np.random.default_rng(1000 + seed)
    offs, xy, hs = [0], [], []
    for i in range(cells):
        for j in range(cells):
            m = int(rng.integers(3, 13))
            ang = np.sort(rng.uniform(0, 2 * np.pi, m))
            ang = np.unique(np.round(ang, 3))
            if len(ang) < 3:
                ang = np.array([0.0, 2.1, 4.2])
            rx, ry = rng.uniform(8, 25), rng.uniform(8, 25)
            rot = rng.uniform(0, np.pi)
            c = np.array([(i + 0.5) * cell, (j + 0.5) * cell]) + rng.uniform(-3, 3, 2)
            p = np.stack([rx * np.cos(ang), ry * np.sin(ang)], 1)
            p = p @ np.array([[np.cos(rot), np.sin(rot)], [-np.sin(rot), np.cos(rot)]]) + c
            xy.append(p.astype(np.float32))
            offs.append(offs[-1] + len(p))
            hs.append(rng.uniform(5, 200))
    scene = Scene(np.array(offs, np.int32), np.concatenate(xy), np.array(hs, np.float32))
    ext = cells * cell
    gx, gy = rng.uniform(0, ext, n_ground), rng.uniform(0, ext, n_ground)
    fx, fy, fz, fnx, fny, fo = [], [], [], [], [], []
    for _ in range(n_facade):
        b = int(rng.integers(0, scene.n_b))
        v = scene.xy[scene.vert_off[b]:scene.vert_off[b + 1]].astype(np.float64)
        e = int(rng.integers(0, len(v)))
        a, bb = v[e], v[(e + 1) % len(v)]
        f = rng.uniform(0.1, 0.9)
        q = a + f * (bb - a)
        n = np.array([bb[1] - a[1], a[0] - bb[0]])
        n /= np.linalg.norm(n)
        fx.append(q[0]); fy.append(q[1]); fz.append(rng.uniform(0.5, scene.height[b] - 0.5))
        fnx.append(n[0]); fny.append(n[1]); fo.append(b)
    f32 = lambda a: np.asarray(a, np.float32)
    pts = Points(f32(np.concatenate([gx, fx])), f32(np.concatenate([gy, fy])),
                 f32(np.concatenate([np.zeros(n_ground), fz])), f32(np.concatenate([np.zeros(n_ground), fnx])),
                 f32(np.concatenate([np.zeros(n_ground), fny])),
                 np.concatenate([np.full(n_ground, -1), fo]).astype(np.int32))
    lat = float(rng.uniform(-60, 60))
    day = dt.date(2019, 1, 1) + dt.timedelta(days=int(rng.integers(0, 365)))
    lon = float(rng.uniform(-180, 180))
    # civil time near solar time (the zone of the longitude), so a day's
    # daylight falls within one civil day
    span = Span(lat, lon, [Day(day.year, day.month, day.day, float(round(lon / 15.0)))], 5.0)
    return scene, pts, span


@pytest.mark.parametrize("seed", range(6))
def test_random_scene_parity(ctx, seed):
    scene, pts, span = random_workload(seed)
    say(f"seed {seed}: lat {span.lat:.1f}, {span.days[0].month}/{span.days[0].day}, {scene.n_b} prisms, "
        f"{pts.n} points")
    g = run_lib(ctx, scene, pts, span, sa.SA_SAMPLED, bits=True)
    op = oracle.sun_path(span)
    o = oracle.sampled(scene, pts, op, bits=True, amb=True)
    frac, n_mism = check_sampled(g, o, op.w)
    say(f"  sampled: {g['K']} instants, ambiguous {frac:.2e}, mismatched bits {n_mism}")
    # the bar: bit-exact outside the silhouette band (check_sampled), and at
    # most 1e-4 of the pairs actually excused by it (measured: none on every
    # seed).  How many pairs the band holds is the scene's and the sky's, not
    # the kernel's: near the equator more roof edges run along the sun's
    # path, 5.9e-4 of the pairs on one seed here; it is bounded loosely.
    assert n_mism <= 1e-4 * g["bits"].size and frac <= 1e-3
    for seg in (30.0, 60.0):
        ga = run_lib(ctx, scene, pts, span, sa.SA_ACCRUAL, seg_min=seg)
        oa = oracle.continuous(scene, pts, oracle.sun_path(span, seg))
        d = np.abs(ga["minutes"] - oa["minutes"]).ravel()
        say(f"  accrual L={seg}: |A-D_L| mean {d.mean():.2e} p99.9 {np.quantile(d, 0.999):.2e} max {d.max():.2e}")
        assert np.quantile(d, 0.999) <= 0.01 and d.mean() <= 1e-3 and d.max() <= 0.5
    assert (oa["minutes"] > 1.0).mean() > 0.1          # the scene shadows a fair share of the points


@pytest.mark.parametrize("seed", [0, 3])
def test_random_scene_gradient(ctx, seed):
    import torch
    scene, pts, span = random_workload(seed)
    path = sa.Path(ctx, sa.sunpath_for_span(span, 30.0))
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    gd = torch.empty(scene.n_b, dtype=torch.float32, device="cuda")
    sa.sa_grad_heights(ctx, sc, dp, path, None, gd)
    ctx.sync()
    g = gd.cpu().numpy().astype(np.float64)
    o = oracle.grad_implicit(scene, pts, oracle.sun_path(span, 30.0))
    big = np.abs(o) > 0.05 * np.abs(o).max()
    rel = np.abs(g - o)[big] / np.abs(o)[big]
    say(f"seed {seed} gradient: {big.sum()} buildings, rel err max {rel.max():.2e}")
    assert big.sum() >= 3
    assert rel.max() <= 1e-3
    assert np.abs(g - o)[~big].max() <= 1e-3 * np.abs(o).max()
