"""The context's launch choices (sa_set_launch, set by the autotuner)
change speed only: accrual counts are equal and minutes equal to float
rounding whatever the segments per launch, and batched counts are equal
whatever the grid size and the tiles a wave takes per grab.  Bad values
are refused."""
import numpy as np
import pytest

import paper_1907_04435_amd as sa
from workloads import make_c2, make_c3

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def test_accrual_segments_per_launch(ctx):
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    out = {}
    for per in (0, 7, 1):
        ctx.set_launch(accrual_segments_per_launch=per)
        c, m, _ = sa.accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL)
        ctx.sync()
        out[per] = (c.cpu().numpy(), m.cpu().numpy())
    ctx.set_launch()
    for per in (7, 1):
        np.testing.assert_array_equal(out[per][0], out[0][0])
        d = np.abs(out[per][1] - out[0][1]).max()
        say(f"  {per} segments per launch: counts equal, max |minutes diff| {d:.2e}")
        assert d <= 1e-3


def test_tile_grid_blocks(ctx):
    """The persistent accrual launch at any size -- one block, blocks not a
    multiple of the eight XCDs, more blocks than units -- gives the same
    counts and minutes (each (tile, bin) unit is computed by one wave
    whichever wave takes it), also with bins that interleave (one part
    per tile) and with several launches per path."""
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    span = w.span
    paths = {"days": sa.Path(ctx, sa.sunpath_for_span(span, 30.0))}
    inter = type(span)(span.lat, span.lon, span.days, span.step_min, [0, 1, 0])
    paths["interleaved bins"] = sa.Path(ctx, sa.sunpath_for_span(inter, 30.0))
    for name, path in paths.items():
        res = {}
        for gb, per in ((0, 0), (1, 0), (13, 0), (100_000, 0), (0, 5)):
            ctx.set_launch(tile_grid_blocks=gb, accrual_segments_per_launch=per)
            c, m, _ = sa.accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL)
            ctx.sync()
            res[(gb, per)] = (c.cpu().numpy(), m.cpu().numpy())
        ctx.set_launch()
        c0, m0 = res[(0, 0)]
        assert c0.sum() > 0
        for key, (c, m) in res.items():
            np.testing.assert_array_equal(c, c0)
            d = np.abs(m - m0).max()
            say(f"  {name}: grid {key[0]}, {key[1]} segments per launch: counts equal, max |minutes diff| {d:.2e}")
            assert d <= 1e-3


def test_batched_grid_and_grab(ctx):
    import torch
    w = make_c3(n_var=12, n_per_var=3000)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    dp = sa.DevicePoints.from_workload(w.points)
    ids = torch.from_numpy(w.extra["var_ids"].astype(np.int32)).cuda()
    hh = torch.from_numpy(w.extra["var_h"].astype(np.float32)).cuda()
    off = torch.from_numpy(w.extra["var_off"].astype(np.int64)).cuda()
    res = []
    for gb, grab in ((2048, 1), (64, 3), (300, 8), (1, 1)):
        ctx.set_launch(batched_grid_blocks=gb, batched_tiles_per_grab=grab)
        c = torch.empty((path.n_bins, dp.n), dtype=torch.int32, device="cuda")
        m = torch.empty((path.n_bins, dp.n), dtype=torch.float32, device="cuda")
        sa.sa_accumulate_batched(ctx, sc, ids, hh, dp, off, path, c, m)
        ctx.sync()
        res.append((c.cpu().numpy(), m.cpu().numpy()))
    ctx.set_launch()
    for c, m in res[1:]:
        np.testing.assert_array_equal(c, res[0][0])
        assert np.abs(m - res[0][1]).max() <= 1e-3


def test_accrual_waves_per_simd(ctx):
    """The accrual kernel's occupancy variants (6, 7, 8 waves per SIMD) give
    equal counts and minutes equal to the last bits (the same arithmetic in
    other registers)."""
    w = make_c2(n_ground=20_000, n_facade=20_000)
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    out = {}
    for occ in (8, 7, 6):
        ctx.set_launch(accrual_waves_per_simd=occ)
        assert ctx.get_launch()["accrual_waves_per_simd"] == occ
        c, m, _ = sa.accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL)
        ctx.sync()
        out[occ] = (c.cpu().numpy(), m.cpu().numpy())
    ctx.set_launch()
    for occ in (7, 6):
        np.testing.assert_array_equal(out[occ][0], out[8][0])
        assert np.abs(out[occ][1] - out[8][1]).max() <= 1e-3


def test_bad_launch_values(ctx):
    with pytest.raises(sa.SAError):
        ctx.set_launch(accrual_segments_per_launch=-1)
    with pytest.raises(sa.SAError):
        ctx.set_launch(batched_tiles_per_grab=5000)
    with pytest.raises(sa.SAError):
        ctx.set_launch(tile_grid_blocks=-3)
    with pytest.raises(sa.SAError):
        ctx.set_launch(accrual_waves_per_simd=5)
    with pytest.raises(sa.SAError):
        ctx.set_launch(sampled_instants_per_packet=6)
    with pytest.raises(sa.SAError):
        ctx.set_launch(sampled_instants_per_packet=32)
    assert ctx.get_launch()["batched_tiles_per_grab"] == 1


def test_few_tiles_pieces_deterministic(ctx):
    """On few tiles the accrual form cuts each bin's run into pieces and adds
    the pieces' sums in a fixed order: two calls give bit-identical counts,
    minutes and FP64 minutes, and they equal whole runs per unit (a
    one-block launch) up to float rounding."""
    import torch
    w = make_c2(n_ground=3_001, n_facade=3_000)    # odd: the FP64 sums start 256-byte aligned
    sc = sa.Scene.from_workload(ctx, w.scene)
    dp = sa.DevicePoints.from_workload(w.points)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 30.0))
    res = []
    for gb in (0, 0, 1):
        ctx.set_launch(tile_grid_blocks=gb)
        c = torch.empty((path.n_bins, dp.n), dtype=torch.int32, device="cuda")
        m = torch.empty((path.n_bins, dp.n), dtype=torch.float32, device="cuda")
        m64 = torch.empty((path.n_bins, dp.n), dtype=torch.float64, device="cuda")
        sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, c, m, minutes64=m64)
        ctx.sync()
        res.append((c.cpu().numpy(), m.cpu().numpy(), m64.cpu().numpy()))
    ctx.set_launch()
    for a, b in zip(res[0], res[1]):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(res[0][0], res[2][0])
    d = np.abs(res[0][2] - res[2][2]).max()
    say(f"  pieces vs whole runs: counts equal, max |FP64 minutes diff| {d:.2e}")
    assert d <= 1e-9 * max(1.0, np.abs(res[2][2]).max())
    assert np.abs(res[0][1] - res[2][1]).max() <= 1e-3
