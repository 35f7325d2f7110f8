"""Entry-point behaviour through the C ABI: output scaling, the add flag,
and argument errors."""
import numpy as np
import pytest

import paper_1907_04435_amd as sa
from workloads import subset_points

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


@pytest.fixture(scope="module")
def setup(ctx, c1):
    pts = c1.points.take(subset_points(c1.points, 1024, seed=21))
    return (sa.Scene.from_workload(ctx, c1.scene), sa.DevicePoints.from_workload(pts),
            sa.Path(ctx, sa.sunpath_for_span(c1.span, 30.0)))


def outputs(path, dp):
    import torch
    mk = lambda dt: torch.empty((path.n_bins, dp.n), dtype=dt, device="cuda")
    return mk(torch.int32), mk(torch.float32), mk(torch.float32)


@pytest.mark.parametrize("mode", [sa.SA_SAMPLED, sa.SA_ACCRUAL])
def test_out_scale_and_add_flag(ctx, setup, mode):
    sc, dp, path = setup
    c, m, L = outputs(path, dp)
    sa.sa_accumulate(ctx, sc, dp, path, mode, c, m, longest=L)
    ctx.sync()
    c0, m0, L0 = c.cpu().numpy(), m.cpu().numpy(), L.cpu().numpy()
    sa.sa_accumulate(ctx, sc, dp, path, mode, c, m, out_scale=1.0 / 60.0, longest=L)
    ctx.sync()
    np.testing.assert_array_equal(c.cpu().numpy(), c0)          # counts are not scaled
    np.testing.assert_allclose(m.cpu().numpy(), m0 / 60.0, rtol=1e-6)
    np.testing.assert_allclose(L.cpu().numpy(), L0 / 60.0, rtol=1e-6)
    sa.sa_accumulate(ctx, sc, dp, path, mode, c, m, flags=sa.SA_FLAG_ADD, longest=L)
    ctx.sync()
    np.testing.assert_array_equal(c.cpu().numpy(), 2 * c0)
    np.testing.assert_allclose(m.cpu().numpy(), m0 / 60.0 + m0, rtol=1e-6)
    np.testing.assert_allclose(L.cpu().numpy(), np.maximum(L0 / 60.0, L0), rtol=1e-6)


def test_argument_errors(ctx, setup):
    import torch
    sc, dp, path = setup
    c, m, _ = outputs(path, dp)
    bits = torch.empty(((path.n_samples + 31) // 32, dp.n), dtype=torch.int32, device="cuda")
    with pytest.raises(sa.SAError) as e:
        sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, c, m, bits)      # bit vectors: sampled only
    assert e.value.code == -1
    with pytest.raises(sa.SAError) as e:
        sa.sa_accumulate(ctx, sc, dp, path, 7, c, m)                        # unknown form
    assert e.value.code == -1
    ids = torch.zeros((1, 1), dtype=torch.int32, device="cuda")
    hh = torch.full((1, 1), 10.0, dtype=torch.float32, device="cuda")
    off = torch.tensor([0, dp.n], dtype=torch.int64, device="cuda")
    opts = sa.sa_accum_opts(sa.SA_ACCRUAL, 0, 1.0, 0, None, m.data_ptr())  # continuous shadow: not batched
    ps = dp.struct()
    import ctypes as C
    rc = sa.lib().sa_accumulate_batched(ctx.handle, sc.handle, 1, 1, ids.data_ptr(), hh.data_ptr(), C.byref(ps),
                                        off.data_ptr(), path.handle, C.byref(opts), c.data_ptr(), m.data_ptr())
    assert rc == -1
    with pytest.raises(sa.SAError) as e:
        sa.sa_building_contribution(ctx, sc, dp, path, None, None)         # no output
    assert e.value.code == -1
    ctx.sync()                                                              # nothing left pending


def test_batched_bad_variant_reported_at_sync(ctx, setup, c1):
    """A variant naming a building id outside the scene is rejected on the
    device; the next sa_sync reports it (and clears it)."""
    import torch
    sc, dp, path = setup
    c, m, _ = outputs(path, dp)
    ids = torch.tensor([[c1.scene.n_b + 5]], dtype=torch.int32, device="cuda")
    hh = torch.full((1, 1), 10.0, dtype=torch.float32, device="cuda")
    off = torch.tensor([0, dp.n], dtype=torch.int64, device="cuda")
    sa.sa_accumulate_batched(ctx, sc, ids, hh, dp, off, path, c, m)
    with pytest.raises(sa.SAError) as e:
        ctx.sync()
    assert e.value.code == -1
    ctx.sync()                                                # cleared


def test_scene_upload_from_device_arrays(ctx, c1):
    """The scene arrays may live in device memory: the hierarchy and the
    results equal those of the same scene uploaded from host arrays."""
    import torch
    host = sa.Scene.from_workload(ctx, c1.scene)
    dev = sa.Scene(ctx, torch.from_numpy(c1.scene.vert_off.astype(np.int32)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(c1.scene.xy, np.float32)).cuda(),
                   torch.from_numpy(c1.scene.height.astype(np.float32)).cuda())
    nh, oh = host.read_bvh()
    nd, od = dev.read_bvh()
    assert np.array_equal(nh, nd) and np.array_equal(oh, od)
    sub = c1.points.take(np.arange(0, c1.points.n, 97))
    dp = sa.DevicePoints.from_workload(sub)
    path = sa.Path(ctx, sa.sunpath_for_span(c1.span, 30.0))
    a = sa.accumulate(ctx, host, dp, path, sa.SA_ACCRUAL)[1]
    b = sa.accumulate(ctx, dev, dp, path, sa.SA_ACCRUAL)[1]
    ctx.sync()
    assert torch.equal(a, b)
    bad = torch.from_numpy(c1.scene.height.astype(np.float32)).cuda()
    bad[3] = -1.0                                           # validated through the host copy
    with pytest.raises(sa.SAError) as e:
        sa.Scene(ctx, torch.from_numpy(c1.scene.vert_off.astype(np.int32)).cuda(),
                 torch.from_numpy(np.ascontiguousarray(c1.scene.xy, np.float32)).cuda(), bad)
    assert e.value.code == -2


def test_valu_peak_measurement(ctx):
    """sa_measure_valu_peak: the FMA-chain lane-op rate lies between a
    third of the derived peak (256 CU x 64 lanes x 2.4 GHz) and the derived
    peak itself (the clock's maximum), and repeats within 10 %."""
    from gpu_util import say
    derived = 256 * 64 * 2.4e9
    a, b = ctx.measure_valu_peak(), ctx.measure_valu_peak()
    say(f"FMA-chain lane-op rate {a / 1e12:.2f} and {b / 1e12:.2f} T/s ({a / derived:.3f} of the derived peak)")
    for v in (a, b):
        assert derived / 3 < v < 1.02 * derived
    assert abs(a - b) <= 0.1 * max(a, b)
