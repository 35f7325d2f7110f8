"""sa_accumulate inside a captured HIP graph: both forms, the spill rounds
(ring of poles), the continuous-shadow kernel and the allocation-free entry
point (whose work counters and clears are fill kernels).  Every replay, with eager
work and synchronisations between replays, must equal the eager result:
exactly for counts, and to float rounding for minutes where the spill
rounds add with atomics (their order, hence the last bits, varies between
runs, eager or replayed)."""
import numpy as np
import pytest

import paper_1907_04435_amd as sa
from workloads import subset_points

from test_gpu_spill import SPAN as RING_SPAN, centre_points, ring_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sa.Context(0)


def capture_and_replay(ctx, call, outputs):
    import torch
    call()                                   # eager result on the default stream
    torch.cuda.synchronize()
    eager = [o.clone() for o in outputs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ctx.set_stream(s)
        call()                               # warm on the capture stream
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            call()
    ctx.set_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for r in range(3):
        for o in outputs:
            o.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outputs, eager):
            if o.dtype == torch.int32:
                assert torch.equal(o, e), f"replay {r}"
            else:
                assert torch.allclose(o, e, rtol=1e-6, atol=1e-4), f"replay {r}"
        _ = (torch.ones(4096, device="cuda") * r).sum().item()   # eager work between replays


@pytest.mark.parametrize("case", ["accrual_small", "sampled_small", "accrual_ring", "continuous_ring",
                                  "accrual_noalloc"])
def test_accumulate_graph_replay(ctx, c1, case):
    import torch
    if case.endswith("ring"):
        scene, pts, span = ring_scene(), centre_points(), RING_SPAN
    else:
        scene, pts, span = c1.scene, c1.points.take(subset_points(c1.points, 4096, seed=3)), c1.span
    path = sa.Path(ctx, sa.sunpath_for_span(span, 30.0))
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    B = path.n_bins
    counts = torch.empty((B, dp.n), dtype=torch.int32, device="cuda")
    mins = torch.empty((B, dp.n), dtype=torch.float32, device="cuda")
    longest = torch.empty((B, dp.n), dtype=torch.float32, device="cuda") if case.startswith("continuous") else None
    mode = sa.SA_SAMPLED if case.startswith("sampled") else sa.SA_ACCRUAL
    outs = [counts, mins] + ([longest] if longest is not None else [])

    fn = sa.sa_accumulate_noalloc if case.endswith("noalloc") else sa.sa_accumulate

    def call():
        fn(ctx, sc, dp, path, mode, counts, mins, longest=longest)

    capture_and_replay(ctx, call, outs)
