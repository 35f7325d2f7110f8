#!/usr/bin/env python3
"""Benchmark: gross shadow of the Manhattan-like block scene on one MI355X.

Workload (default): 20,000 convex prisms on an 18 x 60 block grid, 4,000,000
sample points (2M open-space ground + 2M facade, 1 m lattice), 2019-03-20,
06-21 and 12-21 sunrise..sunset at 1-minute instants (2,159 instants per
point): 8.64e9 point-sun-steps per pass.

One step = one pass of the accrual (sun-movement) form over all points and
days, plus the per-day region sums.  Its throughput in effective
point-sun-step evaluations per second is the headline value.  The sampled
form (one ray per point per instant) is timed over the same points in its
own leg; their ratio and the per-point difference between the two forms
are reported beside it.  Inputs are resident in device memory before any
timed region.

Prints one JSON line (rank 0).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic cost model, VALU lane-operations per unit of work a lane's own
# traversal needs (fixed before any kernel was measured); the instrumented
# launch counts the units:
COST = {
    "ray_box": 14,         # ray vs box slab: 6 FMA + 6 min/max + 2 compares
    "ray_prism": 6,        # ray vs prism: entry/exit and height compare ...
    "ray_edge": 8,         # ... plus 8 per footprint edge (2D Cyrus-Beck)
    "fan_box": 28,         # fan (wedge) vs box: plane-box test and the sector's 2D bound
    "fan_prism": 40,       # fan vs prism: window intersection, angle by a cross/dot ratio ...
    "fan_edge": 10,        # ... plus 10 per footprint edge (2 plane distances and the crossing)
    "insert": 16,          # interval insertion: 4 per comparison, 4 comparisons in the 4-member set
}
LANE_OP_PEAK = 256 * 64 * 2.4e9   # CUs x lanes x clock: one VALU lane-op per lane per cycle


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_ops(work, mode):
    box, prism, edges, inserts = (int(work[i]) for i in range(4))
    if mode == "sampled":
        return box * COST["ray_box"] + prism * COST["ray_prism"] + edges * COST["ray_edge"]
    return box * COST["fan_box"] + prism * COST["fan_prism"] + edges * COST["fan_edge"] + \
        inserts * COST["insert"]


def committed_traffic(workload, seg):
    """HBM bytes per k_accrual launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken (or
    the launch differs from the profiled one)."""
    import hashlib
    p = os.path.join(ROOT, "profiles", "k_accrual_c2_hbm.json")
    if workload != "c2" or seg != 30.0 or not os.path.exists(p):
        return None
    rec = json.load(open(p))
    src = "".join(open(os.path.join(ROOT, "paper_1907_04435_amd", "csrc", f)).read()
                  for f in ("accumulate.hip", "traverse.h"))
    if hashlib.sha256(src.encode()).hexdigest()[:16] != rec["source_hash"]:
        return None
    return rec["traffic_bytes"]


def host_threads():
    """Worker threads for the oracle: the CPUs this process may run on,
    at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _mixed_subset(w, n, seed_g, seed_f):
    """Seeded subset of n points, half ground and half facade."""
    from workloads import subset_points
    ng = w.extra.get("n_ground", w.points.n)
    if ng == w.points.n:
        return subset_points(w.points, n, seed_g)
    return np.concatenate([subset_points(w.points.take(np.arange(ng)), n // 2, seed_g),
                           ng + subset_points(w.points.take(np.arange(ng, w.points.n)), n // 2, seed_f)])


def cpu_baseline(w, seconds_target=15.0):
    """The oracle (FP64, brute force) on a bounded sample of the same
    workload: sampled form, a seeded subset of points, every instant of
    every day, on all the host threads this process may use, and again on
    one thread over an eighth of the sample.  The rate is measured on the
    sample; the full workload's time at that rate is extrapolated."""
    import oracle
    threads = host_threads()
    path = oracle.sun_path(w.span)
    n = 64
    idx = _mixed_subset(w, n, 11, 12)
    t = time.perf_counter()
    oracle.sampled(w.scene, w.points.take(idx), path, threads=threads)
    dt = time.perf_counter() - t
    # grow the sample to land in the target window
    n2 = int(min(4096, max(n, n * seconds_target / max(dt, 1e-3))))
    if n2 > n:
        idx = _mixed_subset(w, n2, 11, 12)
        t = time.perf_counter()
        oracle.sampled(w.scene, w.points.take(idx), path, threads=threads)
        dt = time.perf_counter() - t
    K = len(path.w)
    value = len(idx) * K / dt
    one = idx[:: max(1, len(idx) // max(8, len(idx) // 8))][: max(8, len(idx) // 8)]
    t = time.perf_counter()
    oracle.sampled(w.scene, w.points.take(one), path, threads=1)
    dt1 = time.perf_counter() - t
    full = w.points.n * K
    return {"value": value, "unit": "point-sun-steps/s", "cores": threads, "threads": threads,
            "nproc": os.cpu_count(), "kind": "oracle", "extrapolated": True,
            "single_thread_value": len(one) * K / dt1,
            "full_workload_seconds_extrapolated": full / value,
            "sample": f"{len(idx)} points ({len(idx)//2} ground + {len(idx)//2} facade, seeded) x "
                      f"{K} instants x {w.scene.n_b} prisms, sampled form, {dt:.1f} s on {threads} threads; "
                      f"single thread: {len(one)} of those points, {dt1:.1f} s; the rate is the sample's, "
                      f"the full workload ({full:.3g} point-sun-steps) would take "
                      f"{full / value:.3g} s at it"}


def _err_stats(x, ref):
    d = np.abs(np.asarray(x, np.float64) - ref).ravel()
    return {"mean": float(d.mean()), "p99": float(np.quantile(d, 0.99)), "max": float(d.max()),
            "frac_over_0.5": float((d > 0.5).mean())}


def accuracy_vs_oracle(w, sa, ctx, scene, head_seg, segs=(15.0, 20.0, 30.0, 45.0), n=2048):
    """Part of the CPU-baseline leg.  Method accuracy of both forms against the oracle's continuous
    duration along the sun's actual FP64 path (5-second scan and bisection
    per occluder, unioned): a seeded subset of n points (half ground, half
    facade) over every day of the workload; per point-day |form - truth| in
    minutes.  Accrual form at several knot spacings L and with a knot at
    every instant; sampled form at the workload's instants."""
    import oracle
    idx = _mixed_subset(w, n, 21, 22)
    sub = w.points.take(idx)
    threads = host_threads()
    t = time.perf_counter()
    truth = oracle.continuous_true(w.scene, sub, w.span, threads=threads)["minutes"]
    dt = time.perf_counter() - t
    dp = sa.DevicePoints.from_workload(sub)
    res = {"reference": "oracle: continuous duration on the actual FP64 sun path (Sec. 3.1, 3.2); "
                        "per occluder a 5-second scan with bisection, unioned",
           "points": int(sub.n), "point_days": int(truth.size), "oracle_seconds": dt,
           "oracle_threads": threads,
           "oracle_point_sun_steps_per_s": float(sub.n * len(oracle.sun_path(w.span).w) / dt),
           "statistic": "per point and day, |form - truth| (minutes)"}
    legs = {}
    for L in sorted(set(segs) | {float(head_seg), float(w.span.step_min)}):
        p = sa.Path(ctx, sa.sunpath_for_span(w.span, L))
        _, m, _ = sa.accumulate(ctx, scene, dp, p, sa.SA_ACCRUAL, want_counts=False)
        ctx.sync()
        legs[f"accrual_L{L:g}"] = _err_stats(m.cpu().numpy(), truth)
        p.close()
    p = sa.Path(ctx, sa.sunpath_for_span(w.span, head_seg))
    _, m, _ = sa.accumulate(ctx, scene, dp, p, sa.SA_SAMPLED, want_counts=False)
    ctx.sync()
    legs["sampled"] = _err_stats(m.cpu().numpy(), truth)
    p.close()
    res["forms"] = legs
    ok = [L for L in sorted(set(segs) | {float(head_seg)}) if legs[f"accrual_L{L:g}"]["mean"] <= 0.5]
    res["largest_L_with_mean_within_0.5"] = max(ok) if ok else None
    res["headline_L"] = float(head_seg)
    res["headline_mean_within_0.5"] = legs[f"accrual_L{float(head_seg):g}"]["mean"] <= 0.5
    return res


def _timed(torch, stream, fn, steps):
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, c in evs:
        a.record(stream)
        fn()
        c.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(c) for a, c in evs]


def _base(metric, value, unit, args, ms, cfg, dtype="f32"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}


def bench_c3(args, sa, torch):
    """256 development variants of the block scene, one persistent launch
    with per-variant refit; Jun 21 + Dec 21."""
    from workloads import make_c3
    w = make_c3()
    ctx = sa.Context(0)
    from paper_1907_04435_amd import tune
    launch = {} if args.untuned else tune.apply(ctx)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, args.seg))
    dp = sa.DevicePoints.from_workload(w.points)
    ids = torch.from_numpy(w.extra["var_ids"].astype(np.int32)).cuda()
    hh = torch.from_numpy(w.extra["var_h"].astype(np.float32)).cuda()
    off = torch.from_numpy(w.extra["var_off"].astype(np.int64)).cuda()
    counts = torch.empty((path.n_bins, dp.n), dtype=torch.int32, device="cuda")
    mins = torch.empty((path.n_bins, dp.n), dtype=torch.float32, device="cuda")
    gb = args.grid_blocks
    run = lambda: sa.sa_accumulate_batched(ctx, sc, ids, hh, dp, off, path, counts, mins, grid_blocks=gb)
    for _ in range(args.warmup):
        run()
    ctx.sync()
    ms = _timed(torch, ctx.stream, run, args.steps)
    ctx.sync()
    evals = dp.n * path.n_samples
    m = float(np.mean(ms))
    log(f"c3: {m:.1f} ms per batched pass, launch {launch or 'defaults'}")
    r = _base("point-sun-step evals/s (accrual form, batched variants)", evals / (m / 1e3),
              "point-sun-steps/s", args, m,
              {"workload": w.name, "variants": int(len(off) - 1), "points": dp.n, "buildings": w.scene.n_b,
               "instants_per_point": path.n_samples, "seg_min": args.seg, "point_sun_steps": evals})
    r["tuning"] = {"grid_blocks_arg": gb, **launch}
    return r


def bench_c4(args, sa, torch):
    """Loss = total shadow minutes over the 200k-point park, Mar 20, knots
    every minute; forward and height adjoint for all 5,000 buildings."""
    from workloads import make_c4
    w = make_c4()
    ctx = sa.Context(0)
    from paper_1907_04435_amd import tune
    launch = {} if args.untuned else tune.apply(ctx)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(w.span, 1.0))
    dp = sa.DevicePoints.from_workload(w.points)
    mins = torch.empty((1, dp.n), dtype=torch.float32, device="cuda")
    grad = torch.empty(w.scene.n_b, dtype=torch.float32, device="cuda")
    fwd = lambda: sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, None, mins)
    bwd = lambda: sa.sa_grad_heights(ctx, sc, dp, path, None, grad)
    for _ in range(args.warmup):
        fwd()
        bwd()
    ctx.sync()
    mf = float(np.mean(_timed(torch, ctx.stream, fwd, args.steps)))
    mb = float(np.mean(_timed(torch, ctx.stream, bwd, args.steps)))
    ctx.sync()
    evals = dp.n * path.n_samples
    log(f"c4: forward {mf:.2f} ms, adjoint {mb:.2f} ms")
    r = _base("point-sun-step evals/s (accrual forward + height adjoint)", evals / ((mf + mb) / 1e3),
              "point-sun-steps/s", args, mf + mb,
              {"workload": w.name, "points": dp.n, "buildings": w.scene.n_b, "instants_per_point": path.n_samples,
               "seg_min": 1.0, "point_sun_steps": evals})
    r["forward_ms"], r["adjoint_ms"] = mf, mb
    r["tuning"] = launch
    r["loss_minutes"] = float(mins.double().sum())
    r["grad_nonzero"] = int((grad != 0).sum())
    return r


def bench_sam(args, sa, torch):
    """Raster shadow accrual maps (Sec. 4), the exploration form: the block
    scene's 2M ground points over June 21 at 1-minute instants, knots every
    ``--seg`` minutes, ``--texel`` m texels; agreement with the sampled
    form (a ray per instant along the actual sun direction) on the same
    points and instants."""
    from workloads import Span, make_c2
    w = make_c2(n_facade=0)
    span = Span(w.span.lat, w.span.lon, [w.span.days[1]], w.span.step_min)
    ctx = sa.Context(0)
    from paper_1907_04435_amd import tune
    launch = {} if args.untuned else tune.apply(ctx)
    sc = sa.Scene.from_workload(ctx, w.scene)
    path = sa.Path(ctx, sa.sunpath_for_span(span, args.seg))
    dp = sa.DevicePoints.ground_from_workload(w.points)
    counts = torch.empty((1, dp.n), dtype=torch.int32, device="cuda")
    mins = torch.empty((1, dp.n), dtype=torch.float32, device="cuda")
    run = lambda: sa.sa_sam_accumulate(ctx, sc, dp, path, args.texel, counts, mins)
    for _ in range(args.warmup):
        run()
    ctx.sync()
    steps = max(1, min(args.steps, 3))
    ms = _timed(torch, ctx.stream, run, steps)
    ctx.sync()
    m = float(np.mean(ms))
    # the per-instant rays and the accrual form on the same points and day
    cs = torch.empty_like(counts)
    ms_s = torch.empty_like(mins)
    run_s = lambda: sa.sa_accumulate(ctx, sc, dp, path, sa.SA_SAMPLED, cs, ms_s)
    run_s()
    ms_sampled = float(np.mean(_timed(torch, ctx.stream, run_s, steps)))
    ca, ma = torch.empty_like(counts), torch.empty_like(mins)
    run_a = lambda: sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, ca, ma)
    run_a()
    ms_accrual = float(np.mean(_timed(torch, ctx.stream, run_a, steps)))
    ctx.sync()
    d = (counts.long() - cs.long()).abs().double()
    evals = dp.n * path.n_samples
    log(f"sam: {m:.1f} ms per pass at {args.texel} m texels; |count - sampled| mean {float(d.mean()):.3f}")
    r = _base("point-sun-step evals/s (raster shadow accrual maps)", evals / (m / 1e3), "point-sun-steps/s", args, m,
              {"workload": "block scene ground points, Jun 21", "points": dp.n, "buildings": w.scene.n_b,
               "instants_per_point": path.n_samples, "seg_min": args.seg, "texel_m": args.texel,
               "point_sun_steps": evals})
    r["steps"] = steps
    r["tuning"] = launch
    if not args.no_cpu_baseline:
        # the oracle's raster form on a bounded seeded sample of the same points
        import oracle
        from workloads import subset_points
        sub = w.points.take(subset_points(w.points, 16, 13))
        box = (float(w.scene.xy[:, 0].min()), float(w.scene.xy[:, 1].min()), 0.0,
               float(w.scene.xy[:, 0].max()), float(w.scene.xy[:, 1].max()), float(w.scene.height.max()))
        opath = oracle.sun_path(span, args.seg)
        t = time.perf_counter()
        oracle.sam(w.scene, sub, opath, args.texel, box=box)
        dt = time.perf_counter() - t
        r["cpu_baseline"] = {"value": sub.n * len(opath.w) / dt, "unit": "point-sun-steps/s",
                             "cores": oracle.threads_default(), "kind": "oracle",
                             "sample": f"{sub.n} ground points (seeded) x {len(opath.w)} instants x {w.scene.n_b} "
                                       f"prisms, raster form with its ambiguity test, {dt:.1f} s"}
    r["vs_sampled_form"] = {"mean_abs_count_diff": float(d.mean()), "share_of_points_differing": float((d > 0).double().mean()),
                            "mean_count": float(counts.double().mean()), "mean_count_sampled": float(cs.double().mean()),
                            "sampled_ms_same_points_and_instants": ms_sampled}
    r["accrual_ms_same_points_and_day"] = ms_accrual
    log(f"same points and instants: sampled {ms_sampled:.1f} ms, accrual {ms_accrual:.1f} ms")
    return r


def bench_c5(args, sa, torch):
    """Year-long accumulation: 45k prisms, 16M ground points, all 365 days
    of 2019 at 1-minute instants, four season bins of hours."""
    from workloads import make_c5
    w = make_c5()
    ctx = sa.Context(0)
    from paper_1907_04435_amd import tune
    launch = {} if args.untuned else tune.apply(ctx)
    sc = sa.Scene.from_workload(ctx, w.scene)
    sp = sa.sunpath_for_span(w.span, args.seg)      # the workload's days, with their clock (EDT / EST)
    path = sa.Path(ctx, sp)
    dp = sa.DevicePoints.from_workload(w.points)
    hours = torch.empty((path.n_bins, dp.n), dtype=torch.float32, device="cuda")
    run = lambda: sa.sa_accumulate(ctx, sc, dp, path, sa.SA_ACCRUAL, None, hours, out_scale=1.0 / 60.0)
    steps = max(1, min(args.steps, 1))
    ms = _timed(torch, ctx.stream, run, steps)
    ctx.sync()
    evals = dp.n * path.n_samples
    m = float(np.mean(ms))
    log(f"c5: {m:.0f} ms for the year")
    r = _base("point-sun-step evals/s (accrual form, year in season bins)", evals / (m / 1e3),
              "point-sun-steps/s", args, m,
              {"workload": w.name, "points": dp.n, "buildings": w.scene.n_b, "days": 365,
               "instants_per_point": path.n_samples, "seg_min": args.seg, "bins": path.n_bins,
               "point_sun_steps": evals})
    r["steps"], r["warmup"] = steps, 0
    r["tuning"] = launch
    r["mean_hours_per_bin"] = [float(x) for x in hours.mean(1).cpu()]
    if not args.skip_graph:
        # the direction graph of Sec. 6: segments of a season whose knots
        # share a pair of hemisphere cells computed once; time and error
        # against the full path above, per cell size
        base = hours.clone()
        legs = []
        for bound in (0.25, 0.5, 1.0, 2.0, 3.0, 5.0):
            gp = sa.Path(ctx, sp, graph_bound_deg=bound)
            gh = torch.empty_like(hours)
            gms = _timed(torch, ctx.stream,
                         lambda: sa.sa_accumulate(ctx, sc, dp, gp, sa.SA_ACCRUAL, None, gh, out_scale=1.0 / 60.0), 1)
            ctx.sync()
            err = float((gh - base).abs().sum(0).mean()) * 60.0 / 365.0
            tot = float((gh.sum(dtype=torch.float64) - base.sum(dtype=torch.float64)).abs() /
                        base.sum(dtype=torch.float64))
            legs.append({"cell_deg": bound, "segments": gp.n_segments, "ms": float(np.mean(gms)),
                         "mean_abs_error_min_per_point_day": err, "region_total_rel_error": tot})
            log(f"c5 graph {bound} deg: {gp.n_segments} of {path.n_segments} segments, "
                f"{legs[-1]['ms']:.0f} ms, mean |error| {err:.3f} min/point/day")
            gp.close()
        r["direction_graph"] = {"segments_full": path.n_segments, "legs": legs}
        # the same with knots on the clock: every day's inner knots at the
        # multiples of the spacing in local time, so days share knot times;
        # errors against the full path on those knots
        spc = sa.sunpath_for_span(w.span, args.seg, clock_knots=True)
        pc = sa.Path(ctx, spc)
        basec = torch.empty_like(hours)
        cms = _timed(torch, ctx.stream,
                     lambda: sa.sa_accumulate(ctx, sc, dp, pc, sa.SA_ACCRUAL, None, basec, out_scale=1.0 / 60.0), 1)
        ctx.sync()
        legs_c = []
        for bound in (1.0, 3.0, 5.0, 10.0):
            gp = sa.Path(ctx, spc, graph_bound_deg=bound)
            gh = torch.empty_like(hours)
            gms = _timed(torch, ctx.stream,
                         lambda: sa.sa_accumulate(ctx, sc, dp, gp, sa.SA_ACCRUAL, None, gh, out_scale=1.0 / 60.0), 1)
            ctx.sync()
            err = float((gh - basec).abs().sum(0).mean()) * 60.0 / 365.0
            tot = float((gh.sum(dtype=torch.float64) - basec.sum(dtype=torch.float64)).abs() /
                        basec.sum(dtype=torch.float64))
            legs_c.append({"cell_deg": bound, "segments": gp.n_segments, "ms": float(np.mean(gms)),
                           "mean_abs_error_min_per_point_day": err, "region_total_rel_error": tot})
            log(f"c5 clock knots, graph {bound} deg: {gp.n_segments} of {pc.n_segments} segments, "
                f"{legs_c[-1]['ms']:.0f} ms, mean |error| {err:.3f} min/point/day")
            gp.close()
        r["direction_graph_clock_knots"] = {"segments_full": pc.n_segments, "ms_full": float(np.mean(cms)),
                                            "legs": legs_c}
        # the paper's own setting (Sec. 8.2): 9:00 to 15:00 every day in
        # hourly intervals on the clock, one accumulation over the year;
        # 2,190 intervals, which the paper's graph at 5 degrees reduces to
        # 299 edges
        from workloads import Span
        from workloads.scenes import Day
        pdays = [Day(d.year, d.month, d.day, d.tz_h, (540.0, 900.0)) for d in w.span.days]
        psp = sa.sunpath_for_span(Span(w.span.lat, w.span.lon, pdays, 60.0, [0] * len(pdays)), 60.0,
                                  clock_knots=True)
        pfull = sa.Path(ctx, psp)
        ph = torch.empty((1, dp.n), dtype=torch.float32, device="cuda")
        pms = _timed(torch, ctx.stream,
                     lambda: sa.sa_accumulate(ctx, sc, dp, pfull, sa.SA_ACCRUAL, None, ph, out_scale=1.0 / 60.0), 1)
        ctx.sync()
        pbase = ph.clone()
        plegs = []
        for bound in (1.0, 5.0):
            gp = sa.Path(ctx, psp, graph_bound_deg=bound)
            gms = _timed(torch, ctx.stream,
                         lambda: sa.sa_accumulate(ctx, sc, dp, gp, sa.SA_ACCRUAL, None, ph, out_scale=1.0 / 60.0), 1)
            ctx.sync()
            err = float((ph - pbase).abs().mean()) * 60.0 / len(pdays)
            plegs.append({"cell_deg": bound, "edges": gp.n_segments, "ms": float(np.mean(gms)),
                          "speedup": float(np.mean(pms)) / float(np.mean(gms)),
                          "mean_abs_error_min_per_point_day": err})
            log(f"c5 paper setting, {bound} deg: {pfull.n_segments} intervals -> {gp.n_segments} edges, "
                f"{plegs[-1]['ms']:.0f} ms vs {float(np.mean(pms)):.0f} ms, error {err:.3f} min/point/day")
            gp.close()
        r["direction_graph_paper_setting"] = {"intervals": pfull.n_segments, "ms_full": float(np.mean(pms)),
                                              "paper": {"intervals": 2190, "edges_5deg": 299}, "legs": plegs}
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seg", type=float, default=None,
                    help="accrual knot spacing, minutes (default: the autotuner's choice, else 30)")
    ap.add_argument("--untuned", action="store_true", help="ignore the autotuner's cached choices")
    ap.add_argument("--sampled-steps", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "sam"],
                    help="c2 (default): the block scene, both forms; c3 batched variants; "
                         "c4 forward + height adjoint; c5 year-long season bins; c1 the small scene; "
                         "sam the raster shadow accrual maps on the block scene's ground points")
    ap.add_argument("--texel", type=float, default=2.0, help="sam: texel edge on the shadow plane, metres")
    ap.add_argument("--grid-blocks", type=int, default=0, help="batched persistent launch size (0: tuned/default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-work-count", action="store_true")
    ap.add_argument("--skip-sampled", action="store_true")
    ap.add_argument("--skip-contribution", action="store_true",
                    help="skip the building-contribution leg")
    ap.add_argument("--skip-continuous", action="store_true",
                    help="skip the continuous-shadow leg (accrual form with the longest-run output)")
    ap.add_argument("--skip-graph", action="store_true",
                    help="c5: skip the direction-graph legs (segments merged across days)")
    ap.add_argument("--no-truth", action="store_true",
                    help="skip the accuracy leg (both forms against the oracle's duration on the actual sun path)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(points would shard across GPUs, each holding a copy of the scene)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "dispatches": 3}))
        return
    import paper_1907_04435_amd as sa
    from paper_1907_04435_amd import tune
    from workloads import make_c1, make_c2
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    tuned = {} if args.untuned else tune.load(arch)
    if args.seg is None:
        args.seg = float(tuned.get("seg_min", 30.0))
    if args.workload in ("c3", "c4", "c5", "sam"):
        res = {"c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "sam": bench_sam}[args.workload](args, sa, torch)
        print(json.dumps(res), flush=True)
        return

    t0 = time.perf_counter()
    w = make_c2() if args.workload == "c2" else make_c1()
    log(f"workload {w.name}: {w.scene.n_b} prisms, {w.points.n} points, generated in {time.perf_counter()-t0:.1f} s")
    ctx = sa.Context(0)
    launch = tune.apply(ctx, tuned) if tuned else {}
    stream = ctx.stream
    scene = sa.Scene.from_workload(ctx, w.scene)
    sp_acc = sa.sunpath_for_span(w.span, args.seg)
    path = sa.Path(ctx, sp_acc)
    pts = sa.DevicePoints.from_workload(w.points)
    n, K, B = pts.n, path.n_samples, path.n_bins
    evals = n * K
    dev = "cuda:0"
    counts_a = torch.empty((B, n), dtype=torch.int32, device=dev)
    mins_a = torch.empty((B, n), dtype=torch.float32, device=dev)
    counts_s = torch.empty((B, n), dtype=torch.int32, device=dev)
    mins_s = torch.empty((B, n), dtype=torch.float32, device=dev)
    ng = w.extra.get("n_ground", n)
    region_off = torch.tensor([0, ng, n], dtype=torch.int64, device=dev)
    region_out = torch.empty((B, 2), dtype=torch.float64, device=dev)
    log(f"scene: {scene.info()}; path: {B} bins, {K} instants, {path.n_segments} segments")
    torch.cuda.synchronize()

    def accrual_step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        sa.sa_accumulate(ctx, scene, pts, path, sa.SA_ACCRUAL, counts_a, mins_a)
        if ev is not None:
            ev[1].record(stream)
        for b in range(B):
            sa.sa_region_sum(ctx, mins_a[b], region_off, region_out[b])

    for i in range(args.warmup):
        accrual_step()
        ctx.sync()
        log(f"warmup {i} done")

    # ---- timed accrual steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(args.steps):
        accrual_step(evs[i])
    end.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(end)
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    ms_step = total_ms / args.steps
    log(f"accrual: {ms_step:.1f} ms/step, launches {['%.1f' % x for x in launch_ms]}")
    launch_stats = {"median": float(np.median(launch_ms)), "min": float(np.min(launch_ms)),
                    "max": float(np.max(launch_ms))}

    result = {
        "metric": "point-sun-step evals/s (accrual form; sampled form beside it)",
        "value": evals / (ms_step / 1e3),
        "unit": "point-sun-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "points": n, "ground_points": ng, "facade_points": n - ng,
                   "buildings": w.scene.n_b, "instants_per_point": K, "days": B, "seg_min": args.seg,
                   "point_sun_steps": evals},
        "accumulate_launch_ms": launch_stats,
        "tuning": {"source": "paper_1907_04435_amd/tuning.json" if tuned else "defaults", "seg_min": args.seg,
                   **launch},
    }

    # ---- continuous shadow leg (gross and longest uninterrupted shadow in one pass)
    if not args.skip_continuous:
        longest = torch.empty((B, n), dtype=torch.float32, device=dev)
        sa.sa_accumulate(ctx, scene, pts, path, sa.SA_ACCRUAL, counts_a, mins_a, longest=longest)   # warm
        ctx.sync()
        cev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        cev[0].record(stream)
        for _ in range(2):
            sa.sa_accumulate(ctx, scene, pts, path, sa.SA_ACCRUAL, counts_a, mins_a, longest=longest)
        cev[1].record(stream)
        ctx.sync()
        c_ms = cev[0].elapsed_time(cev[1]) / 2
        log(f"continuous shadow: {c_ms:.1f} ms/pass")
        result["continuous_shadow"] = {"value": evals / (c_ms / 1e3), "unit": "point-sun-steps/s",
                                       "ms_per_pass": c_ms, "kernel": "k_accrual_runs",
                                       "mean_longest_minutes": float(longest.double().mean())}
        del longest

    # ---- building contribution leg (every building's own shadow time on the points)
    if not args.skip_contribution:
        contrib = torch.empty((B, w.scene.n_b), dtype=torch.float64, device=dev)
        sa.sa_building_contribution(ctx, scene, pts, path, None, contrib)   # warm
        ctx.sync()
        bev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        bev[0].record(stream)
        sa.sa_building_contribution(ctx, scene, pts, path, None, contrib)
        bev[1].record(stream)
        ctx.sync()
        b_ms = bev[0].elapsed_time(bev[1])
        log(f"building contribution: {b_ms:.1f} ms/pass")
        result["building_contribution"] = {"value": evals / (b_ms / 1e3), "unit": "point-sun-steps/s",
                                           "ms_per_pass": b_ms, "kernel": "k_contrib",
                                           "buildings_with_shadow": int((contrib > 0).any(0).sum())}
        del contrib

    # ---- sampled leg
    if not args.skip_sampled:
        sa.sa_accumulate(ctx, scene, pts, path, sa.SA_SAMPLED, counts_s, mins_s)   # warm
        ctx.sync()
        sev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
        sev[0].record(stream)
        for _ in range(args.sampled_steps):
            sa.sa_accumulate(ctx, scene, pts, path, sa.SA_SAMPLED, counts_s, mins_s)
        sev[1].record(stream)
        ctx.sync()
        s_ms = sev[0].elapsed_time(sev[1]) / args.sampled_steps
        log(f"sampled: {s_ms:.1f} ms/pass")
        result["sampled"] = {"value": evals / (s_ms / 1e3), "unit": "point-sun-steps/s", "ms_per_pass": s_ms}
        result["accrual_over_sampled"] = (evals / (ms_step / 1e3)) / (evals / (s_ms / 1e3))
        # the outputs that need every instant in order (bitmap replay):
        # bit vectors of Sec. 5 and the continuous shadow, same points
        if not args.skip_continuous:
            bits = torch.empty(((K + 31) // 32, n), dtype=torch.int32, device=dev)
            runs = torch.empty((B, n), dtype=torch.float32, device=dev)
            ordered = {}
            for name, kw in (("bit_vectors", {"bits": bits}), ("continuous_shadow", {"longest": runs})):
                call = lambda: sa.sa_accumulate(ctx, scene, pts, path, sa.SA_SAMPLED, counts_s, mins_s,
                                                kw.get("bits"), longest=kw.get("longest"))
                call()
                ctx.sync()
                ordered[name] = float(np.median(_timed(torch, stream, call, 3)))
            result["sampled"]["ordered_outputs_ms_per_pass"] = ordered
            log(f"sampled with bit vectors {ordered['bit_vectors']:.1f} ms, with the continuous shadow "
                f"{ordered['continuous_shadow']:.1f} ms")
            del bits, runs

    # ---- accuracy over every point: the headline accrual and the sampled
    # form against the accrual form with a knot at every instant (the CPU
    # baseline leg below ties that reference to the oracle on a subset)
    acc = {}
    if not args.no_truth:
        path1 = sa.Path(ctx, sa.sunpath_for_span(w.span, w.span.step_min))
        truth = torch.empty((B, n), dtype=torch.float32, device=dev)
        sa.sa_accumulate(ctx, scene, pts, path1, sa.SA_ACCRUAL, None, truth)
        ctx.sync()

        def errstats(x):
            d = (x - truth).abs()
            return {"mean": float(d.mean()), "p99": float(torch.quantile(d.flatten()[::13].float(), 0.99)),
                    "max": float(d.max()), "frac_over_0.5": float((d > 0.5).float().mean())}
        full = {"reference": f"accrual form with a knot every {w.span.step_min:g} min, all points",
                "accrual": errstats(mins_a)}
        if "sampled" in result:
            full["sampled"] = errstats(mins_s)
        acc["all_points_vs_1min_knots"] = full
        result["accuracy_minutes_per_point_day"] = acc
        del truth, path1

    # ---- instrumented runs: algorithmic work per launch
    if not args.no_work_count:
        work = torch.zeros(8, dtype=torch.int64, device=dev)
        sa.sa_accumulate(ctx, scene, pts, path, sa.SA_ACCRUAL, counts_a, mins_a, work=work)
        ctx.sync()
        wa = work.cpu().numpy()
        ops = algorithmic_ops(wa, "accrual")
        avg_s = float(np.mean(launch_ms)) / 1e3
        achieved = ops / avg_s
        result["roofline"] = {"bound": "alu", "kernel": "k_accrual", "achieved": achieved / 1e12,
                              "peak": LANE_OP_PEAK / 1e12, "unit": "Tlane-op/s", "frac": achieved / LANE_OP_PEAK,
                              "traffic": committed_traffic(args.workload, args.seg),
                              "work_per_launch": {"box_tests": int(wa[0]), "prism_tests": int(wa[1]),
                                                  "prism_edges": int(wa[2]), "inserts": int(wa[3]),
                                                  "node_fetches_per_wave": int(wa[4]),
                                                  "point_segments": int(wa[5]), "spilled": int(wa[6]),
                                                  "leaf_visits_per_wave": int(wa[7]), "lane_ops": ops}}
        log(f"accrual work: {wa.tolist()} -> {ops:.3e} lane-ops, {achieved/1e12:.2f} T/s")
        # the derived peaks checked on this device: FP32 FMA chains (lane-op
        # rate, sa_measure_valu_peak) and a 1 GiB device copy (HBM)
        valu = ctx.measure_valu_peak()
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        cms = min(_timed(torch, torch.cuda.current_stream(), lambda: dst.copy_(src), 3))
        copy_gbs = 2 * src.numel() * 4 / (cms / 1e3) / 1e9
        del src, dst
        result["roofline"]["peak_check"] = {
            "valu_lane_ops_per_s": valu, "valu_of_derived_peak": valu / LANE_OP_PEAK,
            "frac_of_measured_valu": achieved / valu if valu > 0 else None,
            "copy_GB_per_s": copy_gbs, "copy_of_8TBps": copy_gbs / 8000.0}
        log(f"peak check: {valu/1e12:.2f} Tlane-op/s FMA chains, {copy_gbs:.0f} GB/s copy")
        if not args.skip_sampled:
            work.zero_()
            sa.sa_accumulate(ctx, scene, pts, path, sa.SA_SAMPLED, counts_s, mins_s, work=work)
            ctx.sync()
            ws = work.cpu().numpy()
            sops = algorithmic_ops(ws, "sampled")
            result["sampled"]["roofline_frac"] = (sops / (result["sampled"]["ms_per_pass"] / 1e3)) / LANE_OP_PEAK
            result["sampled"]["work_per_pass"] = {"box_tests": int(ws[0]), "prism_tests": int(ws[1]),
                                                  "prism_edges": int(ws[2]),
                                                  "node_fetches_per_wave": int(ws[4]),
                                                  "leaf_visits_per_wave": int(ws[7]), "lane_ops": sops}
            log(f"sampled work: {ws.tolist()} -> {sops:.3e} lane-ops")

    # ---- CPU baseline leg (rank 0, N = 1): the oracle timed on the host
    # cores, and its continuous duration on the actual sun path as the
    # reference of both forms' accuracy on a seeded subset
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(w)
        if not args.no_truth:
            log("accuracy against the oracle ...")
            ref = accuracy_vs_oracle(w, sa, ctx, scene, args.seg)
            ref["all_points_vs_1min_knots"] = acc.get("all_points_vs_1min_knots")
            result["accuracy_minutes_per_point_day"] = ref
            log(f"accuracy: {json.dumps(ref)}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
