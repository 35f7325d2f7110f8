"""CPU oracle (FP64, brute force) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library; the two meet
only in the seeded inputs from ``workloads``.

The C sources (``solar.c``, ``shadow.c``) compute:
  * solar position: NOAA solar-calculator / Meeus low-precision equations;
  * the shadow predicate: brute-force ray vs every convex prism (2D
    Cyrus-Beck + height), and an independent Moller-Trumbore version;
  * sampled gross shadow (count and minutes) with a silhouette-ambiguity
    mask;
  * continuous gross shadow along a piecewise great-circle sun path (grid +
    bisection per occluder, union, measure).

In Python on top of those: the continuous shadow of the sampled form, the
shadow score, the direction graph of Sec. 6 (hemisphere cells, edges on
their members' mean arc, the accrual form over the edges weighted by the
members' durations) and the raster shadow accrual maps of Sec. 4.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp, ip, fp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_float)
        L.orc_julian_day.restype = C.c_double
        L.orc_julian_day.argtypes = [C.c_int, C.c_int, C.c_double]
        L.orc_solar.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_solar_jd.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_day_samples.restype = C.c_int
        L.orc_day_samples.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_double, dp, dp, C.c_int, dp]
        for f in (L.orc_shadow, L.orc_shadow_mt):
            f.restype = C.c_int
            f.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp]
        L.orc_sampled.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, ip, C.c_int, ip, dp,
                                  C.POINTER(C.c_uint32), C.POINTER(C.c_uint8), C.c_int]
        L.orc_continuous.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, ip, C.c_int, ip, C.c_int,
                                     C.c_double, dp, ip, C.c_int, dp, ip, dp, C.c_int]
        L.orc_continuous_true.argtypes = [C.c_void_p, C.c_void_p, C.c_int, ip, dp, dp, ip, C.c_int, C.c_double,
                                          C.c_double, C.c_double, C.c_double, dp, dp, C.c_int]
        L.orc_slerp.argtypes = [dp, dp, C.c_double, dp]
        L.orc_contribution.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, ip, ip, C.c_int, C.c_double, dp,
                                       dp, C.c_int]
        L.orc_grad_implicit.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, ip, ip, C.c_double, dp, dp,
                                        C.c_int]
        L.orc_exit_depths.argtypes = [C.c_void_p, C.c_int64, dp, dp, C.c_double, dp, C.c_int]
        _lib = L
    return _lib


class _Scene(C.Structure):
    _fields_ = [("n_b", C.c_int32), ("vert_off", C.c_void_p), ("xy", C.c_void_p), ("height", C.c_void_p)]


class _Points(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("nx", C.c_void_p), ("ny", C.c_void_p), ("owner", C.c_void_p)]


def _ptr(a, ct=None):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct)) if ct is not None else a.ctypes.data


def _scene(scene):
    keep = (np.ascontiguousarray(scene.vert_off, np.int32), np.ascontiguousarray(scene.xy, np.float32),
            np.ascontiguousarray(scene.height, np.float32))
    s = _Scene(len(keep[2]), keep[0].ctypes.data, keep[1].ctypes.data, keep[2].ctypes.data)
    return s, keep


def _points(pts):
    keep = tuple(np.ascontiguousarray(getattr(pts, k), np.float32) for k in ("x", "y", "z", "nx", "ny")) + \
        (np.ascontiguousarray(pts.owner, np.int32),)
    s = _Points(len(keep[0]), *[k.ctypes.data for k in keep])
    return s, keep


def threads_default() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------
# solar position
# --------------------------------------------------------------------------
def julian_day(y, m, d) -> float:
    return lib().orc_julian_day(int(y), int(m), float(d))


def solar(y, m, d, t_loc_min, tz_h, lat, lon) -> np.ndarray:
    """[dirE, dirN, dirU, elev_deg, azim_deg, decl_deg, eot_min, app_long_deg, obliq_deg]"""
    out = np.zeros(9)
    lib().orc_solar(int(y), int(m), int(d), float(t_loc_min), float(tz_h), float(lat), float(lon),
                    _ptr(out, C.c_double))
    return out


def solar_jd(jd, lat, lon) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_solar_jd(float(jd), float(lat), float(lon), _ptr(out, C.c_double))
    return out


def day_samples(day, lat, lon, step):
    cap = 4000
    t, w, span = np.zeros(cap), np.zeros(cap), np.zeros(2)
    t0, t1 = (day.window if day.window is not None else (-1.0, -1.0))
    K = lib().orc_day_samples(day.year, day.month, day.day, day.tz_h, lat, lon, t0, t1, step,
                              _ptr(t, C.c_double), _ptr(w, C.c_double), cap, _ptr(span, C.c_double))
    if K < 0:
        raise ValueError("day samples: window not in daylight or capacity exceeded")
    return t[:K].copy(), w[:K].copy(), span


@dataclass
class OraclePath:
    dirs: np.ndarray        # [K, 3] FP64 sample directions
    w: np.ndarray           # [K] minutes
    t: np.ndarray           # [K] local minutes
    sample_day: np.ndarray  # [K] int32
    sample_bin: np.ndarray  # [K] int32
    seg_t: np.ndarray       # [J, 2]
    seg_dir: np.ndarray     # [J, 2, 3]
    seg_day: np.ndarray     # [J] int32
    day_bin: np.ndarray     # [n_days] int32
    n_bins: int
    spans: np.ndarray       # [n_days, 2]


def sun_path(span, seg_min: float | None = None, clock_knots: bool = False) -> OraclePath:
    """Sample instants and great-circle knots for every day of ``span``.
    Knots: T0, T0 + L, T0 + 2L, ... and T1 (the last segment may be
    shorter); L = ``seg_min`` (default: the sample step).  ``clock_knots``:
    T0, every multiple of L in local time strictly between T0 and T1, and
    T1."""
    L = float(seg_min if seg_min is not None else span.step_min)
    dirs, ws, ts, sd, sb = [], [], [], [], []
    seg_t, seg_dir, seg_day, spans = [], [], [], []
    day_bin = np.array(span.day_bin if span.day_bin is not None else range(len(span.days)), np.int32)
    for di, day in enumerate(span.days):
        t, w, sp = day_samples(day, span.lat, span.lon, span.step_min)
        spans.append(sp)
        for tk in t:
            dirs.append(solar(day.year, day.month, day.day, tk, day.tz_h, span.lat, span.lon)[:3])
        ws.append(w); ts.append(t)
        sd.append(np.full(len(t), di, np.int32)); sb.append(np.full(len(t), day_bin[di], np.int32))
        if len(t) == 0:
            continue
        T0, T1 = sp
        if clock_knots:
            m = np.floor(T0 / L) + 1.0
            knots = [T0] + [k * L for k in np.arange(m, np.ceil(T1 / L) + 1.0) if T0 < k * L < T1] + [T1]
        else:
            knots = list(np.arange(T0, T1, L))
            if knots[-1] < T1:
                knots.append(T1)
        kd = [solar(day.year, day.month, day.day, tk, day.tz_h, span.lat, span.lon)[:3] for tk in knots]
        for j in range(len(knots) - 1):
            seg_t.append((knots[j], knots[j + 1]))
            seg_dir.append((kd[j], kd[j + 1]))
            seg_day.append(di)
    return OraclePath(np.array(dirs).reshape(-1, 3), np.concatenate(ws), np.concatenate(ts),
                      np.concatenate(sd), np.concatenate(sb), np.array(seg_t).reshape(-1, 2),
                      np.array(seg_dir).reshape(-1, 2, 3), np.array(seg_day, np.int32), day_bin,
                      int(day_bin.max()) + 1 if len(day_bin) else 0, np.array(spans))


def slerp(a, b, f) -> np.ndarray:
    out = np.zeros(3)
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    lib().orc_slerp(_ptr(a, C.c_double), _ptr(b, C.c_double), float(f), _ptr(out, C.c_double))
    return out


# --------------------------------------------------------------------------
# predicate and accumulation
# --------------------------------------------------------------------------
def shadow(scene, p, d, nrm=(0.0, 0.0), owner=-1, mt=False) -> int:
    s, keep = _scene(scene)
    d = np.ascontiguousarray(d, np.float64)
    f = lib().orc_shadow_mt if mt else lib().orc_shadow
    return int(f(C.byref(s), float(p[0]), float(p[1]), float(p[2]), float(nrm[0]), float(nrm[1]),
                 int(owner), _ptr(d, C.c_double)))


def sampled(scene, pts, path: OraclePath, bits=False, amb=False, threads=None):
    """Sampled gross shadow: counts int32 [n_bins, n], minutes FP64
    [n_bins, n], optional bit vectors uint32 [n, ceil(K/32)] and ambiguity
    flags uint8 [n, K]."""
    s, ks = _scene(scene)
    p, kp = _points(pts)
    K, n = len(path.w), pts.n
    counts = np.zeros((path.n_bins, n), np.int32)
    minutes = np.zeros((path.n_bins, n), np.float64)
    b = np.zeros((n, (K + 31) // 32), np.uint32) if bits else None
    a = np.zeros((n, K), np.uint8) if amb else None
    dirs = np.ascontiguousarray(path.dirs, np.float64)
    w = np.ascontiguousarray(path.w, np.float64)
    sbin = np.ascontiguousarray(path.sample_bin, np.int32)
    lib().orc_sampled(C.byref(s), C.byref(p), K, _ptr(dirs, C.c_double), _ptr(w, C.c_double),
                      _ptr(sbin, C.c_int32), path.n_bins, _ptr(counts, C.c_int32),
                      _ptr(minutes, C.c_double), _ptr(b, C.c_uint32), _ptr(a, C.c_uint8),
                      threads or threads_default())
    return dict(counts=counts, minutes=minutes, bits=b, amb=a)


def continuous(scene, pts, path: OraclePath, grid_min=1.0 / 12.0, threads=None):
    """Continuous gross shadow along the piecewise great-circle path of
    ``path``'s knots: minutes FP64 [n_bins, n], counts (sample instants
    inside the shadowed set) int32 [n_bins, n], and longest FP64 [n_bins, n],
    the continuous shadow of Sec. 3.1 (longest uninterrupted stretch of a
    day's shadowed set, maximum over the bin's days)."""
    s, ks = _scene(scene)
    p, kp = _points(pts)
    n = pts.n
    minutes = np.zeros((path.n_bins, n), np.float64)
    counts = np.zeros((path.n_bins, n), np.int32)
    longest = np.zeros((path.n_bins, n), np.float64)
    seg_t = np.ascontiguousarray(path.seg_t, np.float64)
    seg_dir = np.ascontiguousarray(path.seg_dir, np.float64)
    seg_day = np.ascontiguousarray(path.seg_day, np.int32)
    day_bin = np.ascontiguousarray(path.day_bin, np.int32)
    st = np.ascontiguousarray(path.t, np.float64)
    sd = np.ascontiguousarray(path.sample_day, np.int32)
    lib().orc_continuous(C.byref(s), C.byref(p), len(seg_t), _ptr(seg_t, C.c_double),
                         _ptr(seg_dir, C.c_double), _ptr(seg_day, C.c_int32), len(day_bin),
                         _ptr(day_bin, C.c_int32), path.n_bins, float(grid_min),
                         _ptr(st, C.c_double), _ptr(sd, C.c_int32), len(st),
                         _ptr(minutes, C.c_double), _ptr(counts, C.c_int32), _ptr(longest, C.c_double),
                         threads or threads_default())
    return dict(minutes=minutes, counts=counts, longest=longest)


def continuous_true(scene, pts, span, piece_min=5.0, grid_min=1.0 / 12.0, threads=None, spans=None):
    """Continuous gross shadow along the sun's actual path (Sec. 3.1, 3.2):
    per point and day the measure of the times in the day's span [T0, T1]
    (its first and last daylight instant, or the fixed window) at which the
    point is in shadow for the FP64 solar direction at that time; per
    occluder a ``grid_min`` scan (5 s) with every switch bisected, unioned
    over occluders.  Summed into the span's bins: minutes FP64 [n_bins, n];
    longest FP64 [n_bins, n] (the longest member of a day's shadowed set,
    maximum over the bin's days).  ``spans``: [n_days, 2] (T0, T1) to use
    instead of the span's days."""
    s, ks = _scene(scene)
    p, kp = _points(pts)
    nd = len(span.days)
    if spans is None:
        spans = np.array([day_samples(d, span.lat, span.lon, span.step_min)[2] for d in span.days])
    spans = np.ascontiguousarray(np.asarray(spans, np.float64).reshape(nd, 2))
    ymd = np.ascontiguousarray([[d.year, d.month, d.day] for d in span.days], np.int32).reshape(nd, 3)
    tz = np.ascontiguousarray([d.tz_h for d in span.days], np.float64)
    day_bin = np.ascontiguousarray(span.day_bin if span.day_bin is not None else range(nd), np.int32)
    n_bins = int(day_bin.max()) + 1 if nd else 0
    minutes = np.zeros((n_bins, pts.n), np.float64)
    longest = np.zeros((n_bins, pts.n), np.float64)
    lib().orc_continuous_true(C.byref(s), C.byref(p), nd, _ptr(ymd, C.c_int32), _ptr(tz, C.c_double),
                              _ptr(spans, C.c_double), _ptr(day_bin, C.c_int32), n_bins, float(span.lat),
                              float(span.lon), float(piece_min), float(grid_min), _ptr(minutes, C.c_double),
                              _ptr(longest, C.c_double), threads or threads_default())
    return dict(minutes=minutes, longest=longest, spans=spans)


def longest_sampled(shadowed, path: OraclePath):
    """Continuous shadow of the sampled form (Sec. 3.1; with n-bit vectors,
    Sec. 5: the longest run of consecutive 1's): per point and bin, the
    largest total weight (minutes) of a run of consecutive shadowed
    instants within one day, maximum over the bin's days.  ``shadowed``:
    bool [n, K] predicate per point and instant.  FP64 [n_bins, n]."""
    sh = np.asarray(shadowed, bool)
    n = sh.shape[0]
    out = np.zeros((path.n_bins, n), np.float64)
    for d in range(len(path.day_bin)):
        ks = np.flatnonzero(path.sample_day == d)
        best = np.zeros(n)
        cur = np.zeros(n)
        for k in ks:
            cur = np.where(sh[:, k], cur + path.w[k], 0.0)
            best = np.maximum(best, cur)
        b = path.day_bin[d]
        out[b] = np.maximum(out[b], best)
    return out


def contribution(scene, pts, path: OraclePath, weight=None, grid_min=1.0 / 12.0, threads=None):
    """Building contribution (Sec. 7.2): FP64 [n_bins, n_b], per building the
    weighted minutes the points spend in that building's own shadow along
    the path's great-circle segments (overlapping shadows count for every
    building that casts them).  ``weight``: per-point weight (area), None
    = 1."""
    s, ks = _scene(scene)
    p, kp = _points(pts)
    out = np.zeros((path.n_bins, max(scene.n_b, 1)), np.float64)
    seg_t = np.ascontiguousarray(path.seg_t, np.float64)
    seg_dir = np.ascontiguousarray(path.seg_dir, np.float64)
    seg_day = np.ascontiguousarray(path.seg_day, np.int32)
    day_bin = np.ascontiguousarray(path.day_bin, np.int32)
    wt = None if weight is None else np.ascontiguousarray(weight, np.float64)
    lib().orc_contribution(C.byref(s), C.byref(p), len(seg_t), _ptr(seg_t, C.c_double),
                           _ptr(seg_dir, C.c_double), _ptr(seg_day, C.c_int32), _ptr(day_bin, C.c_int32),
                           path.n_bins, float(grid_min), _ptr(wt, C.c_double), _ptr(out, C.c_double),
                           threads or threads_default())
    return out[:, :scene.n_b]


def shadow_score(values, bin_weight, bin_span, area=None):
    """Shadow score of a region (Sec. 7.2): sum over its points of area(p)
    times sum over intervals t of w_t * shadow_t(p), with shadow_t(p) the
    fraction of the interval's daylight the point spends in shadow:
    values[t, p] (minutes) / bin_span[t] (the interval's daylight minutes).
    FP64 scalar."""
    v = np.asarray(values, np.float64)
    a = np.ones(v.shape[1]) if area is None else np.asarray(area, np.float64)
    frac = v / np.asarray(bin_span, np.float64)[:, None]
    return float((np.asarray(bin_weight, np.float64)[:, None] * frac * a[None, :]).sum())


def grad_implicit(scene, pts, path: OraclePath, dl=None, grid_min=1.0 / 12.0, threads=None):
    """d/dH_b of sum over points and bins of dl[bin, p] * continuous minutes
    (dl None = all ones), by implicit differentiation at the union
    boundaries made by roof edges.  FP64 [n_b]."""
    s, ks = _scene(scene)
    p, kp = _points(pts)
    grad = np.zeros(max(scene.n_b, 1), np.float64)
    seg_t = np.ascontiguousarray(path.seg_t, np.float64)
    seg_dir = np.ascontiguousarray(path.seg_dir, np.float64)
    seg_day = np.ascontiguousarray(path.seg_day, np.int32)
    day_bin = np.ascontiguousarray(path.day_bin, np.int32)
    d = None if dl is None else np.ascontiguousarray(dl, np.float64)
    lib().orc_grad_implicit(C.byref(s), C.byref(p), len(seg_t), _ptr(seg_t, C.c_double), _ptr(seg_dir, C.c_double),
                            _ptr(seg_day, C.c_int32), _ptr(day_bin, C.c_int32), float(grid_min),
                            _ptr(d, C.c_double), _ptr(grad, C.c_double), threads or threads_default())
    return grad[:scene.n_b]


def with_height(scene, b, h):
    """Copy of the scene with building b at height h."""
    from workloads import Scene
    hh = scene.height.astype(np.float32).copy()
    hh[b] = h
    return Scene(scene.vert_off, scene.xy, hh)


# --------------------------------------------------------------------------
# direction graph (Sec. 6)
# --------------------------------------------------------------------------
def hemisphere_cell(d, bound_deg):
    """Cell index of each direction d [..., 3] (east, north, up) when the
    sky is cut into cells of bounded angular size (Sec. 6 bins the sun's
    directions so): rings of ``bound`` in elevation, each ring cut into the
    fewest equal azimuth sectors whose width at the ring's lower edge is at
    most ``bound``.  int64 key: ring * 2^32 + sector (a ring has fewer
    than 2^32 sectors for bounds of at least 1e-6 degrees)."""
    b = np.radians(float(bound_deg))
    d = np.asarray(d, np.float64)
    el = np.arcsin(np.clip(d[..., 2], -1.0, 1.0))
    az = np.arctan2(d[..., 0], d[..., 1])
    ring = np.floor(el / b).astype(np.int64)
    n_sec = np.maximum(1, np.ceil(2.0 * np.pi * np.cos(ring * b) / b)).astype(np.int64)
    sec = np.minimum(np.floor((az + np.pi) / (2.0 * np.pi) * n_sec).astype(np.int64), n_sec - 1)
    return ring * (1 << 32) + sec


def direction_graph(path: OraclePath, bound_deg):
    """Edges of the direction graph (Sec. 6): the path's segments grouped by
    output bin and by the pair of cells that hold their start and end
    directions.  Returns a list of member-index lists in order of first
    appearance; the first member of each stands for the edge."""
    ca = hemisphere_cell(path.seg_dir[:, 0, :], bound_deg)
    cb = hemisphere_cell(path.seg_dir[:, 1, :], bound_deg)
    seg_bin = path.day_bin[path.seg_day]
    groups = {}
    for j in range(len(path.seg_t)):
        groups.setdefault((int(seg_bin[j]), int(ca[j]), int(cb[j])), []).append(j)
    return list(groups.values())


def edge_arc(path: OraclePath, group):
    """The arc an edge is computed on (the cluster's representative, Sec.
    6): from the members' mean start direction to their mean end direction,
    each normalised, over the first member's times; a lone segment is its
    own arc."""
    if len(group) == 1:
        return path.seg_dir[group[0]], path.seg_t[group[0]]
    a = path.seg_dir[group, 0].sum(0)
    b = path.seg_dir[group, 1].sum(0)
    return np.stack([a / np.linalg.norm(a), b / np.linalg.norm(b)]), path.seg_t[group[0]]


def graph_continuous(scene, pts, path: OraclePath, bound_deg, grid_min=1.0 / 12.0, threads=None):
    """Accrual form over the direction graph (Sec. 6, Eq. (1)): every edge's
    occluded set is computed once, on its representative arc (``edge_arc``),
    and each member counts with its own duration: the edge's minutes are the
    arc's continuous minutes times (sum of the members' durations) / (the
    arc's duration).  FP64 [n_bins, n] minutes, and the edge lists.  Each
    arc runs as a day of its own through ``continuous``."""
    groups = direction_graph(path, bound_deg)
    E = len(groups)
    arcs = [edge_arc(path, g) for g in groups]
    seg_dir = np.array([d for d, _ in arcs]).reshape(-1, 2, 3)
    seg_t = np.array([tt for _, tt in arcs]).reshape(-1, 2)
    sub = OraclePath(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0, np.int32), np.zeros(0, np.int32),
                     seg_t, seg_dir, np.arange(E, dtype=np.int32), np.arange(E, dtype=np.int32), E, seg_t)
    per_edge = continuous(scene, pts, sub, grid_min, threads)["minutes"]
    out = np.zeros((path.n_bins, pts.n), np.float64)
    dur = path.seg_t[:, 1] - path.seg_t[:, 0]
    seg_bin = path.day_bin[path.seg_day]
    for e, g in enumerate(groups):
        out[seg_bin[g[0]]] += per_edge[e] * (dur[g].sum() / dur[g[0]])
    return out, groups


# --------------------------------------------------------------------------
# shadow accrual map, raster form (Sec. 4)
# --------------------------------------------------------------------------
def sam_grid(box, a, b, texel):
    """Shadow plane and texel grid of one segment (Sec. 4): the plane is
    normal to the start direction ``a`` and lies 1 m behind the corner of
    ``box`` = (x0, y0, z0, x1, y1, z1) farthest from the sun; (u, v) is an
    orthonormal basis of it with u horizontal (u = z x a, or east when the
    sun is at the zenith).  The grid of ``texel``-sized squares covers the
    box's projections along ``a`` and ``b`` (every intermediate projection
    lies between them) with one texel of margin; texel (i, j) spans
    [u0 + i h, u0 + (i + 1) h) x [v0 + j h, v0 + (j + 1) h)."""
    a = np.asarray(a, np.float64) / np.linalg.norm(a)
    b = np.asarray(b, np.float64) / np.linalg.norm(b)
    h = float(texel)
    u = np.cross([0.0, 0.0, 1.0], a)
    u = u / np.linalg.norm(u) if np.linalg.norm(u) > 1e-9 else np.array([1.0, 0.0, 0.0])
    v = np.cross(a, u)
    x0, y0, z0, x1, y1, z1 = [float(t) for t in box]
    corners = np.array([[x, y, z] for x in (x0, x1) for y in (y0, y1) for z in (z0, z1)])
    c = float((corners @ a).min()) - 1.0
    pu, pv = [], []
    for d in (a, b):
        p = sam_project(corners, a, c, d)
        pu.append(p @ u)
        pv.append(p @ v)
    pu, pv = np.concatenate(pu), np.concatenate(pv)
    u0 = np.floor(pu.min() / h) * h - h
    v0 = np.floor(pv.min() / h) * h - h
    nu = int(np.ceil((pu.max() - u0) / h)) + 1
    nv = int(np.ceil((pv.max() - v0) / h)) + 1
    return dict(a=a, u=u, v=v, c=c, u0=u0, v0=v0, h=h, nu=nu, nv=nv)


def sam_project(x, a, c, d):
    """Where the shadow of x falls on the plane {y : y.a = c} for sun
    direction d: x - lam d with lam = (x.a - c) / (d.a), the distance along
    the light, which is the depth the map compares."""
    x = np.asarray(x, np.float64)
    lam = (x @ a - c) / float(np.dot(d, a))
    return x - lam[..., None] * d


def exit_depths(scene, X, d, grow=0.0):
    """Per ray X + lam d (lam >= 0; X [m, 3]): the largest lam at which it
    leaves a prism (the prism's face nearest the sun), -inf where it meets
    none; brute force over every prism in C (``orc_exit_depths``), the same
    steps as ``exit_depths_np``."""
    s, ks = _scene(scene)
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, np.float64)
    out = np.empty(len(X))
    if len(X):
        lib().orc_exit_depths(C.byref(s), len(X), _ptr(X, C.c_double), _ptr(d, C.c_double), float(grow),
                              _ptr(out, C.c_double), threads_default())
    return out


def exit_depths_np(scene, X, d, grow=0.0):
    """Per ray X + lam d (lam >= 0; X [m, 3] on the plane): the largest lam
    at which it leaves a prism (the prism's face nearest the sun), -inf where
    it meets none.  Each prism clipped as a convex solid (Cyrus-Beck): its
    height slab and the inner half-plane of every footprint edge, all moved
    outward by ``grow`` metres (negative: inward)."""
    m = len(X)
    best = np.full(m, -np.inf)
    for k in range(scene.n_b):
        f = scene.footprint(k).astype(np.float64)
        H = float(scene.height[k])
        lo = np.full(m, 0.0)
        hi = np.full(m, np.inf)
        # height slab -grow <= z <= H + grow (the sun is above the horizon: d_z > 0)
        lo = np.maximum(lo, (-grow - X[:, 2]) / d[2])
        hi = np.minimum(hi, (H + grow - X[:, 2]) / d[2])
        ok = np.ones(m, bool)
        for e in range(len(f)):
            p0, p1 = f[e], f[(e + 1) % len(f)]
            ex, ey = p1 - p0
            # inside: cross(e, x - p0) >= -grow |e|, along the ray f0 + lam g
            f0 = ex * (X[:, 1] - p0[1]) - ey * (X[:, 0] - p0[0]) + grow * np.hypot(ex, ey)
            g = ex * d[1] - ey * d[0]
            if g > 0:
                lo = np.maximum(lo, -f0 / g)
            elif g < 0:
                hi = np.minimum(hi, -f0 / g)
            else:
                ok &= f0 >= 0
        hit = ok & (lo <= hi)
        best = np.where(hit, np.maximum(best, hi), best)
    return best


def sam_segments(path: OraclePath):
    """Sample instants of each segment: an instant belongs to the segment
    whose [start, end) holds it, the day's last segment also taking its
    end.  Returns, per segment, the indices into the path's instants."""
    out = []
    for j in range(len(path.seg_t)):
        ta, tb = path.seg_t[j]
        day = path.seg_day[j]
        last = j + 1 == len(path.seg_t) or path.seg_day[j + 1] != day
        k = np.flatnonzero((path.sample_day == day) & (path.t >= ta) & ((path.t < tb) | (last & (path.t <= tb))))
        out.append(k)
    return out


def sam(scene, pts, path: OraclePath, texel, bias=0.01, box=None, eps_texel=2e-3, eps_depth=1e-2, delta=5e-3):
    """Gross shadow by shadow accrual maps (Sec. 4, Step 1 and Step 2), one
    map per segment with a slice per sample instant: slice k holds, per
    texel, the depth of the prisms' surface nearest the sun along the ray
    from the texel's centre in that instant's direction (the great-circle
    direction at the instant, as the accrual form assumes); a point is in
    shadow at instant k when that depth at the texel its shadow falls on
    exceeds its own depth by more than ``bias``.  ``box``: the region every
    prism lies in, (x0, y0, z0, x1, y1, z1); None = the footprints' extent,
    0 .. the tallest prism.

    Returns counts int32 and minutes FP64 [n_bins, n], the decisions
    ``shadowed`` uint8 [n, K], and a flag ``amb`` uint8 [n, K] marking
    (point, instant) decisions a float32 evaluation may take
    either way: the shadow within ``eps_texel`` texels of a texel edge, the
    depths within ``eps_depth`` m of the bias margin, or a decision that
    changes when every prism grows or shrinks by ``delta`` m."""
    if box is None:
        box = (scene.xy[:, 0].min(), scene.xy[:, 1].min(), 0.0,
               scene.xy[:, 0].max(), scene.xy[:, 1].max(), scene.height.max()) if scene.n_b else None
    n, K = pts.n, len(path.t)
    counts = np.zeros((path.n_bins, n), np.int32)
    minutes = np.zeros((path.n_bins, n), np.float64)
    amb = np.zeros((n, K), np.uint8)
    shadowed = np.zeros((n, K), np.uint8)
    if box is None or n == 0:
        return dict(counts=counts, minutes=minutes, shadowed=shadowed, amb=amb)
    Q = np.stack([pts.x, pts.y, pts.z], 1).astype(np.float64)
    for j, ks in enumerate(sam_segments(path)):
        a, b = path.seg_dir[j]
        ta, tb = path.seg_t[j]
        G = sam_grid(box, a, b, texel)
        for k in ks:
            d = slerp(a, b, (path.t[k] - ta) / (tb - ta)) if tb > ta else G["a"]
            lam = (Q @ G["a"] - G["c"]) / float(d @ G["a"])
            P = Q - lam[:, None] * d
            fu, fv = (P @ G["u"] - G["u0"]) / G["h"], (P @ G["v"] - G["v0"]) / G["h"]
            i, jj = np.floor(fu), np.floor(fv)
            inside = (i >= 0) & (i < G["nu"]) & (jj >= 0) & (jj < G["nv"])
            X = G["c"] * G["a"] + (G["u0"] + (i + 0.5) * G["h"])[:, None] * G["u"] + \
                (G["v0"] + (jj + 0.5) * G["h"])[:, None] * G["v"]
            dep = {g: np.where(inside, exit_depths(scene, X, d, g), -np.inf) for g in (0.0, delta, -delta)}
            s = dep[0.0] > lam + bias
            near_edge = np.minimum(np.minimum(fu - i, i + 1 - fu), np.minimum(fv - jj, jj + 1 - fv)) < eps_texel
            near_depth = np.abs(dep[0.0] - lam - bias) <= eps_depth
            unstable = (dep[delta] > lam + bias) != (dep[-delta] > lam + bias)
            amb[:, k] = near_edge | near_depth | unstable
            shadowed[:, k] = s
            b_ = path.sample_bin[k]
            counts[b_] += s
            minutes[b_] += s * path.w[k]
    return dict(counts=counts, minutes=minutes, shadowed=shadowed, amb=amb)
