"""Python binding of libsa, the gfx950 shadow-accumulation library.

Argument marshalling only: every step of the computation runs in the HIP
library (``libsa.so``, built in-tree by ``build.py``).  PyTorch provides
device memory and streams.  The names mirror the C ABI declared in
``include/shadow_accrual.h``; the small classes own library handles.

There is no fallback: if ``libsa.so`` is missing or no HIP device is
present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsa.so")

SA_OK = 0
SA_SAMPLED = 0
SA_ACCRUAL = 1
SA_FLAG_ADD = 1
_ERRORS = {-1: "INVALID_ARG", -2: "GEOMETRY", -3: "CAPACITY", -4: "OOM", -5: "DEVICE", -6: "UNSUPPORTED"}

# Every entry point declared in include/shadow_accrual.h.
EXPORTS = ["sa_create", "sa_destroy", "sa_set_stream", "sa_set_launch", "sa_get_launch", "sa_last_error", "sa_sync",
           "sa_version", "sa_measure_valu_peak",
           "sa_scene_upload", "sa_scene_set_heights", "sa_scene_get_info", "sa_scene_read_bvh",
           "sa_scene_destroy", "sa_sunpath", "sa_path_upload", "sa_path_upload_graph", "sa_path_info", "sa_path_destroy",
           "sa_accumulate", "sa_accumulate_noalloc", "sa_accumulate_batched", "sa_grad_heights", "sa_region_sum",
           "sa_building_contribution", "sa_path_bin_span", "sa_region_score", "sa_sam_accumulate"]


class SAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class sa_site(C.Structure):
    _fields_ = [("lat_deg", C.c_double), ("lon_deg", C.c_double), ("tz_offset_h", C.c_double)]


class sa_timespan(C.Structure):
    _fields_ = [("year", C.c_int32), ("month", C.c_int32), ("day", C.c_int32), ("n_days", C.c_int32),
                ("t_start_min", C.c_double), ("t_end_min", C.c_double), ("step_min", C.c_double),
                ("seg_min", C.c_double), ("knot_clock", C.c_int32)]


class sa_sunpath_buf(C.Structure):
    _fields_ = [("n_days", C.c_int32), ("n_samples", C.c_int32), ("n_knots", C.c_int32),
                ("cap_days", C.c_int32), ("cap_samples", C.c_int32), ("cap_knots", C.c_int32),
                ("day_sample_off", C.c_void_p), ("t_min", C.c_void_p), ("dir", C.c_void_p),
                ("weight", C.c_void_p), ("day_knot_off", C.c_void_p), ("knot_t", C.c_void_p),
                ("knot_dir", C.c_void_p), ("day_bin", C.c_void_p)]


class sa_scene_info(C.Structure):
    _fields_ = [("n_b", C.c_int32), ("n_vert", C.c_int32), ("n_nodes", C.c_int32), ("depth", C.c_int32),
                ("bounds", C.c_float * 4), ("max_height", C.c_float)]


class sa_points(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("nx", C.c_void_p), ("ny", C.c_void_p), ("owner", C.c_void_p)]


class sa_sam_opts(C.Structure):
    _fields_ = [("texel_m", C.c_float), ("bias_m", C.c_float), ("box", C.c_float * 6), ("flags", C.c_uint32),
                ("out_scale", C.c_float), ("max_texels", C.c_int64)]


class sa_launch(C.Structure):
    _fields_ = [("accrual_segments_per_launch", C.c_int32), ("batched_grid_blocks", C.c_int32),
                ("batched_tiles_per_grab", C.c_int32), ("tile_grid_blocks", C.c_int32),
                ("accrual_waves_per_simd", C.c_int32), ("sampled_instants_per_packet", C.c_int32),
                ("reserved", C.c_int32 * 2)]


class sa_accum_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("flags", C.c_uint32), ("out_scale", C.c_float),
                ("grid_blocks", C.c_int32), ("work", C.c_void_p), ("longest", C.c_void_p),
                ("minutes64", C.c_void_p)]


_lib = None


def lib():
    """Load libsa.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1907_04435_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "sa_create": (i32, [i32, vp, C.POINTER(vp)]),
            "sa_destroy": (None, [vp]),
            "sa_set_stream": (i32, [vp, vp]),
            "sa_set_launch": (i32, [vp, C.POINTER(sa_launch)]),
            "sa_get_launch": (i32, [vp, C.POINTER(sa_launch)]),
            "sa_last_error": (C.c_char_p, [vp]),
            "sa_sync": (i32, [vp]),
            "sa_version": (C.c_char_p, []),
            "sa_measure_valu_peak": (i32, [vp, C.POINTER(C.c_double)]),
            "sa_scene_upload": (i32, [vp, i32, vp, vp, vp, C.POINTER(vp)]),
            "sa_scene_set_heights": (i32, [vp, vp, i32, vp, vp]),
            "sa_scene_get_info": (i32, [vp, C.POINTER(sa_scene_info)]),
            "sa_scene_read_bvh": (i32, [vp, vp, vp, vp]),
            "sa_scene_destroy": (None, [vp]),
            "sa_sunpath": (i32, [C.POINTER(sa_site), C.POINTER(sa_timespan), C.POINTER(sa_sunpath_buf)]),
            "sa_path_upload": (i32, [vp, C.POINTER(sa_sunpath_buf), C.POINTER(vp)]),
            "sa_path_upload_graph": (i32, [vp, C.POINTER(sa_sunpath_buf), C.c_double, C.POINTER(vp)]),
            "sa_path_info": (i32, [vp, vp, vp, vp]),
            "sa_path_destroy": (None, [vp]),
            "sa_accumulate": (i32, [vp, vp, C.POINTER(sa_points), vp, C.POINTER(sa_accum_opts), vp, vp, vp]),
            "sa_accumulate_noalloc": (i32, [vp, vp, C.POINTER(sa_points), vp, C.POINTER(sa_accum_opts), vp, vp,
                                            vp]),
            "sa_accumulate_batched": (i32, [vp, vp, i32, i32, vp, vp, C.POINTER(sa_points), vp, vp,
                                            C.POINTER(sa_accum_opts), vp, vp]),
            "sa_grad_heights": (i32, [vp, vp, C.POINTER(sa_points), vp, C.POINTER(sa_accum_opts), vp, vp]),
            "sa_region_sum": (i32, [vp, vp, i64, vp, i32, vp, vp]),
            "sa_building_contribution": (i32, [vp, vp, C.POINTER(sa_points), vp, vp, vp]),
            "sa_sam_accumulate": (i32, [vp, vp, C.POINTER(sa_points), vp, C.POINTER(sa_sam_opts), vp, vp]),
            "sa_path_bin_span": (i32, [vp, vp]),
            "sa_region_score": (i32, [vp, vp, vp, i64, vp, vp, i32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    """Device (torch) or host (numpy) buffer -> address; None -> NULL."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _check(ctx, rc):
    if rc != SA_OK:
        msg = lib().sa_last_error(ctx.handle if ctx is not None else None)
        raise SAError(rc, msg.decode() if msg else "")


# --------------------------------------------------------------------------
# sun path (host)
# --------------------------------------------------------------------------
@dataclass
class SunPath:
    """Host arrays of a sun path (see sa_sunpath_buf)."""
    day_sample_off: np.ndarray
    t_min: np.ndarray
    dir: np.ndarray
    weight: np.ndarray
    day_knot_off: np.ndarray
    knot_t: np.ndarray
    knot_dir: np.ndarray
    day_bin: np.ndarray

    @property
    def n_days(self):
        return len(self.day_bin)

    @property
    def n_samples(self):
        return len(self.t_min)

    @property
    def n_bins(self):
        return int(self.day_bin.max()) + 1 if len(self.day_bin) else 0


def sa_sunpath(lat, lon, tz_h, year, month, day, n_days=1, t_start=-1.0, t_end=-1.0, step=1.0,
               seg=30.0, clock_knots=False) -> SunPath:
    """Sample instants and great-circle knots of ``n_days`` consecutive days
    (t_start < 0: sunrise..sunset whole minutes); ``clock_knots``: inner
    knots at the multiples of ``seg`` in local time (days share knot
    times) instead of every ``seg`` minutes from each day's first instant."""
    L = lib()
    site = sa_site(lat, lon, tz_h)
    span = sa_timespan(year, month, day, n_days, t_start, t_end, step, seg, 1 if clock_knots else 0)
    buf = sa_sunpath_buf()
    rc = L.sa_sunpath(C.byref(site), C.byref(span), C.byref(buf))
    if rc != SA_OK:
        raise SAError(rc, "sa_sunpath sizing failed")
    D, K, J = buf.n_days, buf.n_samples, buf.n_knots
    a = dict(day_sample_off=np.zeros(D + 1, np.int32), t_min=np.zeros(K), dir=np.zeros(3 * K),
             weight=np.zeros(K), day_knot_off=np.zeros(D + 1, np.int32), knot_t=np.zeros(J),
             knot_dir=np.zeros(3 * J), day_bin=np.zeros(D, np.int32))
    buf = sa_sunpath_buf(0, 0, 0, D, K, J, *[a[k].ctypes.data for k in
                                             ("day_sample_off", "t_min", "dir", "weight", "day_knot_off",
                                              "knot_t", "knot_dir", "day_bin")])
    rc = L.sa_sunpath(C.byref(site), C.byref(span), C.byref(buf))
    if rc != SA_OK:
        raise SAError(rc, "sa_sunpath failed")
    a["dir"] = a["dir"].reshape(-1, 3)
    a["knot_dir"] = a["knot_dir"].reshape(-1, 3)
    return SunPath(**a)


def concat_paths(paths, day_bin=None) -> SunPath:
    """Concatenate per-day paths (e.g. separate dates) into one."""
    so, ko, ns, nk = [0], [0], 0, 0
    for p in paths:
        so += list(np.asarray(p.day_sample_off[1:]) + ns)
        ko += list(np.asarray(p.day_knot_off[1:]) + nk)
        ns += p.n_samples
        nk += len(p.knot_t)
    D = len(so) - 1
    db = np.arange(D, dtype=np.int32) if day_bin is None else np.asarray(day_bin, np.int32)
    return SunPath(np.array(so, np.int32), np.concatenate([p.t_min for p in paths]),
                   np.concatenate([p.dir for p in paths]), np.concatenate([p.weight for p in paths]),
                   np.array(ko, np.int32), np.concatenate([p.knot_t for p in paths]),
                   np.concatenate([p.knot_dir for p in paths]), db)


def sunpath_for_span(span, seg_min: float, clock_knots=False) -> SunPath:
    """Library sun path for a ``workloads.Span`` (one call per day, bins as
    the span says)."""
    paths = []
    for d in span.days:
        t0, t1 = (d.window if d.window is not None else (-1.0, -1.0))
        paths.append(sa_sunpath(span.lat, span.lon, d.tz_h, d.year, d.month, d.day, 1, t0, t1,
                                span.step_min, seg_min, clock_knots))
    return concat_paths(paths, span.day_bin)


# --------------------------------------------------------------------------
# objects
# --------------------------------------------------------------------------
class Context:
    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: libsa needs an MI355X (gfx950)")
        self.device = device
        self.torch = torch
        s = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = lib().sa_create(device, C.c_void_p(s.cuda_stream), C.byref(h))
        if rc != SA_OK:
            raise SAError(rc, "sa_create failed")
        self.handle = h
        self.stream = s

    def set_stream(self, stream):
        self.stream = stream
        _check(self, lib().sa_set_stream(self.handle, C.c_void_p(stream.cuda_stream)))

    def sync(self):
        _check(self, lib().sa_sync(self.handle))

    def set_launch(self, accrual_segments_per_launch=0, batched_grid_blocks=0, batched_tiles_per_grab=0,
                   tile_grid_blocks=0, accrual_waves_per_simd=0, sampled_instants_per_packet=0):
        """Launch choices (speed only; see sa_set_launch)."""
        l = sa_launch(int(accrual_segments_per_launch), int(batched_grid_blocks), int(batched_tiles_per_grab),
                      int(tile_grid_blocks), int(accrual_waves_per_simd), int(sampled_instants_per_packet))
        _check(self, lib().sa_set_launch(self.handle, C.byref(l)))

    def measure_valu_peak(self) -> float:
        """FP32 lane-ops per second the device's vector ALUs sustain
        (sa_measure_valu_peak; a roofline measurement aid)."""
        v = C.c_double(0.0)
        _check(self, lib().sa_measure_valu_peak(self.handle, C.byref(v)))
        return float(v.value)

    def get_launch(self) -> dict:
        l = sa_launch()
        _check(self, lib().sa_get_launch(self.handle, C.byref(l)))
        return {k: getattr(l, k) for k, _ in sa_launch._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "handle", None):
            lib().sa_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_or_device(a, np_dtype, torch_dtype):
    """(pointer, object to keep alive, length) of a flat array: a numpy
    array (host) or a device tensor, converted to the given element type."""
    if getattr(a, "is_cuda", False):
        t = a.to(torch_dtype).contiguous().reshape(-1)
        return C.c_void_p(t.data_ptr()), t, int(t.numel())
    h = np.ascontiguousarray(a, np_dtype).reshape(-1)
    return _ptr(h), h, len(h)


class Scene:
    """Prisms uploaded from host arrays or device tensors (vert_off int32
    [n_b + 1], xy float32 [V, 2] or [2V], height float32 [n_b])."""

    def __init__(self, ctx: Context, vert_off, xy, height):
        import torch
        self.ctx = ctx
        pv, kv, _ = _host_or_device(vert_off, np.int32, torch.int32)
        px, kx, _ = _host_or_device(xy, np.float32, torch.float32)
        ph, kh, n_b = _host_or_device(height, np.float32, torch.float32)
        hd = C.c_void_p()
        _check(ctx, lib().sa_scene_upload(ctx.handle, n_b, pv, px, ph, C.byref(hd)))
        del kv, kx, kh
        self.handle = hd
        self.n_b = n_b

    @classmethod
    def from_workload(cls, ctx, scene):
        return cls(ctx, scene.vert_off, scene.xy, scene.height)

    def set_heights(self, ids, h):
        """Host arrays (checked and applied synchronously) or device tensors
        (both; applied on the context's stream, bad entries reported by
        sync)."""
        if getattr(ids, "is_cuda", False) or getattr(h, "is_cuda", False):
            import torch
            ids = ids.to(device=h.device, dtype=torch.int32).contiguous()
            h = h.to(torch.float32).contiguous()
            self._keep = (ids, h)   # alive until the stream has read them
            _check(self.ctx, lib().sa_scene_set_heights(self.ctx.handle, self.handle, int(ids.numel()),
                                                        _ptr(ids), _ptr(h)))
            return
        ids = np.ascontiguousarray(ids, np.int32)
        h = np.ascontiguousarray(h, np.float32)
        _check(self.ctx, lib().sa_scene_set_heights(self.ctx.handle, self.handle, len(ids), _ptr(ids), _ptr(h)))

    def info(self) -> dict:
        i = sa_scene_info()
        _check(self.ctx, lib().sa_scene_get_info(self.handle, C.byref(i)))
        return dict(n_b=i.n_b, n_vert=i.n_vert, n_nodes=i.n_nodes, depth=i.depth,
                    bounds=list(i.bounds), max_height=i.max_height)

    def read_bvh(self):
        inf = self.info()
        nodes = np.zeros((max(inf["n_nodes"], 0), 16), np.int32)
        order = np.zeros(max(self.n_b, 0), np.int32)
        _check(self.ctx, lib().sa_scene_read_bvh(self.ctx.handle, self.handle, _ptr(nodes), _ptr(order)))
        return nodes, order

    def close(self):
        if getattr(self, "handle", None):
            lib().sa_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Path:
    """A sun path on the device.  ``graph_bound_deg``: merge the accrual
    form's segments into direction-graph edges with cells of that size
    (sa_path_upload_graph); None keeps every segment."""

    def __init__(self, ctx: Context, sp: SunPath, graph_bound_deg: float | None = None):
        self.ctx = ctx
        self.host = sp
        keep = [np.ascontiguousarray(sp.day_sample_off, np.int32), np.ascontiguousarray(sp.t_min, np.float64),
                np.ascontiguousarray(sp.dir, np.float64).reshape(-1), np.ascontiguousarray(sp.weight, np.float64),
                np.ascontiguousarray(sp.day_knot_off, np.int32), np.ascontiguousarray(sp.knot_t, np.float64),
                np.ascontiguousarray(sp.knot_dir, np.float64).reshape(-1), np.ascontiguousarray(sp.day_bin, np.int32)]
        buf = sa_sunpath_buf(sp.n_days, sp.n_samples, len(sp.knot_t), sp.n_days, sp.n_samples, len(sp.knot_t),
                             *[k.ctypes.data for k in keep])
        h = C.c_void_p()
        if graph_bound_deg is None:
            _check(ctx, lib().sa_path_upload(ctx.handle, C.byref(buf), C.byref(h)))
        else:
            _check(ctx, lib().sa_path_upload_graph(ctx.handle, C.byref(buf), float(graph_bound_deg), C.byref(h)))
        self.handle = h
        nb, ns, nseg = C.c_int32(), C.c_int32(), C.c_int32()
        _check(ctx, lib().sa_path_info(h, C.byref(nb), C.byref(ns), C.byref(nseg)))
        self.n_bins, self.n_samples, self.n_segments = nb.value, ns.value, nseg.value

    def bin_span(self) -> np.ndarray:
        """Daylight minutes of every output bin (host float64)."""
        out = np.zeros(self.n_bins, np.float64)
        rc = lib().sa_path_bin_span(self.handle, out.ctypes.data)
        if rc != 0:
            raise SAError(rc, "sa_path_bin_span failed")
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().sa_path_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DevicePoints:
    """Sample points as device float32 / int32 tensors (structure of arrays)."""

    def __init__(self, x, y, z, nx=None, ny=None, owner=None):
        self.x, self.y, self.z, self.nx, self.ny, self.owner = x, y, z, nx, ny, owner
        self.n = int(x.numel())

    @classmethod
    def from_workload(cls, pts, device="cuda"):
        import torch
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(f(pts.x), f(pts.y), f(pts.z), f(pts.nx), f(pts.ny),
                   torch.from_numpy(np.ascontiguousarray(pts.owner, np.int32)).to(device))

    @classmethod
    def ground_from_workload(cls, pts, device="cuda"):
        """Positions only, for the raster form (which takes ground-type
        points); refuses points with an owner or a facade normal."""
        import torch
        if np.any(pts.owner >= 0) or np.any(pts.nx != 0) or np.any(pts.ny != 0):
            raise ValueError("ground-type points only (no owner, no facade normal)")
        f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(f(pts.x), f(pts.y), f(pts.z))

    def struct(self) -> sa_points:
        return sa_points(self.n, _ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.nx), _ptr(self.ny),
                         _ptr(self.owner))


# --------------------------------------------------------------------------
# compute entry points
# --------------------------------------------------------------------------
def sa_accumulate(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, mode: int, counts=None,
                  minutes=None, bits=None, flags=0, out_scale=1.0, work=None, longest=None, minutes64=None):
    """Gross shadow into caller-provided device tensors (see the C ABI).
    ``work``: optional device int64 [8] work counters (instrumented run).
    ``longest``: optional device float32 [bins, n] continuous shadow.
    ``minutes64``: optional device float64 [bins, n] accrual minutes before
    their rounding to float32."""
    opts = sa_accum_opts(mode, flags, out_scale, 0, _ptr(work), _ptr(longest), _ptr(minutes64))
    ps = pts.struct()
    _check(ctx, lib().sa_accumulate(ctx.handle, scene.handle, C.byref(ps), path.handle, C.byref(opts),
                                    _ptr(counts), _ptr(minutes), _ptr(bits)))


def sa_accumulate_noalloc(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, mode: int, counts=None,
                          minutes=None, bits=None, flags=0, out_scale=1.0, work=None, longest=None, minutes64=None):
    """sa_accumulate without any allocation inside the call (the library's
    fixed per-device scratch; see the C ABI): for callers that cannot
    allocate."""
    opts = sa_accum_opts(mode, flags, out_scale, 0, _ptr(work), _ptr(longest), _ptr(minutes64))
    ps = pts.struct()
    _check(ctx, lib().sa_accumulate_noalloc(ctx.handle, scene.handle, C.byref(ps), path.handle, C.byref(opts),
                                            _ptr(counts), _ptr(minutes), _ptr(bits)))


def accumulate(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, mode: int, want_counts=True,
               want_bits=False, out_scale=1.0):
    """Allocate outputs and run sa_accumulate: returns (counts [bins, n] int32
    or None, minutes [bins, n] float32, bits [words, n] int32 or None)."""
    torch = ctx.torch
    dev = f"cuda:{ctx.device}"
    counts = torch.empty((path.n_bins, pts.n), dtype=torch.int32, device=dev) if want_counts else None
    minutes = torch.empty((path.n_bins, pts.n), dtype=torch.float32, device=dev)
    bits = torch.empty(((path.n_samples + 31) // 32, pts.n), dtype=torch.int32, device=dev) if want_bits else None
    sa_accumulate(ctx, scene, pts, path, mode, counts, minutes, bits, 0, out_scale)
    return counts, minutes, bits


def continuous_shadow(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, mode: int, out_scale=1.0):
    """Gross and continuous shadow in one pass: returns (minutes [bins, n],
    longest [bins, n]) float32 device tensors; longest is the longest
    uninterrupted shadow of a day, maximum over the bin's days."""
    torch = ctx.torch
    dev = f"cuda:{ctx.device}"
    minutes = torch.empty((path.n_bins, pts.n), dtype=torch.float32, device=dev)
    longest = torch.empty((path.n_bins, pts.n), dtype=torch.float32, device=dev)
    sa_accumulate(ctx, scene, pts, path, mode, None, minutes, None, 0, out_scale, longest=longest)
    return minutes, longest


def sa_accumulate_batched(ctx: Context, scene: Scene, var_ids, var_h, pts: DevicePoints, var_off, path: Path,
                          counts=None, minutes=None, flags=0, out_scale=1.0, grid_blocks=0):
    """Batched development variants (device tensors var_ids [V, k] int32,
    var_h [V, k] float32, var_off [V+1] int64).  ``grid_blocks``: size of
    the persistent launch (0 = library default)."""
    opts = sa_accum_opts(SA_ACCRUAL, flags, out_scale, grid_blocks, None, None, None)
    ps = pts.struct()
    V, k = int(var_ids.shape[0]), int(var_ids.shape[1]) if var_ids.dim() > 1 else 0
    _check(ctx, lib().sa_accumulate_batched(ctx.handle, scene.handle, V, k, _ptr(var_ids), _ptr(var_h),
                                            C.byref(ps), _ptr(var_off), path.handle, C.byref(opts),
                                            _ptr(counts), _ptr(minutes)))


def sa_grad_heights(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, dl_dmin, grad, flags=0,
                    out_scale=1.0):
    """d(sum dl_dmin * minutes * out_scale)/dH into device float grad [n_b]
    (SA_FLAG_ADD in flags adds into it)."""
    opts = sa_accum_opts(SA_ACCRUAL, flags, out_scale, 0, None, None, None)
    ps = pts.struct()
    _check(ctx, lib().sa_grad_heights(ctx.handle, scene.handle, C.byref(ps), path.handle, C.byref(opts),
                                      _ptr(dl_dmin), _ptr(grad)))


def sa_building_contribution(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, weight, contrib):
    ps = pts.struct()
    _check(ctx, lib().sa_building_contribution(ctx.handle, scene.handle, C.byref(ps), path.handle, _ptr(weight),
                                               _ptr(contrib)))


def sa_sam_accumulate(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, texel, counts=None, minutes=None,
                      bias=0.01, box=None, flags=0, out_scale=1.0, max_texels=0):
    """Gross shadow by raster shadow accrual maps (Sec. 4) into device
    outputs [bins, n]; ``box``: (x0, y0, z0, x1, y1, z1) holding every prism
    (None: the scene's own extent)."""
    b = (C.c_float * 6)(*([0.0] * 6 if box is None else [float(v) for v in box]))
    opts = sa_sam_opts(float(texel), float(bias), b, flags, out_scale, int(max_texels))
    ps = pts.struct()
    _check(ctx, lib().sa_sam_accumulate(ctx.handle, scene.handle, C.byref(ps), path.handle, C.byref(opts),
                                        _ptr(counts), _ptr(minutes)))


def sam_accumulate(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, texel, bias=0.01, box=None):
    """Allocate outputs and run sa_sam_accumulate: (counts int32, minutes
    float32), both [bins, n]."""
    torch = ctx.torch
    dev = f"cuda:{ctx.device}"
    counts = torch.empty((path.n_bins, pts.n), dtype=torch.int32, device=dev)
    minutes = torch.empty((path.n_bins, pts.n), dtype=torch.float32, device=dev)
    sa_sam_accumulate(ctx, scene, pts, path, texel, counts, minutes, bias=bias, box=box)
    return counts, minutes


def building_contribution(ctx: Context, scene: Scene, pts: DevicePoints, path: Path, weight=None):
    """Per bin and building (original ids) the weighted minutes the points
    spend in that building's own shadow: device float64 [bins, n_b]."""
    torch = ctx.torch
    out = torch.empty((path.n_bins, scene.n_b), dtype=torch.float64, device=f"cuda:{ctx.device}")
    sa_building_contribution(ctx, scene, pts, path, weight, out)
    return out


def sa_region_score(ctx: Context, path: Path, values, interval_weight, region_off, out, area=None):
    w = np.ascontiguousarray(interval_weight, np.float64)
    if len(w) != path.n_bins:
        raise ValueError("one interval weight per bin of the path")
    _check(ctx, lib().sa_region_score(ctx.handle, path.handle, _ptr(values), int(values.shape[1]), _ptr(w),
                                      _ptr(region_off), int(region_off.numel()) - 1, _ptr(area), _ptr(out)))


def shadow_score(ctx: Context, path: Path, values, interval_weight, region_off, area=None):
    """Shadow score of regions (Sec. 7.2) from per-bin shadow minutes
    ``values`` [bins, n] and one weight in [-1, 1] per bin: returns device
    float64 [n_regions]."""
    torch = ctx.torch
    out = torch.empty(int(region_off.numel()) - 1, dtype=torch.float64, device=values.device)
    sa_region_score(ctx, path, values, interval_weight, region_off, out, area)
    return out


def sa_region_sum(ctx: Context, values, region_off, out, area=None):
    _check(ctx, lib().sa_region_sum(ctx.handle, _ptr(values), int(values.numel()), _ptr(region_off),
                                    int(region_off.numel()) - 1, _ptr(area), _ptr(out)))


def shadow_minutes_fn():
    """torch.autograd.Function: heights [n_b] -> accrual minutes [bins, n];
    backward runs the adjoint kernel (sa_grad_heights)."""
    import torch

    class ShadowMinutes(torch.autograd.Function):
        @staticmethod
        def forward(fctx, heights, sactx, scene, pts, path):
            # heights stay on the device: written and refitted on the stream
            h = heights.detach().to(device=f"cuda:{sactx.device}", dtype=torch.float32).contiguous()
            ids = getattr(scene, "_all_ids", None)
            if ids is None or ids.numel() != scene.n_b:
                ids = torch.arange(scene.n_b, dtype=torch.int32, device=h.device)
                scene._all_ids = ids
            scene.set_heights(ids, h)
            minutes = torch.empty((path.n_bins, pts.n), dtype=torch.float32, device=f"cuda:{sactx.device}")
            sa_accumulate(sactx, scene, pts, path, SA_ACCRUAL, None, minutes)
            fctx.objs = (sactx, scene, pts, path)
            return minutes

        @staticmethod
        def backward(fctx, grad_out):
            sactx, scene, pts, path = fctx.objs
            grad = torch.empty(scene.n_b, dtype=torch.float32, device=f"cuda:{sactx.device}")
            sa_grad_heights(sactx, scene, pts, path, grad_out.contiguous().float(), grad)
            return grad, None, None, None, None

    return ShadowMinutes
