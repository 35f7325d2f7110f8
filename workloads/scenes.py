"""Seeded synthetic city scenes in the shape of the paper's Manhattan workload.

The paper measures on OpenStreetMap Manhattan (about 43k buildings, 1.5M
triangles; Sec. 8.2), which is not available here.  These generators stand
in for it: extruded convex footprints on a Manhattan-like block grid with
18 m streets, long-tailed (lognormal) heights, and ground / facade sample
points on a 1 m lattice, at 40.7 N, -74.0 E.

Everything is deterministic from a numpy ``default_rng(seed)`` (PCG64).
Coordinates are metres in a local east-north-up frame (x east, y north,
z up), stored as float32.  Footprints are convex and counter-clockwise;
prisms stand on z = 0.

Robustness choices that keep the sampled-form parity check well posed:
ground points keep a margin of at least ``GROUND_MARGIN`` from every
footprint boundary they are not inside of, and the small axis-aligned scene
keeps every box edge at least 1 cm from the lattice lines, so no sample
point sits within float32 rounding of a wall.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import datetime as _dt

import numpy as np

NYC = dict(lat=40.7, lon=-74.0)
GROUND_MARGIN = 0.05  # metres between an open-space point and any footprint


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Scene:
    vert_off: np.ndarray  # int32 [n_b + 1]
    xy: np.ndarray        # float32 [V, 2]
    height: np.ndarray    # float32 [n_b]

    @property
    def n_b(self) -> int:
        return int(self.height.shape[0])

    def footprint(self, b: int) -> np.ndarray:
        return self.xy[self.vert_off[b]:self.vert_off[b + 1]]

    def subset(self, ids: np.ndarray) -> "Scene":
        ids = np.asarray(ids, dtype=np.int64)
        m = (self.vert_off[ids + 1] - self.vert_off[ids]).astype(np.int64)
        off = np.zeros(len(ids) + 1, dtype=np.int64)
        off[1:] = np.cumsum(m)
        xy = np.concatenate([self.footprint(int(b)) for b in ids]) if len(ids) else np.zeros((0, 2), np.float32)
        return Scene(off.astype(np.int32), np.ascontiguousarray(xy, dtype=np.float32),
                     self.height[ids].astype(np.float32).copy())

    def centroids(self) -> np.ndarray:
        c = np.zeros((self.n_b, 2))
        m = np.diff(self.vert_off)
        idx = np.repeat(np.arange(self.n_b), m)
        np.add.at(c, idx, self.xy.astype(np.float64))
        return c / m[:, None]


@dataclass
class Points:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    owner: np.ndarray  # int32, -1 for ground points

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def take(self, idx) -> "Points":
        idx = np.asarray(idx)
        return Points(*(np.ascontiguousarray(a[idx]) for a in
                        (self.x, self.y, self.z, self.nx, self.ny, self.owner)))


@dataclass
class Day:
    year: int
    month: int
    day: int
    tz_h: float                  # local civil time = UTC + tz_h
    window: tuple | None = None  # (start_min, end_min) local, or None = sunrise..sunset


@dataclass
class Span:
    lat: float
    lon: float
    days: list
    step_min: float = 1.0
    day_bin: list | None = None  # output bin of each day (None: one bin per day)

    @property
    def n_bins(self) -> int:
        return len(self.days) if self.day_bin is None else int(max(self.day_bin)) + 1


@dataclass
class Workload:
    name: str
    scene: Scene
    points: Points
    span: Span
    extra: dict = field(default_factory=dict)


def _pts(x, y, z=None, nx=None, ny=None, owner=None) -> Points:
    n = len(x)
    f = lambda a, v=0.0: (np.full(n, v, np.float32) if a is None else np.asarray(a, np.float32))
    return Points(f(x), f(y), f(z), f(nx), f(ny),
                  np.full(n, -1, np.int32) if owner is None else np.asarray(owner, np.int32))


def concat_points(parts) -> Points:
    if not parts:
        return _pts(np.zeros(0), np.zeros(0))
    return Points(*(np.concatenate([getattr(p, k) for p in parts]) for k in
                    ("x", "y", "z", "nx", "ny", "owner")))


def subset_points(pts: Points, n: int, seed: int) -> np.ndarray:
    """Indices of a seeded random subset (sorted) of ``n`` points."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(pts.n, size=min(n, pts.n), replace=False))


def _morton2(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0xFFFFFFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
        return v
    return spread(ix) | (spread(iy) << np.uint64(1))


# --------------------------------------------------------------------------
# C1: 64 axis-aligned boxes on a 512 x 512 m site, 128 x 128 ground lattice
# --------------------------------------------------------------------------
def make_c1(seed: int = 1) -> Workload:
    """Small scene: 64 boxes, footprints U(20,60) m, heights U(10,150) m,
    >= 1 m gaps, 128x128 ground points at 4 m spacing (roof-covered ones
    kept), 2019-06-21 08:00-18:00 EDT at 5-minute steps (121 instants)."""
    rng = np.random.default_rng(seed)
    site, n_box, lattice = 512.0, 64, np.arange(128) * 4.0 + 2.0
    boxes = []

    def near_lattice(v):
        return np.min(np.abs(lattice - v)) < 0.01

    tries = 0
    while len(boxes) < n_box:
        tries += 1
        if tries > 2_000_000:
            raise RuntimeError("box placement did not converge")
        w, d = rng.uniform(20.0, 60.0, size=2)
        cx = rng.uniform(w / 2, site - w / 2)
        cy = rng.uniform(d / 2, site - d / 2)
        x0, x1, y0, y1 = (np.float32(cx - w / 2), np.float32(cx + w / 2),
                          np.float32(cy - d / 2), np.float32(cy + d / 2))
        if any(near_lattice(float(v)) for v in (x0, x1, y0, y1)):
            continue
        ok = all(x0 >= b[1] + 1.0 or x1 <= b[0] - 1.0 or y0 >= b[3] + 1.0 or y1 <= b[2] - 1.0
                 for b in boxes)
        if ok:
            boxes.append((float(x0), float(x1), float(y0), float(y1)))
    h = rng.uniform(10.0, 150.0, size=n_box).astype(np.float32)
    xy = np.array([[(b[0], b[2]), (b[1], b[2]), (b[1], b[3]), (b[0], b[3])] for b in boxes],
                  dtype=np.float32).reshape(-1, 2)
    scene = Scene(np.arange(0, 4 * n_box + 1, 4, dtype=np.int32), xy, h)
    gx, gy = np.meshgrid(lattice, lattice, indexing="xy")
    pts = _pts(gx.ravel(), gy.ravel())
    span = Span(NYC["lat"], NYC["lon"], [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=5.0)
    return Workload("c1_boxes64_grid128_jun21_5min", scene, pts, span)


# --------------------------------------------------------------------------
# Manhattan-like generator (C2..C5)
# --------------------------------------------------------------------------
BLOCK_W, BLOCK_D, STREET = 80.0, 270.0, 18.0
PARCEL_W, PARCEL_D = 40.0, 27.0


def _manhattan(rng, cols, rows, n_keep, median_h, sigma_ln=1.0,
               cleared_blocks=None):
    """Convex footprints on a block grid.  Each block holds 2 x 10 parcels of
    40 x 27 m; ``n_keep`` parcels (seeded subset) carry one convex polygon of
    4..12 vertices at sorted random angles on an ellipse whose semi-axes are
    (parcel half-size - 1 m) x U(0.6, 1).  Heights lognormal (median
    ``median_h``, sigma_ln), clipped to [3, 400] m."""
    pc, pr = np.meshgrid(np.arange(cols * 2), np.arange(rows * 10), indexing="xy")
    pc, pr = pc.ravel(), pr.ravel()
    bc, br = pc // 2, pr // 10
    keep_ok = np.ones(pc.shape, bool)
    if cleared_blocks is not None:
        c0, c1, r0, r1 = cleared_blocks
        keep_ok &= ~((bc >= c0) & (bc < c1) & (br >= r0) & (br < r1))
    cand = np.flatnonzero(keep_ok)
    if n_keep > len(cand):
        raise ValueError("more parcels requested than exist")
    sel = np.sort(rng.choice(cand, size=n_keep, replace=False))
    pc, pr, bc, br = pc[sel], pr[sel], bc[sel], br[sel]
    px0 = bc * (BLOCK_W + STREET) + (pc % 2) * PARCEL_W
    py0 = br * (BLOCK_D + STREET) + (pr % 10) * PARCEL_D
    cx, cy = px0 + PARCEL_W / 2, py0 + PARCEL_D / 2
    ax = (PARCEL_W / 2 - 1.0) * rng.uniform(0.6, 1.0, n_keep)
    ay = (PARCEL_D / 2 - 1.0) * rng.uniform(0.6, 1.0, n_keep)
    m = rng.integers(4, 13, n_keep)
    off = np.zeros(n_keep + 1, np.int64)
    off[1:] = np.cumsum(m)
    xy = np.zeros((off[-1], 2), np.float64)
    for b in range(n_keep):
        mb = int(m[b])
        min_gap = np.pi / (2 * mb)
        while True:  # angles sorted, no two closer than min_gap (no sliver edges)
            a = np.sort(rng.uniform(0.0, 2 * np.pi, mb))
            gaps = np.diff(np.concatenate([a, a[:1] + 2 * np.pi]))
            if gaps.min() >= min_gap:
                break
        xy[off[b]:off[b + 1], 0] = cx[b] + ax[b] * np.cos(a)
        xy[off[b]:off[b + 1], 1] = cy[b] + ay[b] * np.sin(a)
    h = np.clip(median_h * np.exp(sigma_ln * rng.standard_normal(n_keep)), 3.0, 400.0)
    extent = (cols * BLOCK_W + (cols - 1) * STREET, rows * BLOCK_D + (rows - 1) * STREET)
    return Scene(off.astype(np.int32), xy.astype(np.float32), h.astype(np.float32)), extent


def _footprint_bboxes(scene: Scene):
    lo = np.minimum.reduceat(scene.xy.astype(np.float64), scene.vert_off[:-1], axis=0)
    hi = np.maximum.reduceat(scene.xy.astype(np.float64), scene.vert_off[:-1], axis=0)
    return lo, hi


def _blocked_cells(scene: Scene, x0: int, y0: int, nx: int, ny: int, margin: float):
    """Boolean [ny, nx] mask of lattice cells (centres at x0+i+0.5, y0+j+0.5)
    that lie inside a footprint or within ``margin`` of one (half-plane
    offset of each convex footprint)."""
    mask = np.zeros((ny, nx), bool)
    lo, hi = _footprint_bboxes(scene)
    X1, Y1 = x0 + nx, y0 + ny
    hit = np.flatnonzero((hi[:, 0] + margin > x0) & (lo[:, 0] - margin < X1) &
                         (hi[:, 1] + margin > y0) & (lo[:, 1] - margin < Y1))
    for b in hit:
        v = scene.footprint(int(b)).astype(np.float64)
        i0 = max(int(np.floor(lo[b, 0] - margin - x0 - 0.5)), 0)
        i1 = min(int(np.ceil(hi[b, 0] + margin - x0 - 0.5)) + 1, nx)
        j0 = max(int(np.floor(lo[b, 1] - margin - y0 - 0.5)), 0)
        j1 = min(int(np.ceil(hi[b, 1] + margin - y0 - 0.5)) + 1, ny)
        if i0 >= i1 or j0 >= j1:
            continue
        gx, gy = np.meshgrid(x0 + np.arange(i0, i1) + 0.5, y0 + np.arange(j0, j1) + 0.5)
        inside = np.ones(gx.shape, bool)
        e = np.roll(v, -1, axis=0) - v
        ln = np.hypot(e[:, 0], e[:, 1])
        for k in range(len(v)):  # outward normal (e_y, -e_x) of a CCW polygon
            sd = ((gx - v[k, 0]) * e[k, 1] - (gy - v[k, 1]) * e[k, 0]) / ln[k]
            inside &= sd <= margin
        mask[j0:j1, i0:i1] |= inside
    return mask


def _open_mask(scene, extent, margin=GROUND_MARGIN):
    """Open-space mask of every 1 m lattice cell of the scene extent."""
    nx, ny = int(np.floor(extent[0])), int(np.floor(extent[1]))
    return ~_blocked_cells(scene, 0, 0, nx, ny, margin)


def _open_lattice(scene, centre, n, extent, margin=GROUND_MARGIN, region=None, mask=None):
    """The ``n`` open-space 1 m lattice cell centres nearest ``centre`` in
    Chebyshev distance (ties by y then x), inside the scene extent (and
    inside the convex polygon ``region`` if given).  Returned in Morton
    order of the cell indices.  ``mask``: precomputed ``_open_mask``."""
    cx, cy = centre
    r = int(np.ceil(np.sqrt(n) / 2)) + 8
    X, Y = int(np.floor(extent[0])), int(np.floor(extent[1]))
    while True:
        x0, y0 = max(int(np.floor(cx - r)), 0), max(int(np.floor(cy - r)), 0)
        x1, y1 = min(int(np.ceil(cx + r)), X), min(int(np.ceil(cy + r)), Y)
        nx, ny = x1 - x0, y1 - y0
        if mask is not None:
            ok = mask[y0:y1, x0:x1].copy()
        else:
            ok = ~_blocked_cells(scene, x0, y0, nx, ny, margin)
        gx, gy = np.meshgrid(x0 + np.arange(nx) + 0.5, y0 + np.arange(ny) + 0.5)
        if region is not None:
            ok &= _in_convex(region, gx, gy)
        cheb = np.maximum(np.abs(gx - cx), np.abs(gy - cy))
        ok &= cheb <= r
        cnt = int(ok.sum())
        full = x0 == 0 and y0 == 0 and x1 >= X and y1 >= Y
        if cnt >= n or full:
            break
        r = int(r * 1.25) + 4
    if cnt < n:
        raise ValueError(f"only {cnt} open cells available, {n} requested")
    fx, fy, fc = gx[ok], gy[ok], cheb[ok]
    order = np.lexsort((fx, fy, fc))[:n]
    fx, fy = fx[order], fy[order]
    mort = _morton2(np.floor(fx).astype(np.int64), np.floor(fy).astype(np.int64))
    o2 = np.argsort(mort, kind="stable")
    return fx[o2], fy[o2]


def _region_points(mask, poly, centre, n):
    """The ``n`` open cells inside convex ``poly`` nearest ``centre``
    (Chebyshev, ties by y then x), Morton order; None if fewer exist."""
    Y, X = mask.shape
    x0, y0 = max(int(np.floor(poly[:, 0].min())), 0), max(int(np.floor(poly[:, 1].min())), 0)
    x1, y1 = min(int(np.ceil(poly[:, 0].max())) + 1, X), min(int(np.ceil(poly[:, 1].max())) + 1, Y)
    if x1 <= x0 or y1 <= y0:
        return None
    gx, gy = np.meshgrid(x0 + np.arange(x1 - x0) + 0.5, y0 + np.arange(y1 - y0) + 0.5)
    ok = mask[y0:y1, x0:x1] & _in_convex(poly, gx, gy)
    if int(ok.sum()) < n:
        return None
    fx, fy = gx[ok], gy[ok]
    fc = np.maximum(np.abs(fx - centre[0]), np.abs(fy - centre[1]))
    order = np.lexsort((fx, fy, fc))[:n]
    fx, fy = fx[order], fy[order]
    o2 = np.argsort(_morton2(np.floor(fx).astype(np.int64), np.floor(fy).astype(np.int64)), kind="stable")
    return fx[o2], fy[o2]


def _in_convex(poly, gx, gy):
    v = np.asarray(poly, np.float64)
    e = np.roll(v, -1, axis=0) - v
    inside = np.ones(np.shape(gx), bool)
    for k in range(len(v)):
        inside &= (e[k, 0] * (gy - v[k, 1]) - e[k, 1] * (gx - v[k, 0])) >= 0.0
    return inside


def _facade_points(scene: Scene, centre, n):
    """1 m x 1 m wall-cell centres with outward normal and owner id, for
    buildings in increasing centroid distance from ``centre``, truncated to
    ``n``.  Per wall edge of length l: floor(l) columns at (j+0.5) m along
    the edge; floor(H) rows at z = k + 0.5."""
    cen = scene.centroids()
    order = np.argsort(np.hypot(cen[:, 0] - centre[0], cen[:, 1] - centre[1]), kind="stable")
    xs, ys, zs, nxs, nys, own = [], [], [], [], [], []
    total = 0
    for b in order:
        v = scene.footprint(int(b)).astype(np.float64)
        e = np.roll(v, -1, axis=0) - v
        ln = np.hypot(e[:, 0], e[:, 1])
        rows = int(np.floor(scene.height[b]))
        if rows == 0:
            continue
        zk = np.arange(rows) + 0.5
        for k in range(len(v)):
            cols = int(np.floor(ln[k]))
            if cols == 0:
                continue
            u = e[k] / ln[k]
            t = np.arange(cols) + 0.5
            px = np.repeat(v[k, 0] + t * u[0], rows)
            py = np.repeat(v[k, 1] + t * u[1], rows)
            pz = np.tile(zk, cols)
            xs.append(px); ys.append(py); zs.append(pz)
            nxs.append(np.full(px.shape, u[1])); nys.append(np.full(px.shape, -u[0]))
            own.append(np.full(px.shape, b, np.int32))
            total += px.size
        if total >= n:
            break
    cat = lambda a: np.concatenate(a)[:n]
    return _pts(cat(xs), cat(ys), cat(zs), cat(nxs), cat(nys), cat(own))


def _sunrise_days(dates, tz_fn):
    return [Day(d.year, d.month, d.day, tz_fn(d), None) for d in dates]


def _nyc_tz(d: _dt.date) -> float:
    """US Eastern civil offset in 2019: EDT from Mar 10 to Nov 2 inclusive."""
    return -4.0 if _dt.date(2019, 3, 10) <= d < _dt.date(2019, 11, 3) else -5.0


def make_c2(seed: int = 2, n_ground: int = 2_000_000, n_facade: int = 2_000_000) -> Workload:
    """Manhattan-like block scene: 18 x 60 blocks of 80 x 270 m, 18 m
    streets, 20,000 convex prisms (4..12 vertices, lognormal heights,
    median 20 m); 2M open-space ground + 2M facade points at 1 m;
    2019-03-20, 06-21, 12-21 sunrise..sunset at 1-minute steps."""
    rng = np.random.default_rng(seed)
    scene, extent = _manhattan(rng, 18, 60, 20_000, 20.0)
    centre = (extent[0] / 2, extent[1] / 2)
    parts = []
    if n_ground:
        gx, gy = _open_lattice(scene, centre, n_ground, extent)
        parts.append(_pts(gx, gy))
    if n_facade:
        parts.append(_facade_points(scene, centre, n_facade))
    pts = concat_points(parts)
    days = _sunrise_days([_dt.date(2019, 3, 20), _dt.date(2019, 6, 21), _dt.date(2019, 12, 21)], _nyc_tz)
    span = Span(NYC["lat"], NYC["lon"], days, step_min=1.0)
    return Workload("c2_manhattan20k_4Mpts_3days_1min", scene, pts, span,
                    extra=dict(extent=extent, n_ground=n_ground, n_facade=n_facade))


def make_c3(seed: int = 3, n_var: int = 256, n_per_var=None, scene_seed: int = 2) -> Workload:
    """Batched development scenarios on the C2 scene: per variant a random
    convex 8-gon park region holding N_v = round(10**U(4, 5.699)) open-space
    points (10k..500k), and 8 distinct buildings with centroid within 300 m
    of the region redrawn to U(50, 500) m.  Jun 21 and Dec 21, 1-minute
    steps, accrual form.  ``n_per_var`` overrides every N_v (test sizes)."""
    rng = np.random.default_rng(seed)
    scene, extent = _manhattan(np.random.default_rng(scene_seed), 18, 60, 20_000, 20.0)
    cen = scene.centroids()
    mask = _open_mask(scene, extent)
    parts, off, var_ids, var_h = [], [0], [], []
    for v in range(n_var):
        nv = int(round(10 ** rng.uniform(4.0, 5.699))) if n_per_var is None else int(n_per_var)
        # region: 8 vertices at sorted angles on an ellipse, sized to hold >= nv open cells
        ang = np.sort(rng.uniform(0, 2 * np.pi, 8))
        aspect = rng.uniform(0.5, 1.0)
        c = np.array([rng.uniform(150, extent[0] - 150), rng.uniform(500, extent[1] - 500)])
        rad = np.sqrt(nv / (0.5 * np.pi * aspect)) * 1.1 + 5
        poly = np.stack([c[0] + rad * np.cos(ang), c[1] + rad * aspect * np.sin(ang)], 1)
        while True:
            got = _region_points(mask, poly, c, nv)
            if got is not None:
                gx, gy = got
                break
            poly = c + (poly - c) * 1.25
        parts.append(_pts(gx, gy))
        off.append(off[-1] + nv)
        d = np.maximum(np.abs(cen[:, 0] - c[0]) - (poly[:, 0].max() - c[0]), 0) ** 2 + \
            np.maximum(np.abs(cen[:, 1] - c[1]) - (poly[:, 1].max() - c[1]), 0) ** 2
        near = np.flatnonzero(d <= 300.0 ** 2)
        if len(near) < 8:
            near = np.argsort(d)[:8]
        ids = np.sort(rng.choice(near, 8, replace=False))
        var_ids.append(ids.astype(np.int32))
        var_h.append(rng.uniform(50.0, 500.0, 8).astype(np.float32))
    pts = concat_points(parts)
    days = _sunrise_days([_dt.date(2019, 6, 21), _dt.date(2019, 12, 21)], _nyc_tz)
    span = Span(NYC["lat"], NYC["lon"], days, step_min=1.0)
    return Workload("c3_variants256_jun21_dec21", scene, pts, span,
                    extra=dict(var_off=np.array(off, np.int64), var_ids=np.stack(var_ids),
                               var_h=np.stack(var_h), extent=extent))


def make_c4(seed: int = 4, n_park: int = 200_000, n_build: int = 5_000) -> Workload:
    """Differentiation scene: C2 generator with median height 30 m and a
    cleared 4 x 2 block park (374 x 558 m) at the centre; the ``n_park``
    open lattice points nearest the park centre and the ``n_build``
    buildings nearest it; Mar 20 sunrise..sunset, 1-minute steps."""
    rng = np.random.default_rng(seed)
    cols, rows = 18, 60
    c0, r0 = cols // 2 - 2, rows // 2 - 1
    full, extent = _manhattan(rng, cols, rows, 20_000, 30.0, cleared_blocks=(c0, c0 + 4, r0, r0 + 2))
    px0, py0 = c0 * (BLOCK_W + STREET), r0 * (BLOCK_D + STREET)
    park = (px0, py0, px0 + 4 * BLOCK_W + 3 * STREET, py0 + 2 * BLOCK_D + STREET)
    pc = ((park[0] + park[2]) / 2, (park[1] + park[3]) / 2)
    cen = full.centroids()
    near = np.sort(np.argsort(np.hypot(cen[:, 0] - pc[0], cen[:, 1] - pc[1]), kind="stable")[:n_build])
    scene = full.subset(near)
    poly = np.array([[park[0], park[1]], [park[2], park[1]], [park[2], park[3]], [park[0], park[3]]])
    gx, gy = _open_lattice(scene, pc, n_park, extent, region=poly)
    days = _sunrise_days([_dt.date(2019, 3, 20)], _nyc_tz)
    span = Span(NYC["lat"], NYC["lon"], days, step_min=1.0)
    return Workload("c4_park200k_build5k_mar20", scene, _pts(gx, gy), span,
                    extra=dict(park=park, extent=extent))


def make_c5(seed: int = 5, n_ground: int = 16_000_000, n_days: int = 365) -> Workload:
    """Year-long accumulation: 35 x 76 blocks (3,412 x 21,870 m), 45,000
    prisms, ``n_ground`` open-space points, every day of 2019 sunrise..sunset
    at 1-minute steps, four meteorological season bins (DJF, MAM, JJA,
    SON)."""
    rng = np.random.default_rng(seed)
    scene, extent = _manhattan(rng, 35, 76, 45_000, 20.0)
    centre = (extent[0] / 2, extent[1] / 2)
    gx, gy = _open_lattice(scene, centre, n_ground, extent, mask=_open_mask(scene, extent))
    dates = [_dt.date(2019, 1, 1) + _dt.timedelta(days=i) for i in range(n_days)]
    season = [{12: 0, 1: 0, 2: 0, 3: 1, 4: 1, 5: 1, 6: 2, 7: 2, 8: 2}.get(d.month, 3) for d in dates]
    span = Span(NYC["lat"], NYC["lon"], _sunrise_days(dates, _nyc_tz), step_min=1.0, day_bin=season)
    return Workload("c5_year_45k_16Mpts_seasons", scene, _pts(gx, gy), span, extra=dict(extent=extent))
