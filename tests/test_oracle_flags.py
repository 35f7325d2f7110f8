"""Pins for the oracle's two ambiguity masks, with rays constructed at known
distances from a silhouette:

* the sampled form's silhouette band (a (point, instant) pair whose
  predicate changes within 1e-5 rad of its direction may go either way in
  float32; both answers are then correct): rays 2e-6 .. 9e-6 rad from a
  roof edge, a vertical edge and a wall's own plane must be flagged, rays
  1.5e-5 rad and farther must not, whatever the edge's orientation about the
  ray;
* the raster form's flags (Sec. 4 maps in float32): a point's shadow within
  2e-3 texel of a texel edge, an exit depth within 1 cm of the bias margin,
  and a texel-centre ray passing 2 mm from a wall must each be flagged;
  their counterparts a texel-half, metres and a metre away must not."""
import math

import numpy as np
import pytest

import oracle
from workloads import Points, Scene


def box_scene(boxes):
    xy = np.array([[(b[0], b[1]), (b[2], b[1]), (b[2], b[3]), (b[0], b[3])] for b in boxes],
                  np.float32).reshape(-1, 2)
    return Scene(np.arange(0, 4 * len(boxes) + 1, 4, dtype=np.int32), xy,
                 np.array([b[4] for b in boxes], np.float32))


def pts(xyz, nrm=None, owner=None):
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    n = len(xyz)
    nrm = np.zeros((n, 2), np.float32) if nrm is None else np.asarray(nrm, np.float32).reshape(-1, 2)
    own = np.full(n, -1, np.int32) if owner is None else np.asarray(owner, np.int32)
    return Points(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), nrm[:, 0].copy(), nrm[:, 1].copy(), own)


def dir_path(dirs, seg=None):
    """An oracle path holding the given instants (one bin, unit weights);
    ``seg``: one segment (a, b) spanning t in [0, 1], the instants at t = 0."""
    dirs = np.asarray(dirs, np.float64).reshape(-1, 3)
    K = len(dirs)
    z = np.zeros(K, np.int32)
    if seg is None:
        st, sd = np.zeros((0, 2)), np.zeros((0, 2, 3))
    else:
        st, sd = np.array([[0.0, 1.0]]), np.asarray(seg, np.float64).reshape(1, 2, 3)
    return oracle.OraclePath(dirs, np.ones(K), np.zeros(K), z, z, st, sd, np.zeros(len(st), np.int32),
                             np.zeros(1, np.int32), 1, np.array([[0.0, 1.0]]))


def turned(d0, axis, delta):
    """d0 turned by delta radians toward the unit vector axis (axis _|_ d0)."""
    return math.cos(delta) * d0 + math.sin(delta) * axis


NEAR = (2e-6, 5e-6, 9e-6)
FAR = (1.5e-5, 5e-5, 1e-3)


def _check_band(scene, P, d0, axis):
    """Turn d0 both ways toward axis: the predicate must differ between the
    two sides (d0 is on a silhouette), every near turn must be flagged and
    every far turn unflagged with its side's predicate."""
    side = {s: oracle.shadow(scene, (P.x[0], P.y[0], P.z[0]), turned(d0, axis, s * 1e-3),
                             (P.nx[0], P.ny[0]), int(P.owner[0])) for s in (-1, 1)}
    assert side[-1] != side[1]
    dirs = [turned(d0, axis, s * e) for e in NEAR + FAR for s in (-1, 1)]
    o = oracle.sampled(scene, P, dir_path(dirs), bits=True, amb=True)
    bits = np.unpackbits(o["bits"].view(np.uint8), axis=1, bitorder="little")[0, :len(dirs)]
    amb = o["amb"][0]
    k = 0
    for e in NEAR + FAR:
        for s in (-1, 1):
            if e in NEAR:
                assert amb[k] == 1, (e, s)
            else:
                assert amb[k] == 0, (e, s)
                assert bits[k] == side[s], (e, s)
            k += 1


def test_band_at_a_roof_edge():
    """A ray from a ground point grazing the north roof edge of a 20 m box."""
    sc = box_scene([(-5.0, -5.0, 5.0, 5.0, 20.0)])
    p = np.array([0.7, 30.0, 0.0])
    q = np.array([1.3, 5.0, 20.0])                   # on the roof edge y = 5, z = 20
    d0 = (q - p) / np.linalg.norm(q - p)
    axis = np.cross([1.0, 0.0, 0.0], q - p)          # normal of the plane through p and the edge
    _check_band(sc, pts([p]), d0, axis / np.linalg.norm(axis))


def test_band_at_a_vertical_edge():
    """A ray grazing the box's north-west vertical edge (a silhouette edge
    seen from the north-east) at mid height."""
    sc = box_scene([(-5.0, -5.0, 5.0, 5.0, 20.0)])
    p = np.array([20.0, 30.0, 0.0])
    q = np.array([-5.0, 5.0, 10.0])
    d0 = (q - p) / np.linalg.norm(q - p)
    axis = np.cross([0.0, 0.0, 1.0], q - p)
    _check_band(sc, pts([p]), d0, axis / np.linalg.norm(axis))


def test_band_at_a_wall_plane():
    """A facade point's wall faces away from the sun when n.d <= 0: rays
    within 1e-5 rad of the wall's plane are flagged."""
    sc = box_scene([(-5.0, -5.0, 5.0, 5.0, 20.0)])
    P = pts([[5.0, 0.0, 3.0]], nrm=[[1.0, 0.0]], owner=[0])
    e = math.radians(30.0)
    d0 = np.array([0.0, math.cos(e), math.sin(e)])   # in the wall's plane
    _check_band(sc, P, d0, np.array([1.0, 0.0, 0.0]))


def test_band_covers_every_edge_orientation():
    """The 8 turned directions sit 1.1e-5 rad from the ray at fixed
    azimuths about it; whatever the edge's orientation among them, a ray
    within 1e-5 rad of a roof edge must be flagged, and one 1.3e-5 to
    4e-5 rad away must not.  60 random points and edge positions."""
    sc = box_scene([(-5.0, -5.0, 5.0, 5.0, 20.0)])
    rng = np.random.default_rng(3)
    for _ in range(60):
        p = np.array([rng.uniform(-40, 40), rng.uniform(15, 60), rng.uniform(0, 15)])
        q = np.array([rng.uniform(-4.5, 4.5), 5.0, 20.0])
        d0 = (q - p) / np.linalg.norm(q - p)
        axis = np.cross([1.0, 0.0, 0.0], q - p)
        axis /= np.linalg.norm(axis)
        s = rng.choice([-1.0, 1.0])
        o = oracle.sampled(sc, pts([p]), dir_path([turned(d0, axis, s * rng.uniform(1e-6, 1e-5)),
                                                  turned(d0, axis, s * rng.uniform(1.3e-5, 4e-5))]), amb=True)
        assert o["amb"][0, 0] == 1 and o["amb"][0, 1] == 0


# --------------------------------------------------------------------------
# raster form (Sec. 4)
# --------------------------------------------------------------------------
E = math.radians(40.0)
A = np.array([0.0, -math.cos(E), math.sin(E)])        # sun due south, 40 degrees up
B = np.array([-math.sin(0.05) * math.cos(E), -math.cos(0.05) * math.cos(E), math.sin(E)])
BOX = (-50.0, -50.0, 0.0, 50.0, 50.0, 60.0)
TEX = 1.0


def _grid():
    G = oracle.sam_grid(BOX, A, B, TEX)
    # the plane basis for a sun due south: u = east, v = (0, sin e, cos e)
    np.testing.assert_allclose(G["u"], [1.0, 0.0, 0.0], atol=1e-12)
    return G


def _ground_point(G, fu, fv):
    """A ground point whose shadow falls at texel coordinates (fu, fv):
    P.u = x and P.v = y sin e for a ground point when the sun is due south."""
    return np.array([G["u0"] + fu * G["h"], (G["v0"] + fv * G["h"]) / math.sin(E), 0.0])


def _sam_flag(scene, q):
    o = oracle.sam(scene, pts([q]), dir_path([A], seg=(A, B)), TEX, box=BOX)
    return int(o["amb"][0, 0]), int(o["shadowed"][0, 0])


FAR_BOX = (30.0, 30.0, 40.0, 40.0, 10.0)


def test_raster_flag_near_a_texel_edge():
    G = _grid()
    sc = box_scene([FAR_BOX])
    assert _sam_flag(sc, _ground_point(G, 50 + 1e-4, 40.5)) == (1, 0)
    assert _sam_flag(sc, _ground_point(G, 50 + 0.5, 40 + 1e-3)) == (1, 0)
    assert _sam_flag(sc, _ground_point(G, 50.5, 40.5)) == (0, 0)
    assert _sam_flag(sc, _ground_point(G, 50.02, 40.98)) == (0, 0)


def test_raster_flag_near_the_depth_margin():
    """A prism around the point: the texel-centre ray (through the point, at
    a texel's middle) leaves its roof at height H, a depth H / sin e past the
    point; flagged when that is within 1 cm of the 1 cm bias."""
    G = _grid()
    q = _ground_point(G, 50.5, 40.5)
    around = lambda h: box_scene([(q[0] - 3.0, q[1] - 3.0, q[0] + 3.0, q[1] + 3.0, h), FAR_BOX])
    # 9 mm past the margin: within 1 cm of it, yet 5 mm of growth or
    # shrinkage (7.8 mm of depth) does not change the decision
    near_h = (0.01 + 0.009) * math.sin(E)
    assert _sam_flag(around(near_h), q) == (1, 1)
    assert _sam_flag(around(2.0), q) == (0, 1)       # deep inside: shadowed, unambiguous


def test_raster_flag_when_a_wall_is_grazed():
    """A 50 m box south of the point whose west wall the texel-centre ray
    passes 2 mm away from: growing the prisms by 5 mm makes it a hit,
    shrinking them does not, so the decision is flagged; 1 m away it is
    not."""
    G = _grid()
    q = _ground_point(G, 50.5, 40.5)
    wall = lambda gap: box_scene([(q[0] + gap, q[1] - 30.0, q[0] + 10.0, q[1] - 5.0, 50.0), FAR_BOX])
    assert _sam_flag(wall(0.002), q) == (1, 0)
    assert _sam_flag(wall(-0.002), q) == (1, 1)
    assert _sam_flag(wall(1.0), q) == (0, 0)
    assert _sam_flag(wall(-1.0), q) == (0, 1)
