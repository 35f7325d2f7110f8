"""Pins for the oracle's continuous shadow (Sec. 3.1: the longest time a
point stays in shadow without interruption; over several days, the maximum
over the days), in both forms: the longest run of consecutive shadowed
instants (sampled, Sec. 5's n-bit vectors) and the longest member of a
day's shadowed set along the great-circle path (accrual)."""
import json
import os

import numpy as np

import oracle
from workloads import Span
from workloads.scenes import Day

from test_oracle_shadow import GOLD, box_scene, pts

JUN21 = Day(2019, 6, 21, -4.0, None)
MAR20 = Day(2019, 3, 20, -4.0, None)


def unit_path(K):
    """K instants of one minute each in one day and one bin."""
    return oracle.OraclePath(np.zeros((K, 3)), np.ones(K), np.arange(float(K)), np.zeros(K, np.int32),
                             np.zeros(K, np.int32), np.zeros((0, 2)), np.zeros((0, 2, 3)), np.zeros(0, np.int32),
                             np.zeros(1, np.int32), 1, np.array([[0.0, K - 1.0]]))


def test_fig2_longest_runs():
    """The paper's example: bit vectors [1,1,1], [0,1,1], [1,0,1] have
    continuous shadow 3, 2 and 1 minutes."""
    with open(os.path.join(GOLD, "paper_fig2_shadow_types.json")) as f:
        g = json.load(f)["points"]
    names = sorted(g)
    bits = np.array([g[k]["bits"] for k in names], bool)
    got = oracle.longest_sampled(bits, unit_path(3))[0]
    for k, v in zip(names, got):
        assert v == g[k]["continuous_min"]
        assert bits[names.index(k)].sum() == g[k]["gross_min"]


def test_longest_run_is_the_longest_not_the_sum():
    # runs of 2, 4 and 1 minutes in one day: continuous 4, gross 7
    bits = np.array([[1, 1, 0, 1, 1, 1, 1, 0, 0, 1]], bool)
    assert oracle.longest_sampled(bits, unit_path(10))[0, 0] == 4.0


WEST = (-40.0, -5.0, -30.0, 5.0, 30.0)    # shadows the points east of it in the afternoon
EAST = (30.0, -5.0, 40.0, 5.0, 30.0)      # ... and this one in the morning


def middle_points():
    x, y = np.meshgrid(np.linspace(-20.0, 20.0, 9), np.linspace(-3.0, 3.0, 4))
    return pts(np.stack([x.ravel(), y.ravel(), np.zeros(x.size)], 1))


def test_single_passage_longest_equals_gross():
    """West of the points, a box shadows them only in the afternoon, while
    the sun's azimuth sweeps monotonically through the box's azimuth range:
    one uninterrupted passage, so continuous = gross."""
    span = Span(40.7, -74.0, [JUN21], step_min=1.0)
    r = oracle.continuous(box_scene([WEST]), middle_points(), oracle.sun_path(span, 30.0))
    assert (r["minutes"] > 1.0).mean() > 0.5
    np.testing.assert_allclose(r["longest"], r["minutes"], rtol=0, atol=1e-9)


def test_two_passages_longest_is_the_larger():
    """Boxes east and west: a morning and an afternoon passage.  Gross adds
    them; continuous shadow is the larger of the two single-box results."""
    span = Span(40.7, -74.0, [JUN21], step_min=1.0)
    path = oracle.sun_path(span, 30.0)
    p = middle_points()
    both = oracle.continuous(box_scene([WEST, EAST]), p, path)
    w = oracle.continuous(box_scene([WEST]), p, path)
    e = oracle.continuous(box_scene([EAST]), p, path)
    two = (w["minutes"] > 1.0) & (e["minutes"] > 1.0)
    assert two.mean() > 0.3
    np.testing.assert_allclose(both["minutes"], w["minutes"] + e["minutes"], atol=1e-8)
    np.testing.assert_allclose(both["longest"], np.maximum(w["longest"], e["longest"]), atol=1e-8)
    assert np.all(both["longest"][two] < both["minutes"][two])


def test_several_days_take_the_maximum():
    p = middle_points()
    sc = box_scene([WEST, EAST])
    sep = oracle.continuous(sc, p, oracle.sun_path(Span(40.7, -74.0, [MAR20, JUN21], 1.0), 30.0))
    one = oracle.continuous(sc, p, oracle.sun_path(Span(40.7, -74.0, [MAR20, JUN21], 1.0, day_bin=[0, 0]), 30.0))
    np.testing.assert_allclose(one["minutes"][0], sep["minutes"].sum(0), atol=1e-8)
    np.testing.assert_allclose(one["longest"][0], sep["longest"].max(0), atol=1e-12)


def test_roof_covered_point_is_shadowed_all_day():
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (480.0, 1080.0))], step_min=5.0)
    r = oracle.continuous(box_scene([(0, 0, 10, 10, 20.0)]), pts([(5.0, 5.0, 0.0)]), oracle.sun_path(span, 30.0))
    assert r["longest"][0, 0] == 600.0 and r["minutes"][0, 0] == 600.0


def test_sampled_longest_converges_to_continuous():
    """One-minute instants against the continuous set (knots every minute):
    a passage of k shadowed instants weighs k minutes, the continuous
    passage lasts between k - 1 and k + 1 minutes."""
    span = Span(40.7, -74.0, [JUN21], step_min=1.0)
    sc, p = box_scene([WEST]), middle_points()
    path = oracle.sun_path(span, 1.0)
    s = oracle.sampled(sc, p, path, bits=True)
    K = len(path.w)
    sh = np.array([[(int(s["bits"][i, k >> 5]) >> (k & 31)) & 1 for k in range(K)] for i in range(p.n)], bool)
    ls = oracle.longest_sampled(sh, path)
    lc = oracle.continuous(sc, p, path)["longest"]
    assert (lc > 10.0).mean() > 0.5
    assert np.abs(ls - lc).max() <= 1.0 + 1e-6
