"""Pins for the oracle's building contribution and shadow score (Sec. 7.2).
Contribution: each building's own shadow time on the points (weighted by
area), overlaps counted for every building.  Score: sum over points and
intervals of the interval's weight times the fraction of its daylight the
point spends in shadow, with the paper's month weights."""
import json
import os

import numpy as np

import oracle
from workloads import Span
from workloads.scenes import Day

from test_oracle_continuous_shadow import EAST, JUN21, WEST, middle_points
from test_oracle_shadow import GOLD, box_scene, pts

SPAN = Span(40.7, -74.0, [JUN21], step_min=1.0)


def test_single_building_contribution_is_its_shadow_time():
    p = middle_points()
    path = oracle.sun_path(SPAN, 30.0)
    w = np.linspace(0.5, 2.0, p.n)
    c = oracle.contribution(box_scene([WEST]), p, path, weight=w)
    m = oracle.continuous(box_scene([WEST]), p, path)["minutes"]
    assert c.shape == (1, 1)
    np.testing.assert_allclose(c[0, 0], (m[0] * w).sum(), rtol=1e-12)
    assert c[0, 0] > 100.0


def test_disjoint_shadows_add_up_and_match_each_alone():
    p = middle_points()
    path = oracle.sun_path(SPAN, 30.0)
    both = oracle.contribution(box_scene([WEST, EAST]), p, path)
    w_alone = oracle.continuous(box_scene([WEST]), p, path)["minutes"].sum()
    e_alone = oracle.continuous(box_scene([EAST]), p, path)["minutes"].sum()
    total = oracle.continuous(box_scene([WEST, EAST]), p, path)["minutes"].sum()
    np.testing.assert_allclose(both[0], [w_alone, e_alone], rtol=1e-12)
    np.testing.assert_allclose(both[0].sum(), total, rtol=1e-9)


def test_overlapping_shadows_count_for_both():
    # two boxes side by side west of the points shadow them at the same time
    p = middle_points()
    path = oracle.sun_path(SPAN, 30.0)
    a = (-40.0, -5.0, -30.0, 5.0, 30.0)
    b = (-52.0, -5.0, -42.0, 5.0, 60.0)
    c = oracle.contribution(box_scene([a, b]), p, path)
    total = oracle.continuous(box_scene([a, b]), p, path)["minutes"].sum()
    assert c[0, 0] > 0 and c[0, 1] > 0
    assert c[0].sum() > total + 10.0
    assert c[0].max() <= total + 1e-9


def test_far_building_contributes_nothing_and_weights_are_linear():
    p = middle_points()
    path = oracle.sun_path(SPAN, 30.0)
    far = (500.0, 500.0, 510.0, 510.0, 10.0)
    c1 = oracle.contribution(box_scene([WEST, far]), p, path)
    assert c1[0, 1] == 0.0
    c2 = oracle.contribution(box_scene([WEST, far]), p, path, weight=np.full(p.n, 2.0))
    np.testing.assert_allclose(c2, 2 * c1, rtol=1e-12)


def test_backfacing_wall_counts_for_its_own_building():
    # points on the north wall of a lone box, facing north: shadowed exactly
    # while the sun is south of the wall's plane
    sc = box_scene([(0.0, 0.0, 20.0, 10.0, 15.0)])
    p = pts([(5.0, 10.0, 2.0), (15.0, 10.0, 7.0)], nrm=[(0.0, 1.0), (0.0, 1.0)], owner=[0, 0])
    path = oracle.sun_path(SPAN, 30.0)
    c = oracle.contribution(sc, p, path)
    m = oracle.continuous(sc, p, path)["minutes"]
    np.testing.assert_allclose(c[0, 0], m.sum(), rtol=1e-12)
    assert 400.0 < m[0, 0] < 895.0


def _month_weights():
    with open(os.path.join(GOLD, "paper_table_month_weights.json")) as f:
        wt = json.load(f)["weights"]
    return np.array([wt[k] for k in ("Jan", "Feb", "Mar", "Apr", "May", "Jun", "Jul", "Aug", "Sep", "Oct",
                                     "Nov", "Dec")], np.float64)


def test_score_of_always_and_summer_only_shadow():
    """With the paper's month weights an always-shadowed point scores 0
    (the weights sum to zero) and one shadowed only in June-August scores
    3 per unit area; the fraction is per interval, so span lengths drop
    out."""
    w = _month_weights()
    span = np.array([600.0 + 20 * k for k in range(12)])      # any daylight per month
    always = span[:, None] * np.ones((1, 3))
    summer = np.zeros((12, 3))
    summer[5:8] = span[5:8, None]
    area = np.array([1.0, 2.0, 0.5])
    assert abs(oracle.shadow_score(always, w, span, area)) < 1e-12
    np.testing.assert_allclose(oracle.shadow_score(summer, w, span, area), 3.0 * area.sum())
    half = 0.5 * summer
    np.testing.assert_allclose(oracle.shadow_score(half, w, span, area), 1.5 * area.sum())
