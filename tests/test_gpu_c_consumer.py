"""The library used from plain C through its C ABI (tests/c_consumer.c):
the program's printed counts and minutes against the oracle on the same
scene, points and path."""
import datetime as dt
import os
import subprocess

import numpy as np
import pytest

import oracle
from workloads import Points, Scene, Span
from workloads.scenes import Day

from gpu_util import say

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def consumer_inputs():
    """The scene, points and span hard-coded in c_consumer.c."""
    xy = np.array([0, 0, 20, 0, 20, 20, 0, 20, 40, 0, 60, 0, 60, 30, 40, 30, 0, 50, 25, 50, 25, 70, 0, 70],
                  np.float32).reshape(-1, 2)
    scene = Scene(np.array([0, 4, 8, 12], np.int32), xy, np.array([30, 60, 15], np.float32))
    f = lambda v: np.array(v, np.float32)
    pts = Points(f([30, 10, 50, 70, 20, 50]), f([10, 35, 40, 10, 10, 30]), f([0, 0, 0, 0, 10, 20]),
                 f([0, 0, 0, 0, 1, 0]), f([0, 0, 0, 0, 0, 1]), np.array([-1, -1, -1, -1, 0, 1], np.int32))
    span = Span(40.7, -74.0, [Day(2019, 6, 21, -4.0)], 5.0)
    return scene, pts, span


def test_c_program_matches_oracle():
    exe = os.path.join(HERE, "_bin", "c_consumer")
    if not os.path.exists(exe):
        import c_consumer_build
        c_consumer_build.build()
    say("running the C consumer")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = [l.split() for l in r.stdout.strip().splitlines()]
    got = {form: (np.array([int(x[2]) for x in rows if x[0] == form]),
                  np.array([float(x[3]) for x in rows if x[0] == form])) for form in ("sampled", "accrual")}
    scene, pts, span = consumer_inputs()
    os_ = oracle.sampled(scene, pts, oracle.sun_path(span), amb=True)
    oa = oracle.continuous(scene, pts, oracle.sun_path(span, 30.0))
    w = oracle.sun_path(span).w
    slack = (os_["amb"].astype(bool) * w[None, :]).sum(1)
    say(f"sampled counts {got['sampled'][0]} vs oracle {os_['counts'][0]}; "
        f"accrual minutes {np.round(got['accrual'][1], 3)} vs oracle {np.round(oa['minutes'][0], 3)}")
    assert np.all(np.abs(got["sampled"][0] - os_["counts"][0]) <= os_["amb"].sum(1))
    assert np.all(np.abs(got["sampled"][1] - os_["minutes"][0]) <= slack + 1e-3)
    assert np.all(np.abs(got["accrual"][1] - oa["minutes"][0]) <= 0.01)
    assert (got["accrual"][1] > 1.0).sum() >= 3          # the scene shadows most points for a while
