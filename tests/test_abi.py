"""Host-side checks of the C-ABI library: it loads, exports every entry
point its header declares, and its host sun path agrees with the oracle's
(two independent implementations of the same published solar equations)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_1907_04435_amd as sa
from workloads import make_c1, Span
from workloads.scenes import Day

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            txt = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(sa_[a-z_]+)\s*\(", txt, re.M))
    return names


def test_header_declares_the_binding_exports():
    assert declared_symbols() == set(sa.EXPORTS)


def test_library_loads_and_exports_every_symbol():
    L = ctypes.CDLL(sa.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert b"gfx950" in sa.lib().sa_version()


def test_sunpath_sizes_year():
    p = sa.sa_sunpath(40.7, -74.0, -5.0, 2019, 1, 1, 365)
    assert p.n_days == 365 and p.n_samples == 263858
    assert np.all(np.diff(p.day_sample_off) >= 545)
    np.testing.assert_allclose(np.linalg.norm(p.dir, axis=1), 1.0, atol=1e-14)
    assert np.all(p.dir[:, 2] > 0)


@pytest.mark.parametrize("seg", [1.0, 30.0, 60.0])
@pytest.mark.parametrize("clock", [False, True])
def test_sunpath_matches_oracle(seg, clock):
    c1 = make_c1()
    spans = [c1.span, Span(40.7, -74.0, [Day(2019, 3, 20, -4.0), Day(2019, 6, 21, -4.0), Day(2019, 12, 21, -5.0)]),
             Span(40.7, -74.0, [Day(2019, 6, 21, -4.0, (7 * 60 + 13.5, 17 * 60 + 2.0))], 0.5)]
    for span in spans:
        lp = sa.sunpath_for_span(span, seg, clock_knots=clock)
        op = oracle.sun_path(span, seg, clock_knots=clock)
        assert lp.n_samples == len(op.w)
        np.testing.assert_allclose(lp.dir, op.dirs, atol=1e-12)
        np.testing.assert_array_equal(lp.t_min, op.t)
        np.testing.assert_allclose(lp.weight, op.w, atol=1e-12)
        # knots: each day's consecutive pairs are the oracle's segments
        segs_t, segs_d = [], []
        for d in range(lp.n_days):
            k0, k1 = lp.day_knot_off[d], lp.day_knot_off[d + 1]
            for k in range(k0, k1 - 1):
                segs_t.append((lp.knot_t[k], lp.knot_t[k + 1]))
                segs_d.append((lp.knot_dir[k], lp.knot_dir[k + 1]))
        np.testing.assert_array_equal(np.array(segs_t), op.seg_t)
        np.testing.assert_allclose(np.array(segs_d), op.seg_dir, atol=1e-12)


def test_clock_knots_fall_on_the_clock():
    """With clock knots every inner knot is a multiple of the spacing in
    local time, the first and last are the day's first and last instants,
    and two days share their inner knot times wherever both are in
    daylight."""
    p = sa.sa_sunpath(40.7, -74.0, -4.0, 2019, 6, 20, 2, step=1.0, seg=30.0, clock_knots=True)
    days = [p.knot_t[p.day_knot_off[d]:p.day_knot_off[d + 1]] for d in range(2)]
    for d, kt in enumerate(days):
        s = p.t_min[p.day_sample_off[d]:p.day_sample_off[d + 1]]
        assert kt[0] == s[0] and kt[-1] == s[-1]
        assert np.all(np.mod(kt[1:-1], 30.0) == 0.0) and np.all(np.diff(kt) > 0)
    assert len(set(days[0][1:-1]) & set(days[1][1:-1])) >= len(days[0]) - 3


def test_sunpath_rejects_night_window():
    with pytest.raises(sa.SAError):
        sa.sa_sunpath(40.7, -74.0, -4.0, 2019, 6, 21, 1, 100.0, 1000.0, 5.0, 30.0)


def test_context_needs_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a HIP device is present")
    with pytest.raises(RuntimeError):
        sa.Context(0)


def test_c_consumer_links_against_the_library():
    """tests/c_consumer.c, a plain C99 program using only the header (built
    with -Wall -Wextra -Werror by the build step), links against libsa.so
    and the HIP runtime, and every shared library it needs resolves."""
    import subprocess
    exe = os.path.join(ROOT, "tests", "_bin", "c_consumer")
    if not os.path.exists(exe):
        import c_consumer_build
        c_consumer_build.build()
    r = subprocess.run(["ldd", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "libsa.so" in r.stdout and "not found" not in r.stdout, r.stdout
