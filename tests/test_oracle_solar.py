"""Pins for the oracle's solar position and day sampling.

The oracle's ephemeris is checked against things other than itself:
textbook worked examples (Meeus), the paper's own Table 1, an independent
published approximation (Spencer 1971), and astronomical invariants.
"""
import datetime as dt
import json
import math
import os

import numpy as np
import pytest

import oracle
from workloads.scenes import Day

GOLD = os.path.join(os.path.dirname(__file__), "golden")
LAT, LON = 40.7, -74.0


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_julian_day_meeus():
    g = gold("meeus_example_7a.json")
    for y, m, d, jd in g["cases"]:
        assert oracle.julian_day(y, m, d) == pytest.approx(jd, abs=1e-6)


def test_solar_coordinates_meeus_example_25a():
    g = gold("meeus_example_25a.json")
    s = oracle.solar_jd(g["jde"], LAT, LON)
    tol = g["tolerance_deg"]
    assert s[7] == pytest.approx(g["apparent_longitude_deg"], abs=tol)
    assert s[5] == pytest.approx(g["declination_deg"], abs=tol)
    assert s[8] == pytest.approx(g["true_obliquity_deg"], abs=tol)


def _spencer(doy, hour_utc):
    """Spencer (1971) Fourier series for declination (rad) and equation of
    time (min): an independent published approximation."""
    g = 2 * math.pi / 365.0 * (doy - 1 + (hour_utc - 12) / 24.0)
    dec = (0.006918 - 0.399912 * math.cos(g) + 0.070257 * math.sin(g) - 0.006758 * math.cos(2 * g)
           + 0.000907 * math.sin(2 * g) - 0.002697 * math.cos(3 * g) + 0.00148 * math.sin(3 * g))
    eot = 229.18 * (0.000075 + 0.001868 * math.cos(g) - 0.032077 * math.sin(g)
                    - 0.014615 * math.cos(2 * g) - 0.040849 * math.sin(2 * g))
    return math.degrees(dec), eot


def test_declination_and_eot_vs_spencer():
    # Spencer's series is fitted to one epoch; the seasons drift against the
    # calendar by a fraction of a day since, which moves its declination by
    # up to ~0.3 deg near the equinoxes.  A coarse, independent check.
    worst_d = worst_e = 0.0
    for doy in range(1, 366, 3):
        d = dt.date(2019, 1, 1) + dt.timedelta(days=doy - 1)
        s = oracle.solar(d.year, d.month, d.day, 12 * 60, 0.0, LAT, LON)
        sd, se = _spencer(doy, 12.0)
        worst_d = max(worst_d, abs(s[5] - sd))
        worst_e = max(worst_e, abs(s[6] - se))
    assert worst_d < 0.35
    assert worst_e < 1.0


def test_declination_at_2019_equinox_and_solstice_instants():
    """Published instants of 2019's equinoxes and solstices (UT): the
    declination is zero at the equinoxes and +/- the obliquity (an extremum)
    at the solstices."""
    g = gold("equinox_solstice_2019.json")
    for (y, m, d, hh, mm, kind) in g["events"]:
        jd = oracle.julian_day(y, m, d + (hh + mm / 60.0) / 24.0)
        s = oracle.solar_jd(jd, LAT, LON)
        if kind == "equinox":
            assert abs(s[5]) < 0.01
        else:
            assert abs(abs(s[5]) - s[8]) < 0.002
            before = oracle.solar_jd(jd - 2.0, LAT, LON)[5]
            after = oracle.solar_jd(jd + 2.0, LAT, LON)[5]
            assert abs(s[5]) >= abs(before) and abs(s[5]) >= abs(after)


@pytest.mark.parametrize("md,dec,tol", [((3, 20), 0.0, 0.5), ((6, 21), 23.44, 0.02), ((12, 21), -23.44, 0.02)])
def test_declination_at_equinox_and_solstices(md, dec, tol):
    s = oracle.solar(2019, md[0], md[1], 12 * 60, -4.0, LAT, LON)
    assert abs(s[5] - dec) < tol


def test_equation_of_time_extremes():
    # the equation of time peaks near +16.4 min in early November and
    # bottoms near -14.2 min in mid February
    e = [oracle.solar(2019, m, d, 12 * 60, 0.0, LAT, LON)[6] for (m, d) in [(11, 3), (2, 11)]]
    assert e[0] == pytest.approx(16.4, abs=0.3)
    assert e[1] == pytest.approx(-14.2, abs=0.3)


@pytest.mark.parametrize("md,tz", [((3, 20), -4.0), ((6, 21), -4.0), ((12, 21), -5.0)])
def test_noon_elevation_and_azimuth_symmetry(md, tz):
    # local apparent noon from the equation of time: hour angle zero
    eot = oracle.solar(2019, *md, 720.0, tz, LAT, LON)[6]
    t_noon = 720.0 - 4.0 * LON - eot + 60.0 * tz
    s = oracle.solar(2019, *md, t_noon, tz, LAT, LON)
    assert s[3] == pytest.approx(90.0 - abs(LAT - s[5]), abs=0.01)
    assert s[4] == pytest.approx(180.0, abs=0.01)   # due south at noon (north of the tropics)
    ts = np.arange(t_noon - 5.0, t_noon + 5.0, 0.05)
    el = [oracle.solar(2019, *md, t, tz, LAT, LON)[3] for t in ts]
    assert abs(ts[int(np.argmax(el))] - t_noon) < 0.2   # highest at apparent noon
    for dtm in (60.0, 180.0):
        a = oracle.solar(2019, *md, t_noon - dtm, tz, LAT, LON)
        b = oracle.solar(2019, *md, t_noon + dtm, tz, LAT, LON)
        # symmetric up to the declination drift over the hours between them
        assert a[3] == pytest.approx(b[3], abs=0.15)
        assert (a[4] - 180.0) == pytest.approx(180.0 - b[4], abs=0.3)


def test_direction_is_unit_and_matches_angles():
    for t in (400.0, 700.0, 1000.0):
        s = oracle.solar(2019, 6, 21, t, -4.0, LAT, LON)
        d = s[:3]
        assert np.linalg.norm(d) == pytest.approx(1.0, abs=1e-14)
        e, a = math.radians(s[3]), math.radians(s[4])
        assert d == pytest.approx([math.sin(a) * math.cos(e), math.cos(a) * math.cos(e), math.sin(e)], abs=1e-12)


def test_paper_table1_linear_interpolation():
    """Reproduce the paper's Table 1 from solar position alone: 1000 random
    times over the year, direction at every minute of an n-minute interval vs
    the normalised linear interpolation of its end directions."""
    g = gold("paper_table1_linear_approx.json")
    rng = np.random.default_rng(1907)
    jd0 = oracle.julian_day(2019, 1, 1.0)
    starts = jd0 + rng.uniform(0, 365, 1000)
    stats = {}
    for n in (60, 120, 240):
        cs = []
        for s in starts:
            D = np.array([oracle.solar_jd(s + k / 1440.0, LAT, LON)[:3] for k in range(n + 1)])
            f = np.arange(n + 1) / n
            L = (1 - f)[:, None] * D[0] + f[:, None] * D[-1]
            L /= np.linalg.norm(L, axis=1)[:, None]
            cs.append(np.sum(L * D, axis=1))
        c = np.concatenate(cs)
        stats[n] = (c.mean(), c.std(), np.median(c))
    i = {m: g["minutes"].index(m) for m in (60, 120, 240)}
    assert stats[60][0] == pytest.approx(g["mean"][i[60]], abs=1e-5)
    assert stats[120][0] == pytest.approx(g["mean"][i[120]], abs=1e-5)
    assert stats[240][0] == pytest.approx(g["mean"][i[240]], abs=3e-5)
    assert stats[120][2] == pytest.approx(g["median"][i[120]], abs=1e-5)
    assert stats[240][2] == pytest.approx(g["median"][i[240]], abs=3e-5)
    assert stats[120][1] == pytest.approx(g["sd"][i[120]], rel=0.2)
    assert stats[240][1] == pytest.approx(g["sd"][i[240]], rel=0.15)


@pytest.mark.parametrize("md,tz,K", [((3, 20), -4.0, 719), ((6, 21), -4.0, 895), ((12, 21), -5.0, 545)])
def test_daylight_samples(md, tz, K):
    t, w, span = oracle.day_samples(Day(2019, *md, tz), LAT, LON, 1.0)
    assert len(t) == K
    assert np.all(np.diff(t) == 1.0)
    assert w.sum() == pytest.approx(span[1] - span[0])
    assert w[0] == 0.5 and w[-1] == 0.5 and np.all(w[1:-1] == 1.0)
    # the minute before the first and after the last are at or below the horizon
    assert oracle.solar(2019, *md, t[0] - 1, tz, LAT, LON)[2] <= 0
    assert oracle.solar(2019, *md, t[-1] + 1, tz, LAT, LON)[2] <= 0
    assert oracle.solar(2019, *md, t[0], tz, LAT, LON)[2] > 0


def test_fixed_window_samples():
    t, w, span = oracle.day_samples(Day(2019, 6, 21, -4.0, (480.0, 1080.0)), LAT, LON, 5.0)
    assert len(t) == 121 and t[0] == 480.0 and t[-1] == 1080.0
    assert w.sum() == pytest.approx(600.0)
    with pytest.raises(ValueError):   # a window reaching into the night is refused
        oracle.day_samples(Day(2019, 6, 21, -4.0, (200.0, 1080.0)), LAT, LON, 5.0)


def test_year_daylight_minutes():
    # every day of 2019 has one contiguous daylight run of 545..896 minutes
    total = 0
    for i in range(0, 365, 7):
        d = dt.date(2019, 1, 1) + dt.timedelta(days=i)
        t, w, span = oracle.day_samples(Day(d.year, d.month, d.day, -5.0), LAT, LON, 1.0)
        assert 540 <= len(t) <= 900
        total += len(t)
    assert total > 0
