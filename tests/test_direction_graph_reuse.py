"""Edge counts of the direction graph of Sec. 6 on a year-long path,
independent of the library and the oracle: the distinct (start bin, end
bin, duration) triples of a year of 30-minute segments at a fine and at the
paper's 5-degree bound (library sun path, host only).  At a fine bound
almost every segment is its own edge; at 5 degrees the reuse is of the
order the paper reports.  The library's graph (`sa_path_upload_graph`)
merges within an output bin and is tested on the GPU."""
import datetime

import numpy as np

import paper_1907_04435_amd as sa
from workloads import Span
from workloads.scenes import Day, _nyc_tz


def year_path(seg_min):
    days, d = [], datetime.date(2019, 1, 1)
    while d.year == 2019:
        days.append(Day(d.year, d.month, d.day, _nyc_tz(d), None))
        d += datetime.timedelta(1)
    return sa.sunpath_for_span(Span(40.7, -74.0, days, 1.0), seg_min)


def edges(sp, bound_deg):
    """Distinct (start bin, end bin, duration) triples; bins: rings of
    `bound` in elevation, each cut into azimuth cells of at most `bound`."""
    b = np.radians(bound_deg)
    kd = sp.knot_dir
    el = np.arcsin(np.clip(kd[:, 2], -1, 1))
    az = np.arctan2(kd[:, 0], kd[:, 1])
    ring = np.floor(el / b).astype(np.int64)
    naz = np.maximum(1, np.ceil(2 * np.pi * np.cos(ring * b) / b)).astype(np.int64)
    cell = np.floor((az + np.pi) / (2 * np.pi) * naz).astype(np.int64)
    key = ring * 1_000_000 + cell
    out, n = set(), 0
    ko, kt = sp.day_knot_off, sp.knot_t
    for i in range(len(ko) - 1):
        for k in range(ko[i], ko[i + 1] - 1):
            out.add((key[k], key[k + 1], round(kt[k + 1] - kt[k], 3)))
            n += 1
    return n, len(out)


def test_direction_graph_reuse_on_a_year():
    sp = year_path(30.0)
    n, fine = edges(sp, 0.1)
    _, coarse = edges(sp, 5.0)
    assert n > 8000
    assert n / fine < 1.1            # at 0.1 deg almost every segment is its own edge
    assert 6.0 < n / coarse < 12.0   # at the paper's 5 deg the reuse is of the paper's order (2,190 -> 299)
