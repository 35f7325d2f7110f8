"""Helpers for the GPU parity tests: run the library through its binding
and compare with the oracle on the same seeded inputs."""
import sys

import numpy as np

import oracle
import paper_1907_04435_amd as sa


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def unpack_words(words_by_point: np.ndarray, K: int) -> np.ndarray:
    """uint32 [n, words] -> uint8 [n, K] (bit k%32 of word k/32)."""
    w = np.ascontiguousarray(words_by_point.astype(np.uint32))
    return np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")[:, :K]


def run_lib(ctx, scene, pts, span, mode, seg_min=30.0, bits=False):
    """Library outputs for a workload as numpy: counts [bins, n], minutes
    [bins, n], bits [n, K] (sampled form only)."""
    sp = sa.sunpath_for_span(span, seg_min)
    path = sa.Path(ctx, sp)
    sc = sa.Scene.from_workload(ctx, scene)
    dp = sa.DevicePoints.from_workload(pts)
    c, m, b = sa.accumulate(ctx, sc, dp, path, mode, want_counts=True, want_bits=bits)
    ctx.sync()
    out = dict(counts=c.cpu().numpy(), minutes=m.cpu().numpy().astype(np.float64))
    if bits:
        out["bits"] = unpack_words(b.cpu().numpy().view(np.uint32).T, sp.n_samples)
    out["K"] = sp.n_samples
    return out


def check_sampled(g, o, w):
    """Bit-exact on every unambiguous (point, instant) pair; counts and
    minutes then differ only by the ambiguous pairs."""
    K = g["K"]
    ob = unpack_words(o["bits"], K)
    amb = o["amb"].astype(bool)
    mism = g["bits"] != ob
    bad = mism & ~amb
    assert not bad.any(), f"{int(bad.sum())} unambiguous mismatches, first at {np.argwhere(bad)[:5].tolist()}"
    na = amb.sum(1)
    dc = np.abs(g["counts"].sum(0) - o["counts"].sum(0))
    assert np.all(dc <= na)
    np.testing.assert_array_equal(g["counts"].sum(0)[na == 0], o["counts"].sum(0)[na == 0])
    wmax = (amb * w[None, :]).sum(1)
    dm = np.abs(g["minutes"].sum(0) - o["minutes"].sum(0))
    assert np.all(dm <= wmax + 1e-3 + 1e-6 * np.abs(o["minutes"].sum(0)))
    return amb.mean(), int(mism.sum())
