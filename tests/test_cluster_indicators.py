"""The library's Sec. 3 indicators (host code behind the C ABI, no GPU
needed) against the oracle's, on the counts the oracle takes from random
phase maps, a hand-built grid and the degenerate cases; and the entry
point's argument checks."""
import ctypes

import numpy as np
import pytest

from oracle import clusters as oc
from paper_0802_2488_amd import _lib, synth

KEYS = ("v_p", "f_p", "v_max", "i", "n")


def library_indicators(st, L, f=-1.0):
    s = _lib.PmClusterStats()
    for k, _ in s._fields_:
        if k != "pad":
            setattr(s, k, int(st[k]))
    out = _lib.PmClusterIndicators()
    rc = _lib.lib().pm_cluster_indicators(ctypes.byref(s), L, f, ctypes.byref(out))
    return rc, {k: getattr(out, k) for k in KEYS}


def phase_maps():
    for L, fv, fp, seed in ((4, 0.3, 0.3, 0), (16, 0.05, 0.3, 2), (32, 0.02, 0.35, 3), (64, 0.08, 0.45, 4)):
        void = synth.bernoulli_mask(L, fv, seed).astype(bool)
        yield L, void, synth.bernoulli_mask(L, fp, 1000 + seed).astype(bool) & ~void
    L = 16
    z = np.zeros((L, L), bool)
    one = z.copy()
    one[5, 7] = True
    yield L, z, z                                              # nothing
    yield L, ~z, z                                             # all void
    yield L, z, ~z                                             # plastic, no void
    yield L, one, synth.bernoulli_mask(L, 0.3, 4).astype(bool) & ~one


@pytest.mark.parametrize("case", range(8))
def test_library_indicators_equal_oracle(case):
    L, void, plastic = list(phase_maps())[case]
    _, st = oc.analyze(void, plastic)
    if st["n_void"] == L * L:
        return   # f = 1: f_p undefined, rejected below
    rc, got = library_indicators(st, L)
    assert rc == 0
    ref = oc.indicators(st, L)
    for k in KEYS:
        assert got[k] == pytest.approx(ref[k], rel=1e-15, abs=1e-300), k
    rc, got = library_indicators(st, L, 0.25)
    assert rc == 0
    ref = oc.indicators(st, L, f=0.25)
    for k in KEYS:
        assert got[k] == pytest.approx(ref[k], rel=1e-15, abs=1e-300), k


def test_library_indicators_rejects_bad_arguments():
    L = 8
    st = dict(n_void=4, n_plastic=8, n_void_clusters=3, n_clusters_raw=3, n_isolated_void_clusters=1,
              n_plastic_only_clusters=1, n_clusters=2, largest=11, largest_label=9, spans_x1=0, spans_x2=0)
    assert library_indicators(st, L)[0] == 0
    assert library_indicators(st, 12)[0] == _lib.PM_EINVAL          # not a power of two
    assert library_indicators(st, L, 1.0)[0] == _lib.PM_EINVAL      # f >= 1
    assert library_indicators(dict(st, largest=65), L)[0] == _lib.PM_EINVAL
    assert library_indicators(dict(st, n_void=-1), L)[0] == _lib.PM_EINVAL
    all_void = dict(st, n_void=64, n_plastic=0)
    assert library_indicators(all_void, L)[0] == _lib.PM_EINVAL     # realised f = 1
    out = _lib.PmClusterIndicators()
    assert _lib.lib().pm_cluster_indicators(None, L, -1.0, ctypes.byref(out)) == _lib.PM_EINVAL
