"""Pins of the strain-map measures (Fig. 1 comparison) by closed forms."""
import numpy as np
import pytest

from oracle import maps
from paper_0802_2488_amd import synth


def shear_field(s):
    """eps_12 = s(x) only: eps_eq = (2 / sqrt 3) |s|."""
    L = s.shape[0]
    e = np.zeros((L, L, 3, 3))
    e[..., 0, 1] = e[..., 1, 0] = s
    return e


def test_uniform_field():
    L = 8
    r = maps.strain_map_metrics(shear_field(np.full((L, L), 0.3)), np.zeros((L, L), bool))
    assert r["mean_eq"] == pytest.approx(2 / np.sqrt(3) * 0.3, rel=1e-14)
    assert r["max_eq"] == pytest.approx(r["mean_eq"], rel=1e-14)
    assert r["checkerboard"] == 0.0 and r["sharpness"] == 0.0 and r["matrix_pixels"] == L * L


def test_checkerboard_index_of_a_pure_oscillation():
    """s = a + b (-1)^(x1 + x2): the mixed difference is 4 b (-1)^(x1 + x2),
    so the index is 4 b / a; every neighbour difference is 2 b, so the
    sharpness is 2 b / a."""
    L, a, b = 8, 0.5, 0.05
    x = np.arange(L)
    s = a + b * (-1.0) ** (x[None, :] + x[:, None])
    r = maps.strain_map_metrics(shear_field(s), np.zeros((L, L), bool))
    assert r["checkerboard"] == pytest.approx(4 * b / a, rel=1e-12)
    assert r["sharpness"] == pytest.approx(2 * b / a, rel=1e-12)


def test_one_axis_variation_has_no_checkerboard():
    L = 16
    x = np.arange(L)
    s = np.broadcast_to(0.2 + 0.1 * np.sin(2 * np.pi * x / L), (L, L))
    r = maps.strain_map_metrics(shear_field(s), np.zeros((L, L), bool))
    assert r["checkerboard"] < 1e-15 and r["sharpness"] > 0.01


def test_voids_and_blocks_touching_them_are_left_out():
    """A huge value in a void changes nothing; blocks and pairs that touch
    the void are dropped (a single void removes 4 blocks and 4 pairs)."""
    L = 8
    rng = np.random.default_rng(0)
    s = 0.2 + 0.01 * rng.random((L, L))
    void = np.zeros((L, L), bool)
    void[3, 4] = True
    a = maps.strain_map_metrics(shear_field(s), void)
    s2 = s.copy()
    s2[3, 4] = 1e6
    b = maps.strain_map_metrics(shear_field(s2), void)
    assert a == b and a["matrix_pixels"] == L * L - 1
    assert a["max_eq"] < 1.0


def test_random_masks_finite():
    L = 32
    void = synth.bernoulli_mask(L, 0.3, 1).astype(bool)
    rng = np.random.default_rng(2)
    e = rng.normal(size=(L, L, 3, 3))
    r = maps.strain_map_metrics(e + np.swapaxes(e, -1, -2), void)
    assert all(np.isfinite(v) for v in r.values())
