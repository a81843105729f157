"""Pins of the oracle's constitutive law and pointwise augmented-Lagrangian step.

The law is pinned by hand-derived closed forms (tests/golden), by the
energy it derives from, and by an independent numerical solve of the
pointwise equation.
"""
import json
import os

import numpy as np
import pytest
import scipy.optimize

from oracle import alm, hencky

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hencky_closed_forms.json")


def _sym(rng, n, scale=1.0):
    a = rng.normal(size=(n, 3, 3)) * scale
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def test_closed_forms_uniform_strain():
    g = json.load(open(GOLD))
    for c in g["cases"]:
        eps = alm.tensor_from_voigt(c["E"])
        sig = hencky.stress(eps, g["mu"], g["lambda"], g["Y"])
        np.testing.assert_allclose(alm.voigt4(sig), c["sigma"], rtol=1e-14, atol=1e-14)


def test_mises_cap_and_branch():
    rng = np.random.default_rng(1)
    eps = _sym(rng, 2000, 0.25)
    sig = hencky.stress(eps, 1.0, 2.0, 1.0)
    seq = hencky.sigma_eq(sig)
    assert np.all(seq <= 1.0 + 1e-12)
    plastic = 3.0 * 1.0 * hencky.eps_eq(eps) > 1.0
    assert plastic.sum() > 100 and (~plastic).sum() > 100
    np.testing.assert_allclose(seq[plastic], 1.0, rtol=1e-12)
    # elastic pixels: sigma_eq = 3 mu eps_eq (Hooke)
    np.testing.assert_allclose(seq[~plastic], 3.0 * hencky.eps_eq(eps[~plastic]), rtol=1e-12)


def test_stress_is_energy_gradient():
    """S = dw/deps by central differences, in both regimes."""
    rng = np.random.default_rng(2)
    eps = _sym(rng, 50, 0.4)
    h = 1e-6
    sig = hencky.stress(eps, 1.0, 2.0, 1.0)
    for a in range(3):
        for b in range(a, 3):
            d = np.zeros((3, 3))
            d[a, b] = d[b, a] = h
            wp = hencky.energy(eps + d, 1.0, 2.0, 1.0)
            wm = hencky.energy(eps - d, 1.0, 2.0, 1.0)
            num = (wp - wm) / (2 * h)
            ana = sig[:, a, b] * (1.0 if a == b else 2.0)
            np.testing.assert_allclose(num, ana, rtol=1e-6, atol=1e-7)


def test_energy_continuity_at_yield():
    for t in (1.0 - 1e-9, 1.0, 1.0 + 1e-9):
        e = t * 0.5   # equibiaxial yield point for mu = Y = 1
        w = hencky.energy(alm.tensor_from_voigt([e, e, 0.0]), 1.0, 2.0, 1.0)
        # elastic energy at the yield point: K/2 (2e)^2 + mu e':e' = 4/3 + 1/6
        assert abs(w - (4.0 / 3.0 + 1.0 / 6.0)) < 1e-8


@pytest.mark.parametrize("c0", [0.5, 2.0])
def test_pointwise_solve_residual(c0):
    """eps returned by the pointwise step satisfies S(eps) + C0:eps = R."""
    rng = np.random.default_rng(3)
    mu, lam, Y = 1.0, 2.0, 1.0
    mu0, lam0 = c0 * mu, c0 * lam
    R = _sym(rng, 3000, 0.5 if c0 < 1 else 1.2)
    void = rng.random(3000) < 0.2
    eps, plastic, margin = hencky.pointwise_solve(R, void, mu, lam, Y, mu0, lam0)
    sig = np.where(void[:, None, None], 0.0, hencky.stress(eps, mu, lam, Y))
    res = sig + hencky.iso(lam0, mu0, eps) - R
    assert np.abs(res).max() < 1e-12 * np.abs(R).max()
    assert plastic.sum() > 100 and (~plastic & ~void).sum() > 100
    # branch flag agrees with the law's own yield test on the solution
    m = ~void
    np.testing.assert_array_equal(plastic[m], (3 * mu * hencky.eps_eq(eps[m]) > Y)[...])
    assert np.all((margin[m] > 0) == plastic[m])


def test_pointwise_solve_matches_numerical_minimiser():
    """Independent check: eps minimises w(eps) + eps:C0:eps/2 - R:eps."""
    rng = np.random.default_rng(4)
    mu, lam, Y, mu0, lam0 = 1.0, 2.0, 1.0, 2.0, 4.0
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for R in _sym(rng, 12, 3.0):
        def f(v):
            e = np.zeros((3, 3))
            for (a, b), x in zip(idx, v):
                e[a, b] = e[b, a] = x
            val = hencky.energy(e, mu, lam, Y) + 0.5 * np.sum(e * hencky.iso(lam0, mu0, e)) - np.sum(R * e)
            return float(val)
        sol = scipy.optimize.minimize(f, np.zeros(6), method="Nelder-Mead",
                                      options=dict(xatol=1e-12, fatol=1e-15, maxiter=40000, maxfev=80000))
        e_ref = np.zeros((3, 3))
        for (a, b), x in zip(idx, sol.x):
            e_ref[a, b] = e_ref[b, a] = x
        eps, _, _ = hencky.pointwise_solve(R[None], np.zeros(1, bool), mu, lam, Y, mu0, lam0)
        np.testing.assert_allclose(eps[0], e_ref, atol=1e-6)


def test_void_pointwise_and_zero_stress():
    rng = np.random.default_rng(5)
    R = _sym(rng, 100)
    eps, plastic, _ = hencky.pointwise_solve(R, np.ones(100, bool), 1.0, 2.0, 1.0, 2.0, 4.0)
    np.testing.assert_allclose(hencky.iso(4.0, 2.0, eps), R, atol=1e-13)
    assert not plastic.any()
    sig = hencky.field_stress(eps, np.ones(100, bool), 1.0, 2.0, 1.0)
    assert np.all(sig == 0.0)


@pytest.mark.parametrize("a,expect", [(3.0, np.sqrt(3.0) - 1.0), (1.0, 1.0 / np.sqrt(3.0) - 1.0)])
def test_margin_is_the_trial_mises_stress_minus_yield(a, expect):
    """Hand values of the margin at a uniform R = diag(a, -a, 0) (pure
    deviator, |dev R| = sqrt(2) a) with mu = 1, mu0 = 2, Y = 1: the trial
    (elastic) step gives dev eps = dev R / (2 (mu + mu0)), so its stress
    deviator is mu dev R / (mu + mu0) and its Mises stress
    sqrt(3/2) sqrt(2) a / 3 = a / sqrt(3); the margin is that minus Y.
    a = 3 is on the capped branch (margin sqrt(3) - 1), a = 1 elastic.  A
    wrong sqrt(3/2), (mu + mu0) or Y would move both values."""
    R = np.diag([a, -a, 0.0])[None]
    eps, plastic, margin = hencky.pointwise_solve(R, np.zeros(1, bool), 1.0, 2.0, 1.0, 2.0, 4.0)
    assert margin[0] == pytest.approx(expect, abs=1e-14)
    assert bool(plastic[0]) == (a == 3.0)


def test_margin_equals_mises_stress_of_the_elastic_trial_strain():
    """Independent route: solve (C + C0):eps_t = R as if elastic, take the
    Mises stress of C:eps_t, subtract Y; on the elastic branch that stress is
    the returned one."""
    rng = np.random.default_rng(12)
    mu, lam, Y, mu0, lam0 = 1.0, 2.0, 1.0, 2.0, 4.0
    R = _sym(rng, 400, 1.5)
    void = np.zeros(400, bool)
    eps, plastic, margin = hencky.pointwise_solve(R, void, mu, lam, Y, mu0, lam0)
    eps_t = hencky.iso_inv(lam + lam0, mu + mu0, R)
    trial = hencky.sigma_eq(hencky.iso(lam, mu, eps_t)) - Y
    np.testing.assert_allclose(margin, trial, rtol=0, atol=1e-12)
    el = ~plastic
    assert el.sum() > 50 and plastic.sum() > 50
    np.testing.assert_allclose(hencky.sigma_eq(hencky.stress(eps[el], mu, lam, Y)) - Y, margin[el], atol=1e-12)
