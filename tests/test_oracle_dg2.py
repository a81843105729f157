"""Pins of the DG2 oracle (Sec. 2, "Discrete Green functions").

The discrete Green tensor of eq. 3 is not mirror symmetric; the four sign
variants map onto one another under the lattice mirrors.  Mirroring the mask
in x1 (pixel x1 -> -x1 mod L) turns the solve with G(q1, q2) into the mirror
image of the solve with G(-q1, q2) on the original mask (x2: G(q1, -q2);
both: G(-q1, -q2)), iterate by iterate.  Hence the DG2 average commutes with
all three mirrors while a single variant does not: this fixes the variant
definitions and the averaging independently of the code that computes them.
"""
import numpy as np
import pytest

from oracle import alm, dg2, hencky
from paper_0802_2488_amd import synth

L = 16


def mir1(a):
    return a[:, (-np.arange(L)) % L]


def mir2(a):
    return a[(-np.arange(L)) % L, :]


def mir12(a):
    return mir1(mir2(a))


def run_variant(mask, E, v, iters=12):
    return alm.Solver(mask, alm.Params(L=L, green_variant=v)).step(E, fixed_iters=iters)


@pytest.fixture(scope="module")
def case():
    mask = synth.bernoulli_mask(L, 0.2, 3)
    E = (0.3, 0.1, 0.2)
    return mask, E


@pytest.mark.parametrize("mf,pairs", [(mir1, {0: 2, 2: 0, 1: 3, 3: 1}), (mir2, {0: 3, 3: 0, 1: 2, 2: 1}),
                                      (mir12, {0: 1, 1: 0, 2: 3, 3: 2})])
def test_mirror_maps_variants_onto_each_other(case, mf, pairs):
    mask, E = case
    for v, w in pairs.items():
        on_mirror = run_variant(mf(mask), E, v)
        ref = run_variant(mask, E, w)
        assert np.abs(on_mirror.sigma - mf(ref.sigma)).max() <= 1e-12
        assert np.abs(on_mirror.eps - mf(ref.eps)).max() <= 1e-12


@pytest.mark.parametrize("mf", [mir1, mir2, mir12])
def test_dg2_commutes_with_mirrors_single_variant_does_not(case, mf):
    mask, E = case
    p = alm.Params(L=L)
    iters = [[12], [12], [12], [12]]
    a = dg2.solve_path(mask, p, [E], fixed_iters=iters)[0]
    b = dg2.solve_path(mf(mask), p, [E], fixed_iters=iters)[0]
    assert np.abs(b.eps - mf(a.eps)).max() <= 1e-12
    assert np.abs(b.sigma_of_avg - mf(a.sigma_of_avg)).max() <= 1e-12
    assert np.abs(b.sigma_avg - mf(a.sigma_avg)).max() <= 1e-12
    assert np.array_equal(b.plastic, mf(a.plastic))
    # the single variant G(q1, q2) is not mirror symmetric
    assert np.abs(b.variants[0].sigma - mf(a.variants[0].sigma)).max() > 1e-3


def test_dg2_homogeneous_medium_is_uniform():
    mask = np.zeros((L, L), np.uint8)
    E = (0.7, 0.2, 0.1)
    r = dg2.solve_path(mask, alm.Params(L=L), [E], fixed_iters=[[3]] * 4)[0]
    ref = hencky.stress(alm.tensor_from_voigt(E), 1.0, 2.0, 1.0)
    for v in r.variants:
        assert np.abs(v.sigma - ref).max() <= 1e-12
    assert np.abs(r.eps - alm.tensor_from_voigt(E)).max() <= 1e-12
    assert np.abs(r.sigma_of_avg - ref).max() <= 1e-12


def test_combine_is_the_plain_average():
    rng = np.random.default_rng(1)
    void = synth.bernoulli_mask(8, 0.3, 5).astype(bool)
    base = rng.normal(size=(8, 8, 3, 3)) * 0.2
    base = 0.5 * (base + np.swapaxes(base, -1, -2))
    d = rng.normal(size=(8, 8, 3, 3)) * 0.05
    d = 0.5 * (d + np.swapaxes(d, -1, -2))
    eps4 = np.stack([base + d, base - d, base + 2 * d, base - 2 * d])
    sig4 = np.stack([hencky.field_stress(e, void, 1.0, 2.0, 1.0) for e in eps4])
    eps, soa, sav, pl, mg = dg2.combine(void, eps4, sig4, 1.0, 2.0, 1.0)
    assert np.abs(eps - base).max() <= 1e-15
    assert np.abs(soa - hencky.field_stress(base, void, 1.0, 2.0, 1.0)).max() <= 1e-14
    assert np.abs(sav - sig4.mean(axis=0)).max() <= 1e-15
    assert np.all(soa[void] == 0.0) and not pl[void].any()
    seq = hencky.sigma_eq(soa)
    assert np.all(seq[pl] >= 1.0 - 1e-12)          # plastic pixels sit on the yield surface
    assert np.all(seq[~pl & ~void] <= 1.0 + 1e-12)


@pytest.mark.parametrize("mf,pairs", [(mir1, {0: 2, 2: 0, 1: 3, 3: 1}), (mir2, {0: 3, 3: 0, 1: 2, 2: 1}),
                                      (mir12, {0: 1, 1: 0, 2: 3, 3: 2})])
def test_each_variant_measures_its_own_equilibrium(case, mf, pairs):
    """A variant's equilibrium indicator is that of its own momenta: under a
    mirror it equals, iterate by iterate, the indicator of the variant it maps
    onto (the backward differences of eq. 1 for every variant would break
    this, since the mirror turns a backward difference into a forward one)."""
    mask, E = case
    for v, w in pairs.items():
        a = run_variant(mf(mask), E, v)
        b = run_variant(mask, E, w)
        assert a.res_eq == pytest.approx(b.res_eq, rel=1e-10)
        s = a.sigma
        own = alm.divergence(s, *alm.FLIPS[v])
        assert np.sqrt(np.mean(np.sum(own ** 2, axis=-1))) / alm.norm3(s.mean(axis=(0, 1))) == \
            pytest.approx(a.res_eq, rel=1e-12)


def test_every_variant_converges_on_its_own_indicator():
    """With a reference medium soft enough to converge quickly (C0 = 0.02 x
    matrix), all four variants reach 1e-8 on all three indicators; mirrored
    pairs need the same number of iterations."""
    mask = synth.bernoulli_mask(L, 0.1, 5)
    E = (0.2, 0.2, 0.0)
    p = alm.Params(L=L, mu0=0.04, lam0=0.08, max_iter=8000)
    res = [alm.Solver(mask, alm.Params(**{**p.__dict__, "green_variant": v})).step(E) for v in range(4)]
    for r in res:
        assert r.converged and r.res_eq < 1e-8, (r.iters, r.res_eq)
    m = mir1(mask)
    r2 = alm.Solver(m, alm.Params(**{**p.__dict__, "green_variant": 2})).step(E)
    assert r2.iters == res[0].iters
