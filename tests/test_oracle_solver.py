"""Pins of the oracle's whole augmented-Lagrangian solve.

Checked against an FFT-free brute-force minimisation on tiny grids, exact
special cases, and invariances and identities the discrete problem of eq. 1
fixes at any size.
"""
import numpy as np
import pytest

from oracle import alm, brute, hencky
from paper_0802_2488_amd import synth


def _params(L, c0=2.0, tol=1e-11, **kw):
    return alm.Params(L=L, mu0=c0 * 1.0, lam0=c0 * 2.0, eta_eq=tol, eta_mac=tol,
                      eta_cmp=tol, **kw)


def _bwd_div(sig):
    s = sig[..., :2, :2]
    return (s[..., :, 0] - np.roll(s[..., :, 0], 1, axis=1)
            + s[..., :, 1] - np.roll(s[..., :, 1], 1, axis=0))


def test_divergence_helper_is_backward_difference():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(8, 8, 3, 3))
    sig = a + np.swapaxes(a, -1, -2)
    np.testing.assert_allclose(alm.divergence(sig), _bwd_div(sig), atol=1e-15)


@pytest.mark.parametrize("E", [(0.3, 0.3, 0.0), (0.0, 0.0, 0.5), (0.2, -0.1, 0.05)])
def test_homogeneous_medium_is_uniform_after_one_iteration(E):
    """f = 0: eps = E and sigma = S(E) everywhere after one iteration."""
    L = 16
    s = alm.Solver(np.zeros((L, L), np.uint8), _params(L))
    s.start(E)
    s.iterate(E)
    Et = alm.tensor_from_voigt(E)
    assert np.abs(s.eps - Et).max() < 1e-14
    np.testing.assert_allclose(s.sigma(), np.broadcast_to(hencky.stress(Et, 1.0, 2.0, 1.0), s.eps.shape),
                               atol=1e-13)
    r = alm.Solver(np.zeros((L, L), np.uint8), _params(L)).step(E)
    assert r.converged and r.iters == 2


@pytest.mark.parametrize("E", [(0.3, 0.1, 0.05), (0.0, 0.0, 0.4)])
def test_all_void_grid_carries_the_mean_strain_and_no_stress(E):
    """f = 1: no pixel has stiffness, so sigma = 0 everywhere, nothing drives
    a fluctuation and eps = E with eps33 = 0 (a void's out-of-plane strain);
    every indicator is 0 against its norm floor and the step converges at
    the first iteration where the test applies."""
    L = 16
    r = alm.Solver(np.ones((L, L), np.uint8), _params(L, c0=0.02)).step(E)
    assert r.converged and r.iters == 2
    assert r.res_eq == 0.0 and r.res_mac == 0.0 and r.res_cmp == 0.0
    assert np.all(r.sigma == 0.0)
    np.testing.assert_allclose(r.eps, np.broadcast_to(alm.tensor_from_voigt(E), r.eps.shape), atol=1e-15)
    assert not r.plastic.any()


def test_zero_load_gives_zero_solution():
    mask = synth.bernoulli_mask(8, 0.2, 0)
    s = alm.Solver(mask, _params(8))
    s.step((0.3, 0.3, 0.0), fixed_iters=5)
    r = s.step((0.0, 0.0, 0.0))
    assert r.converged and r.iters == 0
    assert np.all(r.sigma == 0.0) and np.all(s.eps == 0.0)


@pytest.mark.parametrize("L,f,seed,E", [(8, 0.2, 3, (0.01, 0.02, 0.005)), (6, 0.1, 5, (0.0, 0.0, 0.02))])
def test_elastic_matches_brute_force_least_squares(L, f, seed, E):
    mask = synth.bernoulli_mask(L, f, seed)
    p = _params(L, c0=2.0, tol=1e-13, Y=1e9)
    r = alm.solve_path(mask, p, [E])[-1]
    assert r.converged
    sb = brute.solve_elastic(mask, E, 1.0, 2.0)
    assert np.linalg.norm(r.sigma - sb) / np.linalg.norm(sb) < 1e-10


@pytest.mark.parametrize("L,f,seed,E", [(8, 0.1, 1, (0.6, 0.6, 0.0)),
                                        (8, 0.1, 1, (0.0, 0.0, 0.35)),
                                        (6, 0.15, 2, (0.7, 0.5, 0.1))])
def test_plastic_matches_brute_force_energy_minimum(L, f, seed, E):
    """Plastic loading: sigma from the ALM equals the stress of the L-BFGS
    minimiser of the total energy; the energies agree too."""
    mask = synth.bernoulli_mask(L, f, seed)
    p = _params(L, c0=0.5, tol=1e-11, max_iter=40000)
    r = alm.solve_path(mask, p, [E])[-1]
    assert r.converged and r.plastic.sum() > 0
    sb, W, info = brute.solve_plastic(mask, E, 1.0, 2.0, 1.0)
    assert np.linalg.norm(r.sigma - sb) / np.linalg.norm(sb) < 1e-6
    W_alm = brute.total_energy(r.e, mask, 1.0, 2.0, 1.0)
    assert abs(W_alm - W) < 1e-10 * abs(W)


@pytest.fixture(scope="module")
def converged16():
    L = 16
    mask = synth.bernoulli_mask(L, 0.1, 11)
    p = _params(L, c0=0.5, tol=1e-10, max_iter=60000)
    E = (0.45, 0.45, 0.0)
    r = alm.solve_path(mask, p, [E])[-1]
    return mask, E, r


def test_converged_solution_identities(converged16):
    mask, E, r = converged16
    assert r.converged
    # per-pixel equilibrium (eq. 1, backward differences)
    assert np.abs(_bwd_div(r.sigma)).max() < 1e-7 * np.abs(r.sigma).max()
    # mean of the compatible strain is the prescribed strain
    np.testing.assert_allclose(r.e.mean(axis=(0, 1)), alm.tensor_from_voigt(E), atol=1e-14)
    # Hill-Mandel: <sigma:e> = <sigma>:<e> for equilibrated sigma, compatible e
    lhs = np.mean(np.sum(r.sigma * r.e, axis=(-2, -1)))
    rhs = np.sum(r.sigma.mean(axis=(0, 1)) * r.e.mean(axis=(0, 1)))
    assert abs(lhs - rhs) < 1e-8 * abs(rhs)
    # voids carry exactly zero stress, matrix stress within the Mises cap
    assert np.all(r.sigma[mask.astype(bool)] == 0.0)
    assert hencky.sigma_eq(r.sigma).max() <= 1.0 + 1e-12
    # energy at the solution is below the uniform-strain (Voigt) energy
    W = brute.total_energy(r.e, mask, 1.0, 2.0, 1.0)
    W_voigt = brute.total_energy(np.broadcast_to(alm.tensor_from_voigt(E), r.e.shape), mask, 1.0, 2.0, 1.0)
    assert W < W_voigt
    # eps33 -> 0 (plane strain) and eps -> e at convergence
    assert np.abs(r.eps[..., 2, 2]).max() < 1e-6


def test_multiplier_equals_stress_every_iteration():
    """After each iteration lambda = S(eps) on matrix pixels and 0 on voids
    (exact property of the multiplier update)."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 4)
    s = alm.Solver(mask, _params(L))
    E = (0.7, 0.2, 0.1)
    s.start(E)
    for _ in range(30):
        s.iterate(E)
        assert np.abs(s.lam_mult - s.sigma()).max() < 1e-12


def _run_fixed(mask, E, n, Y=1.0):
    p = _params(mask.shape[0], Y=Y)
    s = alm.Solver(mask, p)
    return s.step(E, fixed_iters=n)


def test_translation_invariance():
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 6)
    E = (0.5, 0.3, 0.2)
    a = _run_fixed(mask, E, 40)
    b = _run_fixed(np.roll(mask, (3, 5), axis=(0, 1)), E, 40)
    np.testing.assert_allclose(np.roll(a.sigma, (3, 5), axis=(0, 1)), b.sigma, atol=1e-11)


def test_transpose_invariance():
    """Swapping the two axes maps the forward/backward scheme onto itself."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 7)
    E = (0.5, 0.3, 0.2)
    a = _run_fixed(mask, E, 40)
    b = _run_fixed(np.ascontiguousarray(mask.T), (E[1], E[0], E[2]), 40)
    P = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]], float)
    at = np.einsum("ia,yxab,jb->xyij", P, a.sigma, P)
    np.testing.assert_allclose(at, b.sigma, atol=1e-11)


def test_mirror_is_not_a_symmetry():
    """The scheme is not mirror symmetric (Sec. 2): flipping x1 changes the field."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 7)
    E = (0.5, 0.3, 0.0)
    a = _run_fixed(mask, E, 40)
    b = _run_fixed(np.ascontiguousarray(mask[:, ::-1]), E, 40)
    assert np.abs(a.sigma[:, ::-1, 0, 0] - b.sigma[..., 0, 0]).max() > 1e-3


def test_positive_homogeneity():
    """sigma(cE; cY) = c sigma(E; Y) iterate by iterate."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 8)
    E = np.array([0.5, 0.3, 0.2])
    a = _run_fixed(mask, E, 30, Y=1.0)
    b = _run_fixed(mask, 2.5 * E, 30, Y=2.5)
    np.testing.assert_allclose(2.5 * a.sigma, b.sigma, atol=1e-11)


def test_elastic_regime_is_linear():
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 9)
    E1 = np.array([0.01, 0.0, 0.0])
    E2 = np.array([0.0, 0.0, 0.01])
    a = _run_fixed(mask, E1, 30, Y=1e9)
    b = _run_fixed(mask, E2, 30, Y=1e9)
    c = _run_fixed(mask, E1 + 2 * E2, 30, Y=1e9)
    np.testing.assert_allclose(a.sigma + 2 * b.sigma, c.sigma, atol=1e-13)


def test_warm_start_only_changes_the_mean_strain():
    """A second load step continues from the stored state: running 10 + 10
    iterations at the same E equals 20 iterations in one step."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 10)
    E = (0.5, 0.3, 0.2)
    s1 = alm.Solver(mask, _params(L))
    s1.step(E, fixed_iters=10)
    a = s1.step(E, fixed_iters=10)
    b = alm.Solver(mask, _params(L)).step(E, fixed_iters=20)
    np.testing.assert_allclose(a.sigma, b.sigma, atol=1e-13)


def test_indicator_normalisations_on_a_hand_example():
    """Two iterations worked by hand.  Homogeneous medium with C = C0 / 2
    (lambda = 2, mu = 1, reference twice that), elastic throughout.  Start
    from eps0 = E + d + delta with d uniform and delta a compatible
    fluctuation (eps11 = a(x1 + 1) - a(x1), eps22 = b(x2 + 1) - b(x2),
    eps12 = (c(x1 + 1) - c(x1)) / 2), lambda0 = C:eps0.  The Green step
    turns the fluctuating tau = -C0:delta_n / 2 into +delta_n / 2
    (G C0 G = -G on compatible fields) and imposes the mean E; the pointwise
    step 3/2 C0:eps = C:eps_n + C0:e then gives
      <eps_n> = E + d / 3^n,  fluctuation (2/3)^n delta,
      e_n - eps_n = -d_{n-1} / 3 - delta_{n-1} / 6.
    Hence after two iterations
      eta_2 = |C:(d/3 - d/9)| / |C:(E + d/9)|,
      r_cmp = sqrt(|d/3|^2 / 9 + <|delta|^2> (4/9) / 36) / |E|,
    with 3-D Frobenius norms (12 and 21 both counted).  Dividing eta_2 by the
    previous mean, dropping the factor 2 on the 12 terms or normalising r_cmp
    by anything but |E| each changes one of these numbers."""
    L = 8
    rng = np.random.default_rng(21)
    a, b, c = (0.02 * rng.normal(size=L) for _ in range(3))
    delta = np.zeros((L, L, 3, 3))
    delta[..., 0, 0] = (np.roll(a, -1) - a)[None, :]
    delta[..., 1, 1] = (np.roll(b, -1) - b)[:, None]
    delta[..., 0, 1] = delta[..., 1, 0] = (0.5 * (np.roll(c, -1) - c))[None, :]
    E = (0.02, 0.0, 0.03)
    Et = alm.tensor_from_voigt(E)
    d = alm.tensor_from_voigt((0.01, 0.0, -0.02))
    p = _params(L, max_iter=10)
    s = alm.Solver(np.zeros((L, L), np.uint8), p)
    s.eps = Et + d + delta
    s.lam_mult = hencky.iso(2.0, 1.0, s.eps)
    r = s.step(E, fixed_iters=2)
    assert not r.plastic.any()
    C = lambda t: hencky.iso(2.0, 1.0, t)   # noqa: E731
    fro = lambda t: float(np.sqrt(np.sum(t * t)))   # noqa: E731
    eta2 = fro(C(d / 3 - d / 9)) / fro(C(Et + d / 9))
    msq = float(np.mean(np.sum(delta * delta, axis=(-2, -1))))
    rcmp = np.sqrt(fro(d / 3) ** 2 / 9 + msq * (4.0 / 9.0) / 36.0) / fro(Et)
    assert r.res_mac == pytest.approx(eta2, rel=1e-10)
    assert r.res_cmp == pytest.approx(rcmp, rel=1e-10)
    np.testing.assert_allclose(r.eps_mean, Et + d / 9, atol=1e-14)
    np.testing.assert_allclose(r.eps - r.eps_mean, (4.0 / 9.0) * delta, atol=1e-14)
