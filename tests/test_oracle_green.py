"""Pins of the oracle's discrete Green tensor (Sec. 2, eqs. 1-3).

The tensor is checked against properties the mathematics fixes, with every
auxiliary operator (stiffness, finite differences) rebuilt here from its
definition rather than taken from the oracle.
"""
import numpy as np
import pytest

from oracle import alm, dg
from paper_0802_2488_amd import synth


LAM0, MU0 = 4.0, 2.0


def C_iso(lam, mu):
    """Isotropic plane-strain stiffness as an explicit 2x2x2x2 array."""
    C = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    C[i, j, k, l] = (lam * (i == j) * (k == l)
                                     + mu * ((i == k) * (j == l) + (i == l) * (j == k)))
    return C


@pytest.mark.parametrize("L", [8, 16])
def test_projection_identity(L):
    """G C0 G = -G: G is minus the C0-orthogonal projector onto compatible fields."""
    G = dg.green_on_grid(L, LAM0, MU0)
    GCG = np.einsum("...ijkl,klmn,...mnpq->...ijpq", G, C_iso(LAM0, MU0), G)
    assert np.abs(GCG + G).max() < 1e-14 * max(1.0, np.abs(G).max())


def test_hermitian_symmetry_stated_in_paper():
    """G_ijkl = conj(G_klij) (Sec. 2, the paragraph after eq. 3)."""
    G = dg.green_on_grid(16, LAM0, MU0)
    assert np.abs(G - np.conj(np.einsum("...ijkl->...klij", G))).max() < 1e-15


def test_lacks_major_symmetry_and_is_complex():
    """The paper notes the nonzero imaginary part breaks major symmetry."""
    G = dg.green_on_grid(16, LAM0, MU0)
    assert np.abs(G.imag).max() > 1e-2
    assert np.abs(G - np.einsum("...ijkl->...klij", G)).max() > 1e-2


def test_conjugate_at_minus_q_and_real_at_self_conjugate_points():
    L = 16
    K = dg.half_spectrum_k(L)
    Kminus = dg.half_spectrum_k(L, True, True)
    G = dg.green_tensor(K, LAM0, MU0)
    Gm = dg.green_tensor(Kminus, LAM0, MU0)
    assert np.abs(Gm - np.conj(G)).max() < 1e-15
    for m2 in (0, L // 2):
        for m1 in (0, L // 2):
            assert np.abs(G[m2, m1].imag).max() < 1e-15


def _fwd_diff_strain(u):
    """eps_ij = [u_j(x+e^i) - u_j(x) + u_i(x+e^j) - u_i(x)] / 2, eq. 1; u: (L, L, 2)."""
    L = u.shape[0]
    du = np.zeros((L, L, 2, 2))   # du[..., i, j] = u_j(x + e^i) - u_j(x)
    du[..., 0, :] = np.roll(u, -1, axis=1) - u     # direction 1 = axis 1
    du[..., 1, :] = np.roll(u, -1, axis=0) - u     # direction 2 = axis 0
    return 0.5 * (du + np.swapaxes(du, -1, -2))


def _bwd_div(s):
    """sum_j s_ij(x) - s_ij(x - e^j), eq. 1; s: (L, L, 2, 2)."""
    return (s[..., :, 0] - np.roll(s[..., :, 0], 1, axis=1)
            + s[..., :, 1] - np.roll(s[..., :, 1], 1, axis=0))


def _embed(a2):
    a = np.zeros(a2.shape[:-2] + (3, 3))
    a[..., :2, :2] = a2
    return a


@pytest.mark.parametrize("L", [8, 12, 16])
def test_compatible_field_is_reproduced(L):
    """For eps = forward-difference strain of any u: e = G * (-C0:eps) = eps.

    Pins the momentum convention k_j = 2 sin(q/2) e^{iq/2} against eq. 1, the
    DFT sign convention, and the sign of G."""
    rng = np.random.default_rng(L)
    u = rng.normal(size=(L, L, 2))
    eps = _fwd_diff_strain(u)
    s = alm.Solver(np.zeros((L, L), np.uint8), alm.Params(L=L, mu0=MU0, lam0=LAM0))
    tau2 = -np.einsum("klmn,...mn->...kl", C_iso(LAM0, MU0), eps)
    e = s.green_step(_embed(tau2), (0.0, 0.0, 0.0))
    assert np.abs(e[..., :2, :2] - eps).max() < 1e-12
    assert np.abs(e[..., 2, :]).max() == 0.0


@pytest.mark.parametrize("L", [8, 16])
def test_green_step_gives_equilibrium_and_mean(L):
    """sigma = C0:e + tau with e = E + G*tau is divergence-free with the
    backward differences of eq. 1 at every pixel, and <e> = E."""
    rng = np.random.default_rng(100 + L)
    t = rng.normal(size=(L, L, 2, 2))
    tau2 = 0.5 * (t + np.swapaxes(t, -1, -2))
    E = (0.3, -0.2, 0.15)
    s = alm.Solver(np.zeros((L, L), np.uint8), alm.Params(L=L, mu0=MU0, lam0=LAM0))
    e = s.green_step(_embed(tau2), E)
    sig = np.einsum("klmn,...mn->...kl", C_iso(LAM0, MU0), e[..., :2, :2]) + tau2
    assert np.abs(_bwd_div(sig)).max() < 1e-12
    np.testing.assert_allclose(e.mean(axis=(0, 1))[:2, :2], [[0.3, 0.15], [0.15, -0.2]], atol=1e-14)


def test_compatibility_of_green_output():
    """G*tau is a forward-difference strain: its Saint-Venant incompatibility
    (the discrete curl-curl built from forward differences) vanishes."""
    L = 16
    rng = np.random.default_rng(7)
    t = rng.normal(size=(L, L, 2, 2))
    tau2 = 0.5 * (t + np.swapaxes(t, -1, -2))
    s = alm.Solver(np.zeros((L, L), np.uint8), alm.Params(L=L, mu0=MU0, lam0=LAM0))
    e = s.green_step(_embed(tau2), (0.0, 0.0, 0.0))[..., :2, :2]
    # eps11 = D1 u1, eps22 = D2 u2, 2 eps12 = D1 u2 + D2 u1, with D forward
    # differences that commute: D2 D2 eps11 + D1 D1 eps22 - 2 D1 D2 eps12 = 0.
    D1 = lambda f: np.roll(f, -1, axis=1) - f
    D2 = lambda f: np.roll(f, -1, axis=0) - f
    inc = D2(D2(e[..., 0, 0])) + D1(D1(e[..., 1, 1])) - 2 * D1(D2(e[..., 0, 1]))
    assert np.abs(inc).max() < 1e-12


def test_continuum_limit():
    """G(q) -> -Gamma0(q) (Moulinec-Suquet) as q -> 0 (Sec. 2), error O(q)."""
    errs = []
    for L in (64, 256, 1024):
        m = np.array([[1, 0], [1, 1], [2, -1]])
        q = 2 * np.pi * m / L
        k = 2 * np.sin(q / 2) * np.exp(0.5j * q)
        G = dg.green_tensor(k, LAM0, MU0)
        Gam = dg.continuum_gamma0(q, LAM0, MU0)
        errs.append(np.abs(G + Gam).max() / np.abs(Gam).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2
    assert errs[0] / errs[2] > 10   # at least first-order convergence


def test_dg1_is_real():
    G1 = dg.green_dg1_on_grid(16, LAM0, MU0)
    assert np.abs(G1.imag).max() < 1e-15


@pytest.mark.parametrize("lam0,mu0", [(LAM0, MU0), (0.7, 0.3)])
def test_green_and_dg1_closed_forms_at_nyquist_points(lam0, mu0):
    """Hand-derived values at the self-conjugate points q = (pi, 0) and
    (pi, pi), where k = 2i on each Nyquist axis and k(-q) = -conj k(q) = k(q),
    so the four sign variants coincide.

    q = (pi, 0), k = (2i, 0): the acoustic tensor is diag(4 lam0 + 8 mu0,
    4 mu0); a unit hydrostatic tau gives eps11 = -1/(lam0 + 2 mu0) (the
    longitudinal wave) and nothing else, a unit tau12 gives eps12 =
    -1/(2 mu0) (the transverse wave).  q = (pi, pi), k = 2i (1, 1): a unit
    hydrostatic tau gives eps11 = eps22 = eps12 = -1/(2 (lam0 + 2 mu0)) with
    eq. 3; in DG1 the sign (-1)^(i+j+k+l) of the two mixed variants cancels
    the eps12 response to the diagonal of tau, and keeps the rest.
    """
    L = 8
    h = L // 2
    G = dg.green_on_grid(L, lam0, mu0, 0)
    G1 = dg.green_dg1_on_grid(L, lam0, mu0)
    hyd = np.eye(2)
    shear = np.array([[0.0, 1.0], [1.0, 0.0]])

    def apply(T, m2, m1, tau):
        return np.einsum("ijkl,kl->ij", T[m2, m1], tau)

    long_ = -1.0 / (lam0 + 2.0 * mu0)
    for T in (G, G1):
        np.testing.assert_allclose(apply(T, 0, h, hyd), [[long_, 0.0], [0.0, 0.0]], atol=1e-14)
        np.testing.assert_allclose(apply(T, 0, h, shear), [[0.0, -0.5 / mu0], [-0.5 / mu0, 0.0]], atol=1e-14)
    diag = -0.5 / (lam0 + 2.0 * mu0)
    np.testing.assert_allclose(apply(G, h, h, hyd), [[diag, diag], [diag, diag]], atol=1e-14)
    np.testing.assert_allclose(apply(G1, h, h, hyd), [[diag, 0.0], [0.0, diag]], atol=1e-14)


def test_fourier_divergence_equals_real_space():
    """The paper evaluates <|div sigma|^2> in Fourier space; Parseval makes it
    equal to the real-space backward-difference form."""
    rng = np.random.default_rng(9)
    L = 16
    a = rng.normal(size=(L, L, 3, 3))
    sig = 0.5 * (a + np.swapaxes(a, -1, -2))
    real = np.mean(np.sum(alm.divergence(sig) ** 2, axis=-1))
    four = alm.divergence_fourier(sig)
    assert abs(real - four) < 1e-12 * real


def test_cg1_is_the_continuum_projection():
    """-G of CG1 is the continuum Gamma0 at every non-Nyquist frequency: G C0 G = -G
    (Gamma0 C0 Gamma0 = Gamma0), real, with major symmetry; Nyquist modes carry nothing."""
    L = 16
    G = dg.green_cg1_on_grid(L, LAM0, MU0)
    C = dg.stiffness_2d(LAM0, MU0)
    GCG = np.einsum("...ijkl,klmn,...mnpq->...ijpq", G, C, G)
    sel = np.ones((L, L // 2 + 1), bool)
    sel[0, 0] = False
    sel[:, L // 2] = False
    sel[L // 2, :] = False
    assert np.abs(GCG[sel] + G[sel]).max() < 1e-14
    assert not np.iscomplexobj(G) or np.abs(G.imag).max() == 0.0
    assert np.abs(G - np.transpose(G, (0, 1, 4, 5, 2, 3))).max() < 1e-15
    assert np.all(G[~sel] == 0.0)
    # on the long-wavelength modes the discrete tensor of eq. 3 approaches CG1
    Gd = dg.green_on_grid(L, LAM0, MU0, 0)
    assert np.abs(Gd[1, 1] - G[1, 1]).max() < 0.2 * np.abs(G[1, 1]).max()


def test_dg1_and_cg1_solves_commute_with_the_x1_mirror():
    """DG1 and CG1 are proper tensors under the lattice mirror, unlike eq. 3:
    the solve on a mask mirrored in x1 with E12 -> -E12 is the mirrored solve
    with the 12 components negated, iterate by iterate."""
    from oracle import alm
    from paper_0802_2488_amd import synth
    L = 16
    mask = synth.bernoulli_mask(L, 0.2, 5)
    mir = lambda a: a[:, (-np.arange(L)) % L]  # noqa: E731
    E = (0.3, 0.1, 0.2)
    for v in (4, 5):
        a = alm.Solver(mask, alm.Params(L=L, green_variant=v)).step(E, fixed_iters=10)
        b = alm.Solver(mir(mask), alm.Params(L=L, green_variant=v)).step((E[0], E[1], -E[2]), fixed_iters=10)
        ref = mir(a.sigma).copy()
        ref[..., 0, 1] *= -1
        ref[..., 1, 0] *= -1
        assert np.abs(b.sigma - ref).max() < 1e-12
    # the plain tensor of eq. 3 is not mirror symmetric in this sense
    a = alm.Solver(mask, alm.Params(L=L)).step(E, fixed_iters=10)
    b = alm.Solver(mir(mask), alm.Params(L=L)).step((E[0], E[1], -E[2]), fixed_iters=10)
    ref = mir(a.sigma).copy()
    ref[..., 0, 1] *= -1
    ref[..., 1, 0] *= -1
    assert np.abs(b.sigma - ref).max() > 1e-3


def test_five_point_average():
    """CG2's post-processing: each pixel and its four neighbours (periodic)."""
    rng = np.random.default_rng(3)
    a = rng.normal(size=(8, 8, 2, 2))
    b = dg.five_point_average(a)
    y, x = 3, 0
    ref = (a[y, x] + a[y, 1] + a[y, 7] + a[2, x] + a[4, x]) / 5.0
    assert np.abs(b[y, x] - ref).max() < 1e-15
    assert np.abs(b.mean(axis=(0, 1)) - a.mean(axis=(0, 1))).max() < 1e-15   # averages are kept
    c = np.ones((8, 8))
    c[::2, ::2] = c[1::2, 1::2] = -1.0      # a checkerboard is damped to 3/5 of its amplitude
    assert np.abs(dg.five_point_average(c) + 0.6 * c).max() < 1e-15


def test_continuum_divergence_of_plane_waves():
    """The CG1 equilibrium indicator (continuum divergence in Fourier space):
    sigma_11 = A cos(2 pi k x1 / L) has d1 sigma_11 = -A (2 pi k / L) sin(.),
    mean square A^2 (2 pi k / L)^2 / 2; sigma_12 = B cos(2 pi k x2 / L) enters
    div_1 only (through d2), with B^2 (2 pi k / L)^2 / 2; a Nyquist
    oscillation (-1)^x1, on which CG1 imposes nothing, counts zero."""
    L, k, A, B = 16, 3, 0.7, -1.3
    x = np.arange(L)
    sig = np.zeros((L, L, 3, 3))
    sig[..., 0, 0] = A * np.cos(2 * np.pi * k * x / L)[None, :]
    assert alm.mean_div2_continuum(sig) == pytest.approx(A * A * (2 * np.pi * k / L) ** 2 / 2, rel=1e-12)
    sig = np.zeros((L, L, 3, 3))
    sig[..., 0, 1] = sig[..., 1, 0] = B * np.cos(2 * np.pi * k * x / L)[:, None]
    assert alm.mean_div2_continuum(sig) == pytest.approx(B * B * (2 * np.pi * k / L) ** 2 / 2, rel=1e-12)
    sig = np.zeros((L, L, 3, 3))
    sig[..., 0, 0] = ((-1.0) ** x)[None, :]
    sig[..., 1, 1] = 2.0
    assert alm.mean_div2_continuum(sig) < 1e-28


def test_cg1_converges_on_its_own_equilibrium():
    """CG1 reaches 1e-8 on all three indicators with the continuum divergence,
    while the backward differences of eq. 1 stay far from equilibrium."""
    L = 16
    mask = synth.bernoulli_mask(L, 0.1, 5)
    p = alm.Params(L=L, mu0=0.04, lam0=0.08, max_iter=20000, green_variant=5)
    s = alm.Solver(mask, p)
    r = s.step((0.2, 0.2, 0.0))
    assert r.converged and r.res_eq < 1e-8
    back = np.sqrt(np.mean(np.sum(alm.divergence(r.sigma) ** 2, axis=-1))) / alm.norm3(r.sigma_mean)
    assert back > 1e-3
