"""Discrete Green tensor of the strain (Sec. 2, "Discrete Green functions").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (eq. 2): momenta q_j = 2 pi m_j / L, m_j = 0..L-1, and the discrete
wave vector k_j = 2 sin(q_j / 2) exp(i q_j / 2).  A field is expanded as
f(x) = sum_q f(q) exp(+i q.x) (numpy's inverse-transform sign), so the forward
difference f(x + e^j) - f(x) becomes i k_j f(q) and the backward difference
f(x) - f(x - e^j) becomes i conj(k_j) f(q).

Array layout: real fields are indexed [x2][x1] (x1 is the contiguous axis and
the direction of e^1); tensor index 0 is direction 1 and index 1 is
direction 2.  Half spectra from a real 2-D FFT over axes (0, 1) are indexed
[m2][m1] with m1 = 0..L/2.
"""
from __future__ import annotations

import numpy as np


def wave_vector(L: int, sign: int = 1) -> np.ndarray:
    """k(m) = 2 sin(q/2) exp(i q/2) at q = sign * 2 pi m / L, m = 0..L-1 (eq. 2).

    sign = -1 evaluates the momentum -q, as needed by the sign-flipped Green
    tensors of the DG1 and DG2 schemes.
    """
    q = sign * 2.0 * np.pi * np.arange(L) / L
    return 2.0 * np.sin(q / 2.0) * np.exp(0.5j * q)


def stiffness_2d(lam0: float, mu0: float) -> np.ndarray:
    """Isotropic stiffness C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk),
    restricted to in-plane indices i, j, k, l in {1, 2} (generalized plane
    strain: q_3 = 0, only indices 1, 2 kept; Sec. 2 after eq. 3)."""
    d = np.eye(2)
    return (lam0 * np.einsum("ij,kl->ijkl", d, d)
            + mu0 * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def acoustic_tensor(k: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """N_ij = conj(k_k) C_iklj k_l (Sec. 2, after eq. 3).  k has shape (..., 2)."""
    C = stiffness_2d(lam0, mu0)
    return np.einsum("...k,iklj,...l->...ij", np.conj(k), C, k)


def green_tensor(k: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Discrete Green tensor of eq. 3 at wave vectors k (shape (..., 2)).

    G_ijkl = -(Ninv_jl k_i k*_k + Ninv_il k_j k*_k + Ninv_jk k_i k*_l
              + Ninv_ik k_j k*_l) / 4,
    with N inverted numerically (the paper inverts it numerically as well).
    Entries where k = 0 (the q = 0 mode) are returned as zero; the mean strain
    is imposed separately.  Output shape (..., 2, 2, 2, 2).
    """
    N = acoustic_tensor(k, lam0, mu0)
    zero = np.all(np.abs(k) == 0.0, axis=-1)
    Nsafe = np.where(zero[..., None, None], np.eye(2), N)
    Ni = np.linalg.inv(Nsafe)
    kc = np.conj(k)
    G = -(np.einsum("...jl,...i,...k->...ijkl", Ni, k, kc)
          + np.einsum("...il,...j,...k->...ijkl", Ni, k, kc)
          + np.einsum("...jk,...i,...l->...ijkl", Ni, k, kc)
          + np.einsum("...ik,...j,...l->...ijkl", Ni, k, kc)) / 4.0
    G[zero] = 0.0
    return G


def half_spectrum_k(L: int, flip1: bool = False, flip2: bool = False) -> np.ndarray:
    """Wave vectors on the rfft2 half-spectrum grid, shape (L, L//2+1, 2).

    flip1 / flip2 evaluate k at -q1 / -q2 (the variants G(-q1, q2), ...)."""
    k1 = wave_vector(L, -1 if flip1 else 1)[: L // 2 + 1]
    k2 = wave_vector(L, -1 if flip2 else 1)
    K = np.empty((L, L // 2 + 1, 2), dtype=complex)
    K[..., 0] = k1[None, :]
    K[..., 1] = k2[:, None]
    return K


def green_on_grid(L: int, lam0: float, mu0: float, variant: int = 0) -> np.ndarray:
    """G(q) of eq. 3 on the half spectrum, shape (L, L//2+1, 2, 2, 2, 2).

    variant 0: G(q1, q2); 1: G(-q1, -q2); 2: G(-q1, q2); 3: G(q1, -q2), the
    four tensors that the DG2 scheme uses in turn (Sec. 2, after eq. 4).
    """
    flips = {0: (False, False), 1: (True, True), 2: (True, False), 3: (False, True)}[variant]
    return green_tensor(half_spectrum_k(L, *flips), lam0, mu0)


def green_dg1_on_grid(L: int, lam0: float, mu0: float) -> np.ndarray:
    """Symmetrised DG1 tensor of eq. 4 on the half spectrum.

    G1 = {G(q1,q2) + G(-q1,-q2) + (-1)^(i+j+k+l) [G(-q1,q2) + G(q1,-q2)]} / 4.
    Pinned by hand-derived closed forms at the self-conjugate points (pi, 0)
    and (pi, pi), by being real valued and by its mirror symmetry.
    """
    G0, G1, G2, G3 = (green_on_grid(L, lam0, mu0, v) for v in range(4))
    idx = np.indices((2, 2, 2, 2)).sum(axis=0)   # i+j+k+l with 0-based indices
    sign = (-1.0) ** idx                           # same parity as 1-based sum
    return (G0 + G1 + sign * (G2 + G3)) / 4.0


def frequencies(L: int) -> np.ndarray:
    """Continuum frequencies of the DFT bins: 2 pi m / L for m < L/2, 2 pi (m - L) / L
    for m > L/2 (the Nyquist bin m = L/2 is handled by the caller)."""
    m = np.arange(L)
    return 2.0 * np.pi * np.where(m < L // 2, m, m - L) / L


def green_cg1_on_grid(L: int, lam0: float, mu0: float) -> np.ndarray:
    """CG1 (Sec. 2): the continuum Green operator, G = -Gamma0(xi), on the half
    spectrum, with xi the continuum frequencies of the bins.  Modes with a
    Nyquist component (m1 = L/2 or m2 = L/2) carry no strain (G = 0) and
    q = 0 is set by the caller; both are readings (the paper only names the
    method).
    """
    xi = frequencies(L)
    X = np.zeros((L, L // 2 + 1, 2))
    X[..., 0] = xi[None, : L // 2 + 1]
    X[..., 1] = xi[:, None]
    X[0, 0] = (1.0, 0.0)            # placeholder for q = 0, overwritten below
    G = -continuum_gamma0(X, lam0, mu0)
    G[0, 0] = 0.0
    G[:, L // 2] = 0.0
    G[L // 2, :] = 0.0
    return G


def green_variant_on_grid(L: int, lam0: float, mu0: float, variant: int) -> np.ndarray:
    """Green tensor of variant 0..3 (sign variants of eq. 3), 4 (DG1) or 5 (CG1)."""
    if variant == 4:
        return green_dg1_on_grid(L, lam0, mu0)
    if variant == 5:
        return green_cg1_on_grid(L, lam0, mu0)
    return green_on_grid(L, lam0, mu0, variant)


def apply_green(G: np.ndarray, tau_hat: np.ndarray) -> np.ndarray:
    """e_hat_ij = G_ijkl tau_hat_kl on the half spectrum (tau_hat: (..., 2, 2))."""
    return np.einsum("...ijkl,...kl->...ij", G, tau_hat)


def continuum_gamma0(xi: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Continuum Green operator Gamma0(xi) of an isotropic medium in 2D plane
    strain (the Moulinec-Suquet operator the paper calls CG1; Sec. 2).

    Gamma0_khij = [d_ki xi_h xi_j + d_hi xi_k xi_j + d_kj xi_h xi_i
                   + d_hj xi_k xi_i] / (4 mu0 |xi|^2)
                  - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) xi_i xi_j xi_k xi_h / |xi|^4,
    returned with indices ordered [k, h, i, j].  The discrete tensor of eq. 3
    tends to -Gamma0 in the long-wavelength limit (Sec. 2).
    """
    d = np.eye(2)
    x2 = np.sum(xi * xi, axis=-1)[..., None, None, None, None]
    t1 = (np.einsum("ki,...h,...j->...khij", d, xi, xi)
          + np.einsum("hi,...k,...j->...khij", d, xi, xi)
          + np.einsum("kj,...h,...i->...khij", d, xi, xi)
          + np.einsum("hj,...k,...i->...khij", d, xi, xi))
    t2 = np.einsum("...i,...j,...k,...h->...khij", xi, xi, xi, xi)
    return t1 / (4.0 * mu0 * x2) - (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) * t2 / x2 ** 2


def five_point_average(a: np.ndarray) -> np.ndarray:
    """CG2 (Sec. 2): the average of a field over each pixel and its four
    nearest neighbours, periodic; axes 0, 1 are x2, x1."""
    return (a + np.roll(a, 1, axis=1) + np.roll(a, -1, axis=1) + np.roll(a, 1, axis=0)
            + np.roll(a, -1, axis=0)) / 5.0
