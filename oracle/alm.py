"""Augmented-Lagrangian Lippmann-Schwinger iteration with the discrete Green
tensor (Sec. 1 and Sec. 2), FP64, on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The discrete problem (Sec. 2, eq. 1): find a periodic displacement on the
L x L lattice such that eps = E + (forward-difference symmetric gradient of u),
sigma = S(eps) on matrix pixels and 0 on voids, and the backward-difference
divergence of sigma vanishes at every pixel.

The method (Sec. 1: Lippmann-Schwinger equation in a homogeneous reference
medium, polarisation computed pointwise in direct space, convolution done by
FFT, convergence improved by an augmented Lagrangian with Uzawa's algorithm).
The paper does not print the augmented-Lagrangian steps; the reading used here
is the published Michel-Moulinec-Suquet scheme, with reference stiffness C0:

  (a) tau = lambda - C0:eps;  e = E + G * tau  (G of eq. 3, built from C0,
      applied in Fourier space; the q = 0 mode carries E);
  (b) pointwise: S(eps) + C0:eps = lambda + C0:e  (voids: S = 0);
  (c) lambda <- lambda + C0:(e - eps).

Started from eps = E, lambda = S(E) on matrix pixels and 0 on voids; later
load steps keep (lambda, eps) and only change E.

Convergence (Sec. 2, "Convergence issues"): eta_1 tests
<|div sigma|^2> against <sigma>:<sigma> (div computed with the backward
differences of eq. 1), eta_2 tests the change of <sigma> between consecutive
iterations.  A third test on the augmented-Lagrangian constraint e = eps is
added.  All three must hold at the same iteration (iteration >= 2).
"""
from __future__ import annotations

import dataclasses
import os

import numpy as np
import scipy.fft as sfft

from . import dg, hencky

# FFT threads: the cores this process may run on (the FFT is a library step;
# the pointwise arithmetic stays plain single-threaded numpy).  Grids below
# 512 use one thread, where starting threads costs more than it saves.
FFT_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def fft_workers(L):
    return FFT_WORKERS if L >= 512 else 1


@dataclasses.dataclass
class Params:
    L: int
    mu: float = 1.0
    lam: float = 2.0
    Y: float = 1.0
    mu0: float = 0.0          # 0 -> 2 mu
    lam0: float = 0.0         # 0 -> 2 lambda
    eta_eq: float = 1e-8
    eta_mac: float = 1e-8
    eta_cmp: float = 1e-8
    max_iter: int = 50000
    green_variant: int = 0    # 0..3: G(q1,q2), G(-q1,-q2), G(-q1,q2), G(q1,-q2); 4: DG1; 5: CG1

    def __post_init__(self):
        if self.mu0 == 0.0:
            self.mu0 = 2.0 * self.mu
        if self.lam0 == 0.0:
            self.lam0 = 2.0 * self.lam


def tensor_from_voigt(E3):
    """(E11, E22, E12) with E33 = E13 = E23 = 0 as a 3 x 3 tensor."""
    E = np.zeros((3, 3))
    E[0, 0], E[1, 1] = E3[0], E3[1]
    E[0, 1] = E[1, 0] = E3[2]
    return E


def norm3(a):
    """Frobenius norm of a 3 x 3 tensor (12 and 21 both count)."""
    return float(np.sqrt(np.sum(np.asarray(a) ** 2)))


FLIPS = {0: (False, False), 1: (True, True), 2: (True, False), 3: (False, True)}


def divergence(sig, flip1=False, flip2=False):
    """Discrete divergence of eq. 1: sum_j sigma_ij(x) - sigma_ij(x - e^j).

    sig: (L, L, 3, 3) indexed [x2][x1]; returns (L, L, 2) for i = 1, 2.
    Direction 1 is axis 1 (x1), direction 2 is axis 0 (x2).

    flip1 / flip2: the divergence of the sign-flipped Green tensors of DG2
    (Sec. 2).  G(-q1, q2) evaluates k_1 of eq. 2 at -q1, i.e. -conj(k_1(q1)),
    so its strains are the differences u(x - e^1) - u(x) and the equilibrium
    they are orthogonal to uses i conj(k_1(-q1)) = -i k_1(q1): the difference
    sigma_i1(x) - sigma_i1(x + e^1) along that direction.
    """
    s = sig[..., :2, :2]
    d1 = s[..., :, 0] - np.roll(s[..., :, 0], -1 if flip1 else 1, axis=1)   # j = 1
    d2 = s[..., :, 1] - np.roll(s[..., :, 1], -1 if flip2 else 1, axis=0)   # j = 2
    return d1 + d2


def mean_div2_continuum(sig):
    """<|div sigma|^2> with the continuum divergence of the CG1 scheme,
    evaluated in Fourier space as the paper does (Sec. 2, "Convergence
    issues"): i xi_j sigma_ij(q) with xi the continuum frequencies of the
    bins; the modes with a Nyquist component, on which the continuum Green
    operator imposes nothing, are left out.  Parseval with the unnormalised
    DFT: the mean over the pixels is the sum over the modes divided by L^4.
    """
    L = sig.shape[0]
    S = sfft.fft2(sig[..., :2, :2], axes=(0, 1), workers=fft_workers(L))
    xi = dg.frequencies(L)
    keep = np.arange(L) != L // 2
    x1 = xi[None, :]
    x2 = xi[:, None]
    v = x1[..., None] * S[..., :, 0] + x2[..., None] * S[..., :, 1]
    w = (keep[None, :] & keep[:, None]).astype(float)
    return float(np.sum(w[..., None] * np.abs(v) ** 2)) / L ** 4


def divergence_fourier(sig):
    """<|div sigma|^2> evaluated in Fourier space, as the paper computes it.

    With eq. 2 the backward difference is i conj(k_l); Parseval gives
    <|div|^2> = sum_q |conj(k_l) sigma_kl(q)|^2 / L^4 (full spectrum).
    """
    L = sig.shape[0]
    S = sfft.fft2(sig[..., :2, :2], axes=(0, 1), workers=fft_workers(L))
    k1 = dg.wave_vector(L)[None, :]
    k2 = dg.wave_vector(L)[:, None]
    v = np.conj(k1)[..., None] * S[..., :, 0] + np.conj(k2)[..., None] * S[..., :, 1]
    return float(np.sum(np.abs(v) ** 2)) / L ** 4


@dataclasses.dataclass
class StepResult:
    sigma: np.ndarray          # (L, L, 3, 3)
    eps: np.ndarray            # (L, L, 3, 3)
    e: np.ndarray              # compatible strain of the last iteration
    plastic: np.ndarray        # bool (L, L)
    margin: np.ndarray         # trial Mises - Y, -inf on voids
    sigma_mean: np.ndarray     # (3, 3)
    eps_mean: np.ndarray
    iters: int
    converged: bool
    res_eq: float
    res_mac: float
    res_cmp: float


class Solver:
    """One realization: void mask + material + reference medium."""

    def __init__(self, mask, p: Params):
        self.p = p
        self.void = np.asarray(mask).astype(bool)
        L = p.L
        assert self.void.shape == (L, L)
        self.G = dg.green_variant_on_grid(L, p.lam0, p.mu0, p.green_variant)
        self.lam_mult = None   # Lagrange multiplier lambda (L, L, 3, 3)
        self.eps = None
        # equilibrium of the Green tensor in use: the sign variants of DG2
        # take the differences of their own momenta, CG1 the continuum
        # divergence; DG1 (no projection) the backward differences of eq. 1
        self.flips = FLIPS.get(p.green_variant, (False, False))

    # -- building blocks --------------------------------------------------
    def c0(self, a):
        return hencky.iso(self.p.lam0, self.p.mu0, a)

    def green_step(self, tau, E):
        """e = E + G * tau (step (a)); tau and e are (L, L, 3, 3), e33 = 0."""
        L = self.p.L
        t_hat = sfft.rfft2(tau[..., :2, :2], axes=(0, 1), workers=fft_workers(L))
        e_hat = dg.apply_green(self.G, t_hat)
        e_hat[0, 0] = tensor_from_voigt(E)[:2, :2] * (L * L)
        e2 = sfft.irfft2(e_hat, s=(L, L), axes=(0, 1), workers=fft_workers(L))
        e = np.zeros((L, L, 3, 3))
        e[..., :2, :2] = e2
        return e

    def start(self, E):
        """Initial state: eps = E, lambda = S(E) on matrix pixels, 0 on voids."""
        L = self.p.L
        Et = np.broadcast_to(tensor_from_voigt(E), (L, L, 3, 3)).copy()
        self.eps = Et
        self.lam_mult = hencky.field_stress(Et, self.void, self.p.mu, self.p.lam, self.p.Y)

    def iterate(self, E):
        """One augmented-Lagrangian iteration (a), (b), (c).  Returns e, plastic, margin."""
        p = self.p
        tau = self.lam_mult - self.c0(self.eps)
        e = self.green_step(tau, E)
        R = self.lam_mult + self.c0(e)
        eps_new, plastic, margin = hencky.pointwise_solve(
            R, self.void, p.mu, p.lam, p.Y, p.mu0, p.lam0)
        self.lam_mult = self.lam_mult + self.c0(e - eps_new)
        self.eps = eps_new
        return e, plastic, margin

    def equilibrium_indicator(self, sig, ns):
        """eta_1 of the scheme in use: sqrt(<|div sigma|^2>) / |<sigma>|."""
        if self.p.green_variant == 5:
            return float(np.sqrt(mean_div2_continuum(sig))) / ns
        return float(np.sqrt(np.mean(np.sum(divergence(sig, *self.flips) ** 2, axis=-1)))) / ns

    def sigma(self):
        return hencky.field_stress(self.eps, self.void, self.p.mu, self.p.lam, self.p.Y)

    # -- one load step ----------------------------------------------------
    def step(self, E, fixed_iters=None) -> StepResult:
        """Solve at overall strain E = (E11, E22, E12) from the current state.

        fixed_iters: run exactly this many iterations (iteration-locked
        comparison) instead of stopping on the convergence test.
        """
        p = self.p
        L = p.L
        Et = tensor_from_voigt(E)
        nE = norm3(Et)
        if nE == 0.0:
            z = np.zeros((L, L, 3, 3))
            self.eps = z.copy()
            self.lam_mult = z.copy()
            zb = np.zeros((L, L), bool)
            return StepResult(z, z.copy(), z.copy(), zb, np.full((L, L), -np.inf),
                              np.zeros((3, 3)), np.zeros((3, 3)), 0, True, 0.0, 0.0, 0.0)
        if self.eps is None:
            self.start(E)
        floor_s = 1e-12 * p.mu * nE
        prev_mean = None
        it = 0
        converged = False
        r_eq = r_mac = r_cmp = np.inf
        while True:
            e, plastic, margin = self.iterate(E)
            it += 1
            sig = self.sigma()
            smean = sig.mean(axis=(0, 1))
            ns = max(norm3(smean), floor_s)
            r_cmp = float(np.sqrt(np.mean(hencky.frob2(e - self.eps)))) / nE
            if prev_mean is not None:
                r_mac = norm3(smean - prev_mean) / ns
            prev_mean = smean
            if fixed_iters is not None:
                if it >= fixed_iters:
                    r_eq = self.equilibrium_indicator(sig, ns)
                    converged = it >= 2 and r_eq < p.eta_eq and r_mac < p.eta_mac and r_cmp < p.eta_cmp
                    break
                continue
            if it >= 2 and r_mac < p.eta_mac and r_cmp < p.eta_cmp:
                r_eq = self.equilibrium_indicator(sig, ns)
                if r_eq < p.eta_eq:
                    converged = True
                    break
            if it >= p.max_iter:
                r_eq = self.equilibrium_indicator(sig, ns)
                break
        sig = self.sigma()
        return StepResult(sig, self.eps.copy(), e, plastic, margin,
                          sig.mean(axis=(0, 1)), self.eps.mean(axis=(0, 1)),
                          it, converged, r_eq, r_mac, r_cmp)


def solve_path(mask, p: Params, E_path, fixed_iters=None):
    """Solve a load ramp; returns the list of per-step results.

    fixed_iters: optional sequence of iteration counts, one per step.
    """
    s = Solver(mask, p)
    out = []
    for n, E in enumerate(np.asarray(E_path, dtype=float)):
        fi = None if fixed_iters is None else int(fixed_iters[n])
        out.append(s.step(E, fixed_iters=fi))
    return out


def voigt4(a):
    """(..., 3, 3) -> (..., 4) with components (11, 22, 33, 12)."""
    return np.stack([a[..., 0, 0], a[..., 1, 1], a[..., 2, 2], a[..., 0, 1]], axis=-1)


def from_voigt4(v):
    """(..., 4) components (11, 22, 33, 12) -> symmetric (..., 3, 3)."""
    v = np.asarray(v, dtype=float)
    a = np.zeros(v.shape[:-1] + (3, 3))
    a[..., 0, 0], a[..., 1, 1], a[..., 2, 2] = v[..., 0], v[..., 1], v[..., 2]
    a[..., 0, 1] = a[..., 1, 0] = v[..., 3]
    return a
