"""Elastic-perfectly plastic Mises law in deformation theory (Hencky) and the
pointwise step of the augmented Lagrangian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2 (first paragraph) and Sec. 3: matrix pixels are elastic-perfectly
plastic with flow stress Y under deformation theory; void pixels carry zero
stress; the plastic zone is where the Mises norm of the stress equals Y.
Fig. 1 defines the equivalent strain eps_eq = [(2/3) e'_ij e'_ij]^(1/2) with
the three-dimensional deviator e' = eps - I tr(eps) / 3.

All tensors here are full 3 x 3 arrays (..., 3, 3); in plane strain the
components 13 and 23 are zero and 33 is tracked.
"""
from __future__ import annotations

import numpy as np

I3 = np.eye(3)
SQRT23 = np.sqrt(2.0 / 3.0)


def trace(a):
    return np.trace(a, axis1=-2, axis2=-1)


def deviator(a):
    return a - trace(a)[..., None, None] * I3 / 3.0


def frob2(a):
    """A:A summed over all nine components (so 12 and 21 both count)."""
    return np.sum(a * a, axis=(-2, -1))


def bulk_modulus(lam, mu):
    """Three-dimensional bulk modulus K = lambda + 2 mu / 3."""
    return lam + 2.0 * mu / 3.0


def iso(lam, mu, a):
    """C:a for the isotropic stiffness: lambda tr(a) I + 2 mu a."""
    return lam * trace(a)[..., None, None] * I3 + 2.0 * mu * a


def iso_inv(lam, mu, a):
    """C^-1 : a for the isotropic stiffness."""
    tr_eps = trace(a) / (3.0 * lam + 2.0 * mu)
    return (a - lam * tr_eps[..., None, None] * I3) / (2.0 * mu)


def eps_eq(eps):
    """Equivalent strain of Fig. 1: sqrt(2/3 e':e')."""
    return np.sqrt(2.0 / 3.0 * frob2(deviator(eps)))


def sigma_eq(sig):
    """Mises norm of the stress: sqrt(3/2 s:s)."""
    return np.sqrt(1.5 * frob2(deviator(sig)))


def stress(eps, mu, lam, Y):
    """Hencky-Mises stress S(eps) of a matrix pixel.

    Volumetric part K tr(eps) I; deviatoric part 2 mu e' while the elastic
    Mises stress 3 mu eps_eq stays at or below Y, else the deviator is capped
    at Mises norm Y along e' (perfect plasticity, deformation theory).
    """
    K = bulk_modulus(lam, mu)
    e = deviator(eps)
    ne = np.sqrt(frob2(e))
    elastic = 2.0 * mu * ne <= SQRT23 * Y
    scale = np.where(elastic, 2.0 * mu, SQRT23 * Y / np.where(elastic, 1.0, ne))
    return K * trace(eps)[..., None, None] * I3 + scale[..., None, None] * e


def energy(eps, mu, lam, Y):
    """Strain-energy density w(eps) whose gradient is S (pins S).

    w = K/2 tr^2 + mu e':e' in the elastic range, else
    w = K/2 tr^2 + Y eps_eq - Y^2 / (6 mu).  C^1 and convex.
    """
    K = bulk_modulus(lam, mu)
    tr = trace(eps)
    q = eps_eq(eps)
    elastic = 3.0 * mu * q <= Y
    dev = np.where(elastic, 1.5 * mu * q * q, Y * q - Y * Y / (6.0 * mu))
    return 0.5 * K * tr * tr + dev


def pointwise_solve(R, void, mu, lam, Y, mu0, lam0):
    """Pointwise step of the augmented Lagrangian: solve S(eps) + C0:eps = R.

    Matrix pixels: the volumetric part gives tr(eps) = tr(R) / (3 (K + K0));
    with r = dev R and rho = |r|, the trial (elastic) solution
    dev eps = r / (2 (mu + mu0)) holds while 2 mu |dev eps| <= sqrt(2/3) Y,
    i.e. rho <= sqrt(2/3) Y (mu + mu0) / mu (ties count as elastic); beyond
    it the stress deviator is sqrt(2/3) Y r / rho and
    dev eps = (r - s) / (2 mu0).
    Void pixels carry zero stress, so C0:eps = R.

    Returns (eps, plastic, margin) where margin is the trial Mises stress
    minus Y (positive on the capped branch).
    """
    K = bulk_modulus(lam, mu)
    K0 = bulk_modulus(lam0, mu0)
    tr_eps = trace(R) / (3.0 * (K + K0))
    r = deviator(R)
    rho = np.sqrt(frob2(r))
    margin = np.sqrt(1.5) * mu * rho / (mu + mu0) - Y
    plastic = rho > SQRT23 * Y * (mu + mu0) / mu
    safe_rho = np.where(plastic, rho, 1.0)
    s_pl = (SQRT23 * Y / safe_rho)[..., None, None] * r
    dev_el = r / (2.0 * (mu + mu0))
    dev_pl = (r - s_pl) / (2.0 * mu0)
    dev = np.where(plastic[..., None, None], dev_pl, dev_el)
    eps_m = dev + tr_eps[..., None, None] * I3 / 3.0
    eps_v = iso_inv(lam0, mu0, R)
    v = void.astype(bool)
    eps = np.where(v[..., None, None], eps_v, eps_m)
    plastic = plastic & ~v
    margin = np.where(v, -np.inf, margin)
    return eps, plastic, margin


def field_stress(eps, void, mu, lam, Y):
    """Stress field: S(eps) on matrix pixels, exactly zero on voids (Sec. 3)."""
    sig = stress(eps, mu, lam, Y)
    return np.where(void.astype(bool)[..., None, None], 0.0, sig)
