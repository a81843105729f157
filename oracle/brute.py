"""FFT-free brute-force solution of the discrete problem on tiny grids.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The discrete problem of eq. 1 is the stationarity condition of the total
strain energy W(u) = sum_x w(eps(x)) over periodic displacements u, with
eps = E + forward-difference symmetric gradient of u and w = 0 on voids:
by summation by parts the derivative of W is minus the backward-difference
divergence of sigma.  W is convex and C^1, so minimising it gives the
solution without any Fourier transform, Green tensor or Lagrangian.

Elastic loading: the normal equations B^T D B u = -B^T D E are solved with a
least-squares routine (the system is singular: rigid translations and the
displacements of isolated void pixels are free).  Plastic loading: W is
minimised with L-BFGS using the exact gradient.  The stress is unique, the
displacement is not, so results are compared on sigma.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse as sp

from . import hencky


def strain_operator(L: int) -> sp.csr_matrix:
    """Sparse B with eps_vec = B u, eps_vec = (eps11, eps22, eps12) per pixel.

    u is ordered (x2, x1, component); eps_ij = [u_j(x+e^i) - u_j(x)
    + u_i(x+e^j) - u_i(x)] / 2 (eq. 1), direction 1 = x1, direction 2 = x2.
    """
    rows, cols, vals = [], [], []

    def uidx(x2, x1, c):
        return ((x2 % L) * L + (x1 % L)) * 2 + c

    for x2 in range(L):
        for x1 in range(L):
            p = x2 * L + x1
            # eps11 = u1(x + e1) - u1(x)
            rows += [3 * p, 3 * p]
            cols += [uidx(x2, x1 + 1, 0), uidx(x2, x1, 0)]
            vals += [1.0, -1.0]
            # eps22 = u2(x + e2) - u2(x)
            rows += [3 * p + 1, 3 * p + 1]
            cols += [uidx(x2 + 1, x1, 1), uidx(x2, x1, 1)]
            vals += [1.0, -1.0]
            # eps12 = [u2(x + e1) - u2(x) + u1(x + e2) - u1(x)] / 2
            rows += [3 * p + 2] * 4
            cols += [uidx(x2, x1 + 1, 1), uidx(x2, x1, 1), uidx(x2 + 1, x1, 0), uidx(x2, x1, 0)]
            vals += [0.5, -0.5, 0.5, -0.5]
    n = L * L
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * n, 2 * n))


def _to_tensor(ev):
    """(n, 3) plane-strain components -> (n, 3, 3) with eps33 = 0."""
    t = np.zeros(ev.shape[:-1] + (3, 3))
    t[..., 0, 0], t[..., 1, 1] = ev[..., 0], ev[..., 1]
    t[..., 0, 1] = t[..., 1, 0] = ev[..., 2]
    return t


def solve_elastic(mask, E, mu, lam):
    """Linear-elastic solution by least squares; returns sigma (L, L, 3, 3)."""
    L = mask.shape[0]
    B = strain_operator(L).toarray()
    n = L * L
    m = (~mask.astype(bool)).reshape(n).astype(float)
    # w = lam/2 (e11+e22)^2 + mu (e11^2 + e22^2 + 2 e12^2) on matrix pixels.
    Dp = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, 4 * mu]])
    D = np.kron(np.diag(m), Dp)
    Ev = np.tile(np.asarray(E, float), n)
    A = B.T @ D @ B
    b = -B.T @ D @ Ev
    u = np.linalg.lstsq(A, b, rcond=None)[0]
    ev = (Ev + B @ u).reshape(n, 3)
    eps = _to_tensor(ev).reshape(L, L, 3, 3)
    sig = hencky.iso(lam, mu, eps)
    return np.where(mask.astype(bool)[..., None, None], 0.0, sig)


def solve_plastic(mask, E, mu, lam, Y, gtol=1e-13, maxiter=200000):
    """Minimise W(u) with L-BFGS; returns (sigma (L, L, 3, 3), W, info)."""
    L = mask.shape[0]
    n = L * L
    B = strain_operator(L)
    Ev = np.tile(np.asarray(E, float), n)
    v = mask.astype(bool).reshape(n)

    def fun(u):
        ev = (Ev + B @ u).reshape(n, 3)
        eps = _to_tensor(ev)
        w = hencky.energy(eps, mu, lam, Y)
        w[v] = 0.0
        sig = hencky.stress(eps, mu, lam, Y)
        sig[v] = 0.0
        # dW/d(eps11, eps22, eps12) = (sig11, sig22, 2 sig12)
        g = np.stack([sig[:, 0, 0], sig[:, 1, 1], 2.0 * sig[:, 0, 1]], axis=-1).reshape(-1)
        return float(w.sum()), B.T @ g

    res = scipy.optimize.minimize(fun, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                                  options=dict(maxiter=maxiter, maxcor=50, gtol=gtol,
                                               ftol=1e-300, maxfun=maxiter * 2))
    ev = (Ev + B @ res.x).reshape(n, 3)
    eps = _to_tensor(ev)
    sig = hencky.stress(eps, mu, lam, Y)
    sig[v] = 0.0
    return sig.reshape(L, L, 3, 3), res.fun, res


def total_energy(eps, mask, mu, lam, Y):
    """W = sum over matrix pixels of w(eps)."""
    w = hencky.energy(eps, mu, lam, Y)
    return float(np.where(mask.astype(bool), 0.0, w).sum())
