"""Seeded synthetic inputs: void masks, load ramps and workload mixes.

This module holds no arithmetic of the solution method.  It only draws the
inputs that the method is applied to, so both the HIP path and the CPU oracle
tests take their inputs from here.

Disorder model (Sec. 2, first paragraph): every pixel of the L x L periodic
lattice is independently a void with probability f (pixelwise disorder with
zero correlation length, Sec. 1).  The draw is counter based so that any pixel
can be regenerated on its own, on the host or on the device:

    pixel p = x2 * L + x1 is a void  iff  u(p) < f,
    u(p) = (mix(seed ^ mix(p)) >> 11) * 2**-53,

where mix is the SplitMix64 output function (Steele, Lea and Flood, OOPSLA
2014): z += 0x9E3779B97F4A7C15; z = (z ^ z>>30) * 0xBF58476D1CE4E5B9;
z = (z ^ z>>27) * 0x94D049BB133111EB; return z ^ z>>31.  The device-side
generator in the C library implements the same definition independently.

Load ramps: the overall strain is imposed and increased step by step
(Sec. 2, end of "Discrete Green functions").  Step n of N applies
e_n = n * e_max / N, with E = (e, e, 0) for equibiaxial loading and
E = (0, 0, e) (tensor component eps_12) for simple shear.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output function applied elementwise to uint64 input."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed, counter):
    """Counter-based uniform in [0, 1) with 53 random bits."""
    c = np.asarray(counter, dtype=np.uint64)
    z = splitmix64(np.uint64(seed) ^ splitmix64(c))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def bernoulli_mask(L: int, f: float, seed: int) -> np.ndarray:
    """uint8 array [x2][x1] of shape (L, L); 1 marks a void pixel."""
    p = np.arange(L * L, dtype=np.uint64)
    return (uniform01(seed, p) < f).astype(np.uint8).reshape(L, L)


def circular_void(L: int, f: float) -> np.ndarray:
    """One circular void of area fraction f centred in the periodic cell (the
    single-inclusion cell of Sec. 2's method comparison): pixel (x1, x2) is a
    void iff its centre lies within radius L sqrt(f / pi) of the cell centre."""
    c = np.arange(L) + 0.5 - L / 2.0
    r2 = c[None, :] ** 2 + c[:, None] ** 2
    return (r2 < (L * L) * f / np.pi).astype(np.uint8)


def load_path(kind: str, n_steps: int, e_max: float) -> np.ndarray:
    """(n_steps, 3) array of (E11, E22, E12); step n (1-based) applies n*e_max/N."""
    e = e_max * np.arange(1, n_steps + 1, dtype=np.float64) / n_steps
    E = np.zeros((n_steps, 3))
    if kind == "equibiaxial":
        E[:, 0] = e
        E[:, 1] = e
    elif kind == "shear":
        E[:, 2] = e
    else:
        raise ValueError(f"unknown loading kind {kind!r}")
    return E


def default_emax(kind: str, Y: float, mu: float) -> float:
    """Ramp end point: 3Y/mu for equibiaxial loading, 4Y/mu for shear."""
    return (3.0 if kind == "equibiaxial" else 4.0) * Y / mu


# Workload descriptions (sizes, porosities, loadings) used by the tests and
# the benchmark.  Material constants mu = 1, lambda = 2, Y = 1.  c0 is the
# reference medium (lambda0, mu0) = c0 (lambda, mu): twice the matrix where
# the workload states it, else a soft medium (see C0_SOFT).
MATERIAL = dict(mu=1.0, lam=2.0, Y=1.0)

# Reference-medium scale of the workloads that leave it open: a medium this
# soft balances the augmented-Lagrangian residuals on porous grids (measured
# with the oracle on 64^2 to 128^2 grids of f = 0.1 to 0.3; twice the matrix
# leaves the equilibrium residual near 1e-5 after 2e4 iterations where this
# one reaches 1e-15).  It only sets the iteration count, not the solution.
C0_SOFT = 0.01

WORKLOADS = {
    "fp64_L64": dict(L=64, f=0.1, seeds=(0, 1, 2, 3, 4), kind="equibiaxial",
                     steps=10, tol=1e-8, precision="fp64", c0=2.0),
    "fp32_L1024": dict(L=1024, f=0.2, seeds=(0,), kind="equibiaxial",
                       steps=50, tol=1e-6, precision="fp32", c0=C0_SOFT),
    "fp32_L4096_shear": dict(L=4096, f=0.3, seeds=(0,), kind="shear",
                             steps=40, tol=1e-6, precision="fp32", c0=C0_SOFT),
}


def batch_realizations(n: int = 256, base_seed: int = 1000):
    """Realizations of the uneven batched workload.

    Realization r has seed 1000 + r, L drawn uniformly from {128, 256, 512},
    f uniform in [0.05, 0.4], equibiaxial loading for even r and shear for odd
    r, 20 load steps each.
    """
    out = []
    for r in range(n):
        seed = base_seed + r
        uL = uniform01(seed, np.uint64(0xA11CE))
        uf = uniform01(seed, np.uint64(0xF00D))
        L = (128, 256, 512)[min(int(uL * 3), 2)]
        f = 0.05 + 0.35 * float(uf)
        kind = "equibiaxial" if r % 2 == 0 else "shear"
        out.append(dict(r=r, seed=seed, L=L, f=f, kind=kind, steps=20))
    return out


def serving_trace(n: int = 200, seed: int = 7, rate: float = 1.0):
    """Requests of the serving workload, in arrival order.

    Poisson arrivals at `rate` requests per second (exponential gaps drawn
    from the counter-based uniform), L from {64, 256, 1024, 2048} with
    weights 0.4 / 0.3 / 0.2 / 0.1, f uniform in [0.05, 0.4], equibiaxial or
    shear loading with probability 1/2 each, and 10 to 40 load steps.
    """
    out = []
    t = 0.0
    for i in range(n):
        u = [float(uniform01(seed, np.uint64(8 * i + k))) for k in range(5)]
        t += -np.log1p(-u[0]) / rate
        L = 64 if u[1] < 0.4 else 256 if u[1] < 0.7 else 1024 if u[1] < 0.9 else 2048
        f = 0.05 + 0.35 * u[2]
        kind = "equibiaxial" if u[3] < 0.5 else "shear"
        steps = 10 + min(int(u[4] * 31), 30)
        out.append(dict(i=i, arrival=t, L=L, f=f, kind=kind, steps=steps, seed=seed * 100003 + i))
    return out

