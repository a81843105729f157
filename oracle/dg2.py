"""DG2: the average of four discrete-Green solves (Sec. 2, "Discrete Green
functions", the second work-around for the missing major symmetry of eq. 3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same system is solved to convergence four times, with the Green tensor
of eq. 3 taken at (q1, q2), (-q1, -q2), (-q1, q2) and (q1, -q2) in turn, and
the four converged strain fields are averaged.  Variant numbering follows
alm.Params.green_variant: 0, 1, 2, 3 in that order.

The paper states the strain average; which stress goes with it is not
stated (reading C14): both the stress of the averaged strain, S(eps_bar)
(zero on voids), and the average of the four stresses are reported.  The
plastic mask of DG2 is that of eps_bar: matrix pixels whose trial Mises
stress 3 mu eps_eq(eps_bar) exceeds Y.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import alm, hencky


@dataclasses.dataclass
class DG2Step:
    eps: np.ndarray            # (L, L, 3, 3) average of the four strains
    sigma_of_avg: np.ndarray   # S(eps), 0 on voids
    sigma_avg: np.ndarray      # average of the four stresses
    plastic: np.ndarray        # bool (L, L), plastic mask of eps
    margin: np.ndarray         # 3 mu eps_eq(eps) - Y, -inf on voids
    variants: list             # the four alm.StepResult


def combine(void, eps4, sig4, mu, lam, Y):
    """Average four strain (and stress) fields, (4, L, L, 3, 3) each."""
    void = np.asarray(void).astype(bool)
    eps = np.mean(eps4, axis=0)
    sig_avg = np.mean(sig4, axis=0)
    sig_of_avg = hencky.field_stress(eps, void, mu, lam, Y)
    margin = np.where(void, -np.inf, 3.0 * mu * hencky.eps_eq(eps) - Y)
    return eps, sig_of_avg, sig_avg, margin > 0.0, margin


def solve_path(mask, p: alm.Params, E_path, fixed_iters=None):
    """DG2 over a load ramp: four variant solvers stepped together.

    fixed_iters: optional (4, nsteps) iteration counts (iteration-locked
    comparison), one row per variant.
    """
    solvers = [alm.Solver(mask, dataclasses.replace(p, green_variant=v)) for v in range(4)]
    out = []
    for n, E in enumerate(np.asarray(E_path, dtype=float)):
        res = []
        for v, s in enumerate(solvers):
            fi = None if fixed_iters is None else int(fixed_iters[v][n])
            res.append(s.step(E, fixed_iters=fi))
        eps, soa, sav, pl, mg = combine(mask, np.stack([r.eps for r in res]), np.stack([r.sigma for r in res]),
                                        p.mu, p.lam, p.Y)
        out.append(DG2Step(eps, soa, sav, pl, mg, res))
    return out
