"""Measures of a strain map for the comparison of the methods (Sec. 2,
Fig. 1: the checkerboard pattern of CG1 that CG2 does not remove, the
blurring of DG1, DG2 free of both).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fig. 1 displays the equivalent strain eps_eq = [(2/3) e':e']^(1/2) with the
three-dimensional deviator e' = eps - I tr(eps) / 3.  The paper compares the
maps by eye; the numbers here are readings of "checkerboard" and "blur" on
the matrix pixels (voids are physically irrelevant, Sec. 2):

  checkerboard: root mean square of the mixed second difference
      eps_eq(x) - eps_eq(x + e1) - eps_eq(x + e2) + eps_eq(x + e1 + e2)
  over the 2 x 2 blocks of matrix pixels, divided by the mean of eps_eq;
  sharpness: root mean square of the differences between nearest matrix
      neighbours (both directions), divided by the same mean.

The lattice is periodic.  Written with numpy rolls over whole arrays.
"""
from __future__ import annotations

import numpy as np

from . import hencky


def strain_map_metrics(eps, void):
    """eps: (L, L, 3, 3) strain, void: (L, L) bool.  Returns a dict with
    mean_eq, max_eq, checkerboard, sharpness, matrix_pixels."""
    m = ~np.asarray(void).astype(bool)
    q = hencky.eps_eq(np.asarray(eps, dtype=float))

    def sh(a, d1, d2):            # value at x + d1 e1 + d2 e2
        return np.roll(np.roll(a, -d1, axis=1), -d2, axis=0)

    mean = float(q[m].mean()) if m.any() else 0.0
    mx = float(q[m].max()) if m.any() else 0.0
    blocks = m & sh(m, 1, 0) & sh(m, 0, 1) & sh(m, 1, 1)
    d = q - sh(q, 1, 0) - sh(q, 0, 1) + sh(q, 1, 1)
    p1 = m & sh(m, 1, 0)
    p2 = m & sh(m, 0, 1)
    g1 = sh(q, 1, 0) - q
    g2 = sh(q, 0, 1) - q
    ref = mean if mean > 0 else 1.0
    cb = float(np.sqrt(np.mean(d[blocks] ** 2))) / ref if blocks.any() else 0.0
    npairs = int(p1.sum() + p2.sum())
    sharp = float(np.sqrt((np.sum(g1[p1] ** 2) + np.sum(g2[p2] ** 2)) / npairs)) / ref if npairs else 0.0
    return dict(mean_eq=mean, max_eq=mx, checkerboard=cb, sharpness=sharp, matrix_pixels=int(m.sum()))
