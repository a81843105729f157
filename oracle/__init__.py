"""CPU oracle for the discrete-Green augmented-Lagrangian FFT solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 statement of
what the GPU library computes.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library and imports nothing from it.

Modules
    dg      discrete Fourier momenta, acoustic tensor and discrete Green tensor
            (Sec. 2, eqs. 1-3), plus the symmetrised and continuum variants.
    hencky  elastic-perfectly plastic Mises law in deformation theory and the
            pointwise step of the augmented Lagrangian (Sec. 2 and 3).
    alm     the augmented-Lagrangian / Uzawa iteration, its convergence
            indicators (Sec. 2, "Convergence issues") and the load ramp.
    brute   FFT-free brute-force solvers for tiny grids (L <= 8).
    dg2     the DG2 average of the four sign variants of the Green tensor
            (Sec. 2, "Discrete Green functions").
    clusters  void / plastic clusters and the Sec. 3 indicators.
    maps    measures of a strain map for the comparison of the methods
            (Fig. 1: checkerboard index and sharpness of eps_eq).

Every function states the passage it follows.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""
