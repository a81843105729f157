"""MI355X-native discrete-Green FFT solver for 2D elastic-perfectly plastic,
pixelwise disordered porous media (Willot & Pellegrini, arXiv:0802.2488).

The computation lives in libpm.so (HIP kernels for gfx950 behind the C ABI of
include/pm.h).  ``solver`` wraps it for Python; ``synth`` draws seeded
synthetic inputs.  Importing the package loads nothing from the GPU.
"""
__all__ = ["synth", "solver", "build"]
