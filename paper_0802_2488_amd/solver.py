"""Python face of the C ABI: one realization solved on one GPU.

Thin wrapper: it allocates device memory with torch (the library never
allocates device memory), passes raw pointers and the current HIP stream to
libpm.so, and returns the per-step results.  Every step of the method runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import PM_FP32, PM_FP64, PmParams, PmStepOut, check, lib


@dataclasses.dataclass
class StepResult:
    sigma_mean: np.ndarray     # (11, 22, 33, 12)
    eps_mean: np.ndarray
    res_eq: float
    res_mac: float
    res_cmp: float
    iters: int
    converged: bool
    status: int
    sigma: torch.Tensor | None = None      # (4, L, L) device
    eps: torch.Tensor | None = None
    plastic: torch.Tensor | None = None    # (L, L) uint8 device


def make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=0.0, lam0=0.0, tol=1e-6, eta_eq=None, eta_mac=None,
                eta_cmp=None, max_iter=5000, check_every=0, precision="fp32", green_variant=0) -> PmParams:
    prec = {"fp32": PM_FP32, "fp64": PM_FP64}[precision]
    return PmParams(L, mu, lam, Y, mu0, lam0,
                    tol if eta_eq is None else eta_eq,
                    tol if eta_mac is None else eta_mac,
                    tol if eta_cmp is None else eta_cmp,
                    max_iter, check_every, prec, green_variant)


def device_mask(L: int, f: float, seed: int, device="cuda") -> torch.Tensor:
    """Bernoulli void mask generated on the device by the library."""
    m = torch.empty((L, L), dtype=torch.uint8, device=device)
    check(lib().pm_bernoulli_mask(m.data_ptr(), L, f, seed, 1, _stream(device)), "pm_bernoulli_mask")
    return m


def _stream(device="cuda") -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Solver:
    """One realization: mask (device uint8 L x L, 1 = void) and parameters."""

    def __init__(self, mask: torch.Tensor, params: PmParams, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the solver needs a HIP device")
        self.params = params
        self.L = params.L
        self.dtype = torch.float64 if params.precision == PM_FP64 else torch.float32
        self.mask = mask.to(device=device, dtype=torch.uint8).contiguous()
        if tuple(self.mask.shape) != (self.L, self.L):
            raise ValueError(f"mask shape {tuple(self.mask.shape)} != ({self.L}, {self.L})")
        nbytes = lib().pm_workspace_bytes(ctypes.byref(params))
        if nbytes == 0:
            raise _lib.PmError(_lib.PM_EINVAL, "pm_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = nbytes
        self.device = device
        h = ctypes.c_void_p()
        check(lib().pm_solver_create(ctypes.byref(h), ctypes.byref(params), self.mask.data_ptr(),
                                     self._ws_ptr, nbytes, _stream(device)), "pm_solver_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().pm_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, E, fields=True, raise_on_noconv=False) -> StepResult:
        """One load step at E = (E11, E22, E12)."""
        L = self.L
        out = PmStepOut()
        sig = eps = pl = None
        if fields:
            sig = torch.empty((4, L, L), dtype=self.dtype, device=self.device)
            eps = torch.empty((4, L, L), dtype=self.dtype, device=self.device)
            pl = torch.empty((L, L), dtype=torch.uint8, device=self.device)
            out.sigma, out.eps, out.plastic = sig.data_ptr(), eps.data_ptr(), pl.data_ptr()
        Ec = (ctypes.c_double * 3)(*[float(x) for x in E])
        rc = lib().pm_solver_step(self.handle, Ec, ctypes.byref(out))
        if rc not in (_lib.PM_OK, _lib.PM_ENOCONV, _lib.PM_ENAN) or (rc != _lib.PM_OK and raise_on_noconv):
            check(rc, "pm_solver_step")
        return StepResult(np.array(out.sigma_mean[:]), np.array(out.eps_mean[:]), out.res_eq, out.res_mac,
                          out.res_cmp, out.iters, bool(out.converged), rc, sig, eps, pl)

    def set_max_iter(self, max_iter: int):
        """Iteration limit of the following load steps (the state is kept)."""
        check(lib().pm_solver_set_max_iter(self.handle, int(max_iter)), "pm_solver_set_max_iter")
        self.params.max_iter = int(max_iter)

    def timing(self, enable: bool, every: int = 1):
        """Start (resetting totals) or stop per-kernel event timing of every
        `every`-th iteration; returns the totals."""
        t = _lib.PmKernelTiming()
        check(lib().pm_solver_timing(self.handle, int(every) if enable else 0, ctypes.byref(t)), "pm_solver_timing")
        return {k: getattr(t, k) for k, _ in t._fields_}

    # -- kernel-level hooks -------------------------------------------------
    def buffers(self):
        """Views of the workspace: the stress state (L, L, 4), components
        (11, 22, 33, 12) of a pixel side by side, and the raw half spectrum
        (L*L/2*3*2,) in the tiled layout of pm_spectrum_tile."""
        e = ctypes.c_void_p()
        s = ctypes.c_void_p()
        check(lib().pm_solver_buffers(self.handle, ctypes.byref(e), ctypes.byref(s)), "pm_solver_buffers")
        L = self.L
        es = 8 if self.dtype == torch.float64 else 4
        base = self.workspace.data_ptr()
        eo = (e.value - base) // es
        so = (s.value - base) // es
        flat = self.workspace.view(self.dtype)
        eps_t = flat[eo: eo + 4 * L * L].view(L, L, 4)
        spec_t = flat[so: so + L * (L // 2) * 6]
        return eps_t, spec_t

    def tile(self) -> int:
        return lib().pm_spectrum_tile(self.L, self.params.precision)

    def debug_forward(self, real3: torch.Tensor):
        check(lib().pm_debug_forward(self.handle, real3.contiguous().data_ptr()), "pm_debug_forward")

    def debug_inverse(self, out3: torch.Tensor):
        check(lib().pm_debug_inverse(self.handle, out3.data_ptr()), "pm_debug_inverse")

    def debug_green(self, E):
        Ec = (ctypes.c_double * 3)(*[float(x) for x in E])
        check(lib().pm_debug_green(self.handle, Ec), "pm_debug_green")


def solve_path(mask, params: PmParams, E_path, fields=True):
    s = Solver(mask, params)
    try:
        return [s.step(E, fields=fields) for E in E_path]
    finally:
        s.close()


def autotune(L: int, precision="fp32", iters=20, device="cuda") -> dict:
    """Time the kernel variants for (L, precision) and put the fastest into effect."""
    prec = {"fp32": PM_FP32, "fp64": PM_FP64}[precision]
    n = lib().pm_autotune_workspace_bytes(L, prec)
    if n == 0:
        raise _lib.PmError(_lib.PM_EINVAL, "pm_autotune_workspace_bytes")
    ws = torch.empty(n + 256, dtype=torch.uint8, device=device)
    base = ws.data_ptr()
    out = _lib.PmTuneResult()
    check(lib().pm_autotune(L, prec, iters, base + (-base) % 256, n, _stream(device), ctypes.byref(out)),
          "pm_autotune")
    return {"row_variant": out.row_variant, "col_variant": out.col_variant,
            "ms_per_iteration": [[out.ms_per_iteration[r][c] for c in range(2)] for r in range(2)]}


def set_tuning(L: int, precision="fp32", row_variant=0, col_variant=0):
    prec = {"fp32": PM_FP32, "fp64": PM_FP64}[precision]
    check(lib().pm_set_tuning(L, prec, row_variant, col_variant), "pm_set_tuning")


def get_tuning(L: int, precision="fp32"):
    prec = {"fp32": PM_FP32, "fp64": PM_FP64}[precision]
    r, c = ctypes.c_int32(), ctypes.c_int32()
    check(lib().pm_get_tuning(L, prec, ctypes.byref(r), ctypes.byref(c)), "pm_get_tuning")
    return r.value, c.value

