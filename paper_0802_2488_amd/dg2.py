"""DG2 driver: the four sign variants of the discrete Green tensor solved in
one batch and combined load step by load step (Sec. 2, "Discrete Green
functions").

The variants G(q1, q2), G(-q1, -q2), G(-q1, q2), G(q1, -q2) are
green_variant 0..3.  Each runs as a batch slot admitted with the hold flag,
so after every load step it waits with that step's converged fields; when
all four wait, pm_dg2_combine forms the average strain, the stress of the
average, the average stress and the plastic mask, and the slots resume.
Argument marshalling and orchestration only; all arithmetic runs in the
library.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from . import batch as pmb
from ._lib import PM_FP64, PmDg2Out, PmParams, check, lib


@dataclasses.dataclass
class DG2Step:
    eps: torch.Tensor | None            # (4, L, L) average strain
    sigma_of_avg: torch.Tensor | None   # S(average strain), 0 on voids
    sigma_avg: torch.Tensor | None      # average of the four stresses
    plastic: torch.Tensor | None        # (L, L) uint8, plastic mask of the average strain
    eps_mean: np.ndarray
    sigma_of_avg_mean: np.ndarray
    sigma_avg_mean: np.ndarray
    plastic_fraction: float
    records: list                       # the four variants' step records


def combine(params: PmParams, mask: torch.Tensor, eps4, sig4=None, fields=True, stream=None):
    """pm_dg2_combine on four (4, L, L) strain (and stress) fields."""
    L = params.L
    dev = mask.device
    dt = torch.float64 if params.precision == PM_FP64 else torch.float32
    nws = lib().pm_dg2_workspace_bytes(ctypes.byref(params))
    if nws == 0:
        raise _lib.PmError(_lib.PM_EINVAL, "pm_dg2_workspace_bytes")
    ws = torch.empty(nws // 8 + 1, dtype=torch.float64, device=dev)
    out = PmDg2Out()
    res = [None] * 4
    if fields:
        res = [torch.empty((4, L, L), dtype=dt, device=dev) for _ in range(3)] + \
              [torch.empty((L, L), dtype=torch.uint8, device=dev)]
        out.eps, out.sigma_of_avg, out.sigma_avg, out.plastic = (t.data_ptr() for t in res)
    for t in list(eps4) + (list(sig4) if sig4 is not None else []):
        if t.dtype != dt or tuple(t.shape) != (4, L, L) or not t.is_contiguous():
            raise ValueError("fields must be contiguous (4, L, L) tensors of the field precision")
    pe = (ctypes.c_void_p * 4)(*[t.data_ptr() for t in eps4])
    ps = None if sig4 is None else (ctypes.c_void_p * 4)(*[t.data_ptr() for t in sig4])
    st = torch.cuda.current_stream(dev).cuda_stream if stream is None else stream
    check(lib().pm_dg2_combine(ctypes.byref(params), mask.data_ptr(), pe, ps, ws.data_ptr(), ws.numel() * 8,
                               ctypes.byref(out), st), "pm_dg2_combine")
    return DG2Step(res[0], res[1], res[2] if sig4 is not None else None, res[3],
                   np.array(out.eps_mean[:]), np.array(out.sigma_of_avg_mean[:]), np.array(out.sigma_avg_mean[:]),
                   out.plastic_fraction, [])


def solve_path(mask: torch.Tensor, params: PmParams, E_path, tick_iters: int = 16, fields=True):
    """DG2 over a load ramp; returns one DG2Step per load step."""
    E = np.asarray(E_path, dtype=np.float64).reshape(-1, 3)
    n = E.shape[0]
    mask = mask.to(device="cuda", dtype=torch.uint8).contiguous()
    variants = []
    for v in range(4):
        p = PmParams.from_buffer_copy(params)
        p.green_variant = v
        variants.append(p)
    pool = pmb.overhead_bytes(4) + sum(pmb.slot_bytes(p, n) for p in variants)
    b = pmb.Batch(pool, max_slots=4)
    try:
        slots = [b.admit(mask, p, E, hold=True) for p in variants]
        if any(s is None for s in slots):
            raise RuntimeError("the four DG2 slots do not fit in their pool")
        patience = int(params.max_iter) // tick_iters + 3
        out = []
        for step in range(n):
            for _ in range(patience):
                b.tick(tick_iters)
                if all(b.poll(s)["steps_done"] > step for s in slots):
                    break
            else:
                raise RuntimeError(f"DG2 load step {step + 1} did not end within {patience} ticks")
            got = [b.fetch(s) for s in slots]
            r = combine(params, mask, [g[1] for g in got], [g[0] for g in got], fields=fields)
            r.records = [b.records(s, step, 1)[0] for s in slots]
            out.append(r)
            if step + 1 < n:
                for s in slots:
                    b.resume(s)
        for s in slots:
            b.release(s)
        return out
    finally:
        b.close()
