"""Python face of the batch / serving C ABI: many realizations on one GPU.

A ``Batch`` owns one device pool (a torch uint8 tensor; the library carves
slot workspaces out of it and never allocates device memory).  Realizations
are admitted with their own mask, parameters and load ramp; every
``tick(iters)`` runs that many iterations on all running slots, ends the load
steps that finished and starts the next ones on the device.  Argument
marshalling only: every step of the method runs in the library's kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import PM_FP64, PmParams, PmSlotInfo, PmStepOut, PmStepRecord, check, lib


@dataclasses.dataclass
class Record:
    sigma_mean: np.ndarray
    eps_mean: np.ndarray
    res_eq: float
    res_mac: float
    res_cmp: float
    plastic_fraction: float
    iters: int
    status: int          # 1 converged, 2 stopped at max_iter, 3 non-finite


def _stream(device="cuda") -> int:
    return torch.cuda.current_stream(device).cuda_stream


def slot_bytes(params: PmParams, nsteps: int) -> int:
    n = lib().pm_batch_slot_bytes(ctypes.byref(params), int(nsteps))
    if n == 0:
        raise _lib.PmError(_lib.PM_EINVAL, "pm_batch_slot_bytes")
    return n


def overhead_bytes(max_slots: int) -> int:
    return lib().pm_batch_overhead_bytes(int(max_slots))


class Batch:
    def __init__(self, pool_bytes: int, max_slots: int = 256, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("the batch engine needs a HIP device")
        self.device = device
        self.pool = torch.empty(int(pool_bytes) + 256, dtype=torch.uint8, device=device)
        base = self.pool.data_ptr()
        self._ptr = base + (-base) % 256
        self.pool_bytes = int(pool_bytes)
        self.max_slots = max_slots
        h = ctypes.c_void_p()
        check(lib().pm_batch_create(ctypes.byref(h), self._ptr, self.pool_bytes, max_slots, _stream(device)),
              "pm_batch_create")
        self.handle = h
        self._masks = {}        # slot -> mask tensor, alive until release

    def close(self):
        if getattr(self, "handle", None):
            lib().pm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, mask: torch.Tensor, params: PmParams, E_path, hold: bool = False) -> int | None:
        """Slot id, or None when the pool or the slot table is full.  hold:
        wait after every load step until resume() (fields of that step)."""
        m = mask.to(device=self.device, dtype=torch.uint8).contiguous()
        if tuple(m.shape) != (params.L, params.L):
            raise ValueError(f"mask shape {tuple(m.shape)} != ({params.L}, {params.L})")
        E = np.ascontiguousarray(np.asarray(E_path, dtype=np.float64).reshape(-1, 3))
        slot = ctypes.c_int32(-1)
        rc = lib().pm_batch_admit(self.handle, ctypes.byref(params), m.data_ptr(), E.shape[0],
                                  E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _lib.PM_ADMIT_HOLD if hold else 0, ctypes.byref(slot))
        if rc == _lib.PM_EBUSY:
            return None
        check(rc, "pm_batch_admit")
        self._masks[slot.value] = m
        return slot.value

    def tick(self, iters: int) -> int:
        """Run iters iterations on every running slot; returns how many still run."""
        n = ctypes.c_int32(0)
        check(lib().pm_batch_tick(self.handle, int(iters), ctypes.byref(n)), "pm_batch_tick")
        return n.value

    def poll(self, slot: int) -> dict:
        info = PmSlotInfo()
        check(lib().pm_batch_poll(self.handle, slot, ctypes.byref(info)), "pm_batch_poll")
        return {k: getattr(info, k) for k, _ in info._fields_}

    def records(self, slot: int, first: int = 0, count: int | None = None) -> list[Record]:
        if count is None:
            count = self.poll(slot)["steps_done"] - first
        arr = (PmStepRecord * max(count, 1))()
        check(lib().pm_batch_records(self.handle, slot, first, count, arr), "pm_batch_records")
        return [Record(np.array(r.sigma_mean[:]), np.array(r.eps_mean[:]), r.res_eq, r.res_mac, r.res_cmp,
                       r.plastic_fraction, r.iters, r.status) for r in arr[:count]]

    def fetch(self, slot: int, fields=True):
        """Current fields of a slot: (sigma, eps, plastic, PmStepOut)."""
        info = self.poll(slot)
        L = info["L"]
        dt = torch.float64 if info["precision"] == PM_FP64 else torch.float32
        out = PmStepOut()
        sig = eps = pl = None
        if fields:
            sig = torch.empty((4, L, L), dtype=dt, device=self.device)
            eps = torch.empty((4, L, L), dtype=dt, device=self.device)
            pl = torch.empty((L, L), dtype=torch.uint8, device=self.device)
            out.sigma, out.eps, out.plastic = sig.data_ptr(), eps.data_ptr(), pl.data_ptr()
        check(lib().pm_batch_fetch(self.handle, slot, ctypes.byref(out)), "pm_batch_fetch")
        return sig, eps, pl, out

    def set_graphs(self, enable: bool):
        """Replay each tick as a HIP graph once its slot table ran eagerly (default on)."""
        check(lib().pm_batch_set_graphs(self.handle, 1 if enable else 0), "pm_batch_set_graphs")

    def resume(self, slot: int):
        check(lib().pm_batch_resume(self.handle, slot), "pm_batch_resume")

    def release(self, slot: int):
        check(lib().pm_batch_release(self.handle, slot), "pm_batch_release")
        self._masks.pop(slot, None)


def run_all(batch: Batch, jobs, tick_iters: int = 16, on_finish=None):
    """Admit jobs (mask, params, E_path) as room allows and tick until all are
    done.  Returns the records of each job, in job order.  on_finish(i, slot)
    is called before a finished slot is released."""
    pending = list(range(len(jobs)))
    live = {}
    recs = [None] * len(jobs)
    # every load step ends within max_iter iterations, so some slot must make
    # progress within that many ticks; anything else is an engine error
    patience = max(int(j[1].max_iter) for j in jobs) // tick_iters + 3 if jobs else 0
    last, idle = None, 0
    while pending or live:
        while pending:
            i = pending[0]
            s = batch.admit(*jobs[i])
            if s is None:
                if not live:
                    raise RuntimeError(f"job {i} does not fit in an empty pool")
                break
            live[s] = i
            pending.pop(0)
        batch.tick(tick_iters)
        progress = []
        for s in list(live):
            info = batch.poll(s)
            progress.append((s, info["steps_done"]))
            if info["finished"]:
                i = live.pop(s)
                recs[i] = batch.records(s)
                if on_finish is not None:
                    on_finish(i, s)
                batch.release(s)
        idle = idle + 1 if progress == last else 0
        last = progress
        if idle > patience:
            raise RuntimeError(f"no slot advanced within {idle} ticks of {tick_iters} iterations")
    return recs
