"""Serving loop over the batch engine, and the one-at-a-time baseline.

Requests (mask parameters, load type, ramp length) arrive over time; each
is admitted into the batch engine in arrival order as soon as the pool has
room, and every tick advances all admitted requests together.  A request's
latency runs from its arrival to the moment its last step record is on the
host, so it includes queueing, mask generation and admission.  The baseline
serves the same trace first come, first served, one request at a time with
a single solver.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import batch as pmb
from . import solver as pms
from . import synth


def request_job(req, tol=1e-6, max_iter=500, precision="fp32", material=None, c0=None):
    """(device mask, params, ramp) of one request; reference medium
    c0 x matrix (default: the soft medium of the workloads)."""
    m = dict(synth.MATERIAL if material is None else material)
    c0 = synth.C0_SOFT if c0 is None else c0
    mask = pms.device_mask(req["L"], req["f"], req["seed"])
    params = pms.make_params(req["L"], mu=m["mu"], lam=m["lam"], Y=m["Y"], mu0=c0 * m["mu"], lam0=c0 * m["lam"],
                             tol=tol, max_iter=max_iter, precision=precision)
    path = synth.load_path(req["kind"], req["steps"], synth.default_emax(req["kind"], m["Y"], m["mu"]))
    return mask, params, path


def _wait_until(t0, t):
    dt = t - (time.perf_counter() - t0)
    if dt > 0:
        time.sleep(dt)


def serve_batched(trace, pool_bytes=16 << 30, max_slots=256, tick_iters=16, tol=1e-6, max_iter=500,
                  ignore_arrivals=False, records=None):
    """Serve the trace through one batch; returns latencies (s), pixel-iterations, wall (s)
    and iterations per request.  records: a dict that receives each request's
    step records (index -> list of batch.Record)."""
    import torch

    b = pmb.Batch(pool_bytes, max_slots=max_slots)
    n = len(trace)
    lat = [None] * n
    iters = [0] * n
    queue = collections.deque()
    live = {}
    nxt = 0
    work = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        while nxt < n or queue or live:
            now = time.perf_counter() - t0
            while nxt < n and (ignore_arrivals or trace[nxt]["arrival"] <= now):
                queue.append(nxt)
                nxt += 1
            while queue:
                i = queue[0]
                s = b.admit(*request_job(trace[i], tol, max_iter))
                if s is None:
                    if not live:
                        raise RuntimeError(f"request {i} does not fit in an empty pool of {pool_bytes} bytes")
                    break
                live[s] = queue.popleft()
            if not live:
                _wait_until(t0, trace[nxt]["arrival"])
                continue
            b.tick(tick_iters)
            for s in list(live):
                if not b.poll(s)["finished"]:
                    continue
                i = live.pop(s)
                recs = b.records(s)
                b.release(s)
                if records is not None:
                    records[i] = recs
                it = sum(r.iters for r in recs)
                iters[i] = it
                work += trace[i]["L"] ** 2 * it
                lat[i] = time.perf_counter() - t0 - (0.0 if ignore_arrivals else trace[i]["arrival"])
        wall = time.perf_counter() - t0
    finally:
        b.close()
    return np.array(lat), work, wall, iters


def serve_fifo(trace, tol=1e-6, max_iter=500, ignore_arrivals=False, records=None):
    """First come, first served, one request at a time on a single solver.
    records: a dict that receives each request's step results."""
    import torch

    n = len(trace)
    lat = [None] * n
    iters = [0] * n
    work = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, req in enumerate(trace):
        if not ignore_arrivals:
            _wait_until(t0, req["arrival"])
        mask, params, path = request_job(req, tol, max_iter)
        s = pms.Solver(mask, params)
        it = 0
        res = []
        for E in path:
            r = s.step(E, fields=False)
            it += r.iters
            res.append(r)
        s.close()
        if records is not None:
            records[i] = res
        iters[i] = it
        work += req["L"] ** 2 * it
        lat[i] = time.perf_counter() - t0 - (0.0 if ignore_arrivals else req["arrival"])
    wall = time.perf_counter() - t0
    return np.array(lat), work, wall, iters


def percentiles(lat):
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(np.mean(lat)), "max_s": float(np.max(lat))}
