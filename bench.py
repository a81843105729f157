"""Benchmark: pixel-iterations per second of the discrete-Green augmented-
Lagrangian solve on one MI355X.

Workload: one realization, L = 4096, Bernoulli voids f = 0.3 (seed 0), matrix
mu = 1, lambda = 2, Y = 1, reference medium 0.01 x matrix, simple shear
E = (0, 0, e) ramped over 40 load steps to 4 Y / mu, tolerance 1e-6, FP32
fields with FP64 norms.  A "step" is one load step of that ramp: the device
iterates to convergence (or max_iter) from the previous step's state and
writes sigma, eps and the plastic mask.  Warmup steps are the first load
steps of the ramp; timed steps follow them.

Output: one JSON line with the throughput, the per-kernel roofline of the
dominant kernel (HIP event timing on the solver's stream over the timed
region) beside a measured device copy rate, the FP32 stress error of every
timed step against an FP64 solve of the same iterations, the converged
fraction of every workload, the same throughput in FP64, the batched and
serving workloads, the extension rows, and the CPU oracle timed on a
bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["pm_fft.hpp", "pm_kernels.hpp", "pm_internal.h", "pm_row_f32.hip", "pm_col_f32.hip"]
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_L4096_fp32_shear.md")


def kernel_sources_digest() -> str:
    """SHA-256 over the code of the FP32 row and column kernels' sources:
    comments and blank space are dropped first, so editing a comment does
    not retire counter figures taken from the same code."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_0802_2488_amd", "csrc", name), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                  # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of k_row / k_column from the committed counter
    summary, if it was taken from the kernels as they are now; else None."""
    try:
        with open(COUNTERS_FILE) as fh:
            lines = fh.read().splitlines()
    except OSError:
        return None
    vals = {}
    for ln in lines:
        if ln.startswith("traffic:"):
            for kv in ln.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("sources_sha256") != kernel_sources_digest():
        return None
    return {"k_row": float(vals["k_row_bytes"]), "k_column": float(vals["k_column_bytes"])}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--L", type=int, default=4096)
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain device copy of 256 MiB five times (reference for HBM byte counters)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 256-realization workload")
    ap.add_argument("--no-next", action="store_true", help="skip the DG2 / cluster / method measurements")
    ap.add_argument("--batch-n", type=int, default=256)
    ap.add_argument("--batch-max-iter", type=int, default=500)
    ap.add_argument("--batch-conv-max-iter", type=int, default=20000,
                    help="iteration limit of the batched workload run to the tolerance (FP64)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--serve-n", type=int, default=200, help="requests of the serving trace")
    ap.add_argument("--serve-max-iter", type=int, default=200)
    ap.add_argument("--serve-pool-gb", type=float, default=16.0)
    ap.add_argument("--tick", type=int, default=16, help="iterations per batch tick of the serving loop")
    ap.add_argument("--batch-tick", type=int, default=0,
                    help="iterations per tick of the batched workload (0: the iteration limit, one graph per load step)")
    return ap.parse_args()


def copy_reference():
    """Plain device-to-device copy of known size, for scaling HBM byte counters."""
    import torch

    n = 64 * 1024 * 1024                     # 64 Mi floats = 256 MiB per buffer
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_reference_bytes_read": 4 * n, "copy_reference_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


def algorithmic_bytes(L: int, fs: int):
    """Compulsory HBM bytes per launch of the row and column passes.

    Half spectrum: L rows x (L/2 + 1) momenta x 3 complex values.
    Row pass: read + write the spectrum, read + write the stress state
    (4 components per pixel; it also carries the void flag, so the
    iteration pass does not read the mask).
    Column pass: read + write the spectrum.
    """
    spec = L * (L // 2 + 1) * 3 * 2 * fs
    row = 2 * spec + 2 * 4 * L * L * fs
    col = 2 * spec
    return row, col


def run_gpu(L, precision, steps, warmup, max_iter, timing=True, fp64_check=False):
    """The benchmark workload; with fp64_check an FP64 solver runs the same
    load steps with the FP32 solver's iteration counts (lock-stepped), and the
    relative L2 stress difference of every timed step is recorded (the FP64
    path matches the FP64 oracle to 1e-10, so this is the FP32 stress error
    against the oracle up to that)."""
    import torch

    from paper_0802_2488_amd import synth
    from paper_0802_2488_amd import solver as pms

    w = synth.WORKLOADS["fp32_L4096_shear"]
    kind, nsteps, c0 = w["kind"], w["steps"], w["c0"]
    path = synth.load_path(kind, nsteps, synth.default_emax(kind, 1.0, 1.0))
    assert warmup + steps <= nsteps
    mask = pms.device_mask(L, w["f"], 0)
    params = pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=w["tol"], max_iter=max_iter,
                             precision=precision)
    s = pms.Solver(mask, params)
    ref = None
    warm_iters = []
    for n in range(warmup):
        warm_iters.append(s.step(path[n], fields=False).iters)
    if fp64_check:
        ref = pms.Solver(mask, pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=0.0,
                                               max_iter=1, precision="fp64"))
        for n, it in enumerate(warm_iters):
            _step_locked(ref, path[n], it)
    torch.cuda.synchronize()
    if timing:
        s.timing(True, every=8)   # events on every 8th iteration: their own cost stays small
    t0 = time.perf_counter()
    recs = []
    for n in range(warmup, warmup + steps):
        r = s.step(path[n])
        recs.append(r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = s.timing(False) if timing else None
    s.close()
    errs = []
    if ref is not None:
        # the FP32 fields of every timed step were kept; replay them in FP64
        for n, r in zip(range(warmup, warmup + steps), recs):
            s64 = _step_locked(ref, path[n], r.iters)
            errs.append(float(torch.linalg.vector_norm(r.sigma.double() - s64) / torch.linalg.vector_norm(s64)))
            del s64
        ref.close()
    iters = sum(r.iters for r in recs)
    last_plastic = recs[-1].plastic
    info = dict(
        iters_per_step=[r.iters for r in recs],
        converged=[r.converged for r in recs],
        converged_fraction=sum(r.converged for r in recs) / len(recs),
        res_eq=[r.res_eq for r in recs],
        res_mac=[r.res_mac for r in recs],
        res_cmp=[r.res_cmp for r in recs],
        sigma12_mean=[float(r.sigma_mean[3]) for r in recs],
        plastic_fraction=[float(r.plastic.float().mean()) for r in recs],
    )
    if errs:
        info["stress_rel_l2_vs_fp64"] = errs
    return dict(value=L * L * iters / dt, seconds=dt, iters=iters, info=info, timing=tm, last_plastic=last_plastic)


def _step_locked(solver, E, iters):
    """One load step of exactly `iters` iterations (tolerances 0); returns the stress (device, FP64)."""
    solver.set_max_iter(int(iters))
    return solver.step(E).sigma


def copy_bandwidth():
    """Achievable device copy rate: a 1 GiB device-to-device copy (read and
    write counted), best of 5, HIP events on the current stream."""
    import torch

    n = 256 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = None
    for _ in range(6):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    del src, dst
    return {"what": "device-to-device copy of 1 GiB (torch copy_), best of 6", "GBs": 2 * 4 * n / (best * 1e-3) / 1e9}


def batch_jobs(n, max_iter, precision="fp32"):
    """The uneven batched workload: masks on the device, tol 1e-6."""
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    jobs = []
    for r in synth.batch_realizations(n):
        mask = pms.device_mask(r["L"], r["f"], r["seed"])
        c0 = synth.C0_SOFT
        params = pms.make_params(r["L"], mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=1e-6, max_iter=max_iter,
                                 precision=precision)
        path = synth.load_path(r["kind"], r["steps"], synth.default_emax(r["kind"], 1.0, 1.0))
        jobs.append((mask, params, path))
    return jobs


def synth_realizations(n):
    from paper_0802_2488_amd import synth

    return list(synth.batch_realizations(n))


def run_batch(jobs, tick):
    import torch

    from paper_0802_2488_amd import batch as pmb

    pool = pmb.overhead_bytes(len(jobs)) + sum(pmb.slot_bytes(p, len(path)) for _, p, path in jobs)
    b = pmb.Batch(pool, max_slots=len(jobs))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = pmb.run_all(b, jobs, tick_iters=tick)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    work = sum(j[1].L ** 2 * sum(r.iters for r in rr) for j, rr in zip(jobs, recs))
    return dict(value=work / dt, seconds=dt, pixel_iters=work, pool_bytes=pool,
                converged_steps=sum(r.status == 1 for rr in recs for r in rr),
                steps=sum(len(rr) for rr in recs), recs=recs)


def run_sequential(jobs):
    import torch

    from paper_0802_2488_amd import solver as pms

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0
    for mask, params, path in jobs:
        s = pms.Solver(mask, params)
        for E in path:
            work += params.L ** 2 * s.step(E, fields=False).iters
        s.close()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dict(value=work / dt, seconds=dt, pixel_iters=work)


def autotune_sizes(sizes, precision="fp32"):
    """Autotune the kernel variants of each size (not timed); returns the choices."""
    from paper_0802_2488_amd import solver as pms

    out = {}
    for L in sizes:
        r = pms.autotune(L, precision, iters=10 if L >= 2048 else 30)
        out[str(L)] = r
    return out


def batched_section(a):
    tuning = autotune_sizes((128, 256, 512))
    jobs = batch_jobs(a.batch_n, a.batch_max_iter)
    tick = a.batch_tick or a.batch_max_iter
    full = run_batch(jobs, tick)
    print(f"# batched done: {full['value']:.4e} px-iter/s in {full['seconds']:.1f} s", file=sys.stderr, flush=True)
    # same-work comparison on every realization of the workload, first 2 load steps
    sample = [(m, p, path[:2]) for m, p, path in jobs]
    sb = run_batch(sample, tick)
    sq = run_sequential(sample)
    print(f"# sequential sample done: {sq['value']:.4e} px-iter/s", file=sys.stderr, flush=True)
    # the same realizations run to the tolerance: FP64 (the FP32 primal
    # residual has a floor above 1e-6 at these loads), first 2 load steps
    conv = run_batch([(m, p, path[:2]) for m, p, path in batch_jobs(a.batch_n, a.batch_conv_max_iter, "fp64")], 64)
    real = synth_realizations(a.batch_n)
    by_f = {}
    for lo, hi in ((0.05, 0.15), (0.15, 0.25), (0.25, 0.35), (0.35, 0.4)):
        sel = [rr for r, rr in zip(real, conv["recs"]) if lo <= r["f"] < hi or (hi == 0.4 and r["f"] >= hi)]
        n = sum(len(rr) for rr in sel)
        by_f[f"{lo}-{hi}"] = {"steps": n, "converged_fraction": sum(x.status == 1 for rr in sel for x in rr) / max(n, 1)}
    its = sorted(x.iters for rr in conv["recs"] for x in rr if x.status == 1)
    print(f"# batched to tolerance done: {conv['converged_steps']}/{conv['steps']} steps in {conv['seconds']:.1f} s",
          file=sys.stderr, flush=True)
    return {
        "workload": f"{a.batch_n} realizations (seed 1000 + r, L uniform on {{128, 256, 512}}, f ~ U[0.05, 0.4], "
                    f"even r equibiaxial to 3Y/mu, odd r shear to 4Y/mu, 20 load steps, tol 1e-6, FP32, "
                    f"reference medium 0.01 x matrix, max_iter {a.batch_max_iter}), one batch, "
                    f"{tick} iterations per tick"
                    + (" (one graph per load step)" if tick == a.batch_max_iter else ""),
        "value": full["value"], "unit": "pixel-iters/s", "seconds": full["seconds"],
        "pixel_iters": full["pixel_iters"], "steps": full["steps"], "converged_steps": full["converged_steps"],
        "converged_fraction": full["converged_steps"] / max(full["steps"], 1),
        "pool_bytes": full["pool_bytes"],
        "autotuned": tuning,
        "same_work_sample": {"what": f"all {len(jobs)} realizations, load steps 1-2",
                             "batched": sb["value"], "sequential": sq["value"],
                             "speedup": sb["value"] / sq["value"]},
        "to_tolerance": {"what": f"all {a.batch_n} realizations, load steps 1-2, FP64, tol 1e-6 on all three "
                                 f"indicators, max_iter {a.batch_conv_max_iter}, 64 iterations per tick",
                         "value": conv["value"], "seconds": conv["seconds"], "steps": conv["steps"],
                         "converged_fraction": conv["converged_steps"] / max(conv["steps"], 1),
                         "converged_fraction_by_f": by_f,
                         "iters_of_converged_steps": {"p50": its[len(its) // 2] if its else None,
                                                      "p90": its[(9 * len(its)) // 10] if its else None,
                                                      "max": its[-1] if its else None}},
    }


def serving_section(a):
    from paper_0802_2488_amd import serve, synth

    pool = int(a.serve_pool_gb * (1 << 30))
    base = synth.serving_trace(a.serve_n, 7, 1.0)
    # capacity: the same requests all present at t = 0
    _, w_cap, wall_cap, _ = serve.serve_batched(base, pool_bytes=pool, tick_iters=a.tick,
                                                max_iter=a.serve_max_iter, ignore_arrivals=True)
    cap = a.serve_n / wall_cap
    rate = 0.8 * cap
    print(f"# serving capacity {cap:.2f} req/s; arrivals at {rate:.2f} req/s", file=sys.stderr, flush=True)
    trace = synth.serving_trace(a.serve_n, 7, rate)
    recs = {}
    lat_b, w_b, wall_b, _ = serve.serve_batched(trace, pool_bytes=pool, tick_iters=a.tick, max_iter=a.serve_max_iter,
                                                records=recs)
    nsteps = sum(len(r) for r in recs.values())
    conv_steps = sum(x.status == 1 for r in recs.values() for x in r)
    conv_req = sum(all(x.status == 1 for x in r) for r in recs.values())
    print(f"# serving batched done: p50 {np.percentile(lat_b, 50):.3f} s", file=sys.stderr, flush=True)
    lat_f, w_f, wall_f, _ = serve.serve_fifo(trace, max_iter=a.serve_max_iter)
    print(f"# serving fifo done: p50 {np.percentile(lat_f, 50):.3f} s", file=sys.stderr, flush=True)
    return {
        "workload": f"{a.serve_n} requests (seed 7), Poisson arrivals at 0.8 x measured batched capacity, "
                    f"L in {{64, 256, 1024, 2048}} w.p. 0.4/0.3/0.2/0.1, f ~ U[0.05, 0.4], equibiaxial or shear "
                    f"w.p. 1/2, 10-40 load steps, tol 1e-6, FP32, reference medium 0.01 x matrix, max_iter "
                    f"{a.serve_max_iter}, pool {a.serve_pool_gb:g} GiB, {a.tick} iterations per tick",
        "capacity_req_per_s": cap, "arrival_rate_req_per_s": rate,
        "converged_step_fraction": conv_steps / max(nsteps, 1),
        "converged_request_fraction": conv_req / max(len(recs), 1),
        "latency_note": "latency of each request to its last step record; steps that reach max_iter end there "
                        "(see converged fractions)",
        "batched": dict(serve.percentiles(lat_b), pixel_iters_per_s=w_b / wall_b, wall_s=wall_b),
        "fifo_one_at_a_time": dict(serve.percentiles(lat_f), pixel_iters_per_s=w_f / wall_f, wall_s=wall_f),
    }


def next_rows_section(plastic_4096=None):
    """Measurements of the extension rows: DG2, plastic clusters, DG1 / CG1."""
    import torch

    from paper_0802_2488_amd import clusters, dg2
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    out = {}
    c0 = synth.C0_SOFT
    # DG2 combination kernel bandwidth
    L = 1024
    mask = pms.device_mask(L, 0.2, 0)
    p = pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=1e-6, max_iter=200, precision="fp32")
    eps4 = [torch.randn((4, L, L), device="cuda") for _ in range(4)]
    sig4 = [torch.randn((4, L, L), device="cuda") for _ in range(4)]
    dg2.combine(p, mask, eps4, sig4)
    torch.cuda.synchronize()
    reps = 20
    t1 = time.perf_counter()
    for _ in range(reps):
        dg2.combine(p, mask, eps4, sig4)
    torch.cuda.synchronize()
    tc = (time.perf_counter() - t1) / reps
    del eps4, sig4
    cb = L * L * (4 * 16 + 4 * 16 + 1 + 3 * 16 + 1)
    out["dg2_combine"] = {"L": L, "ms": 1e3 * tc, "GBs": cb / tc / 1e9, "bytes_per_call": cb}
    # plastic clusters of the benchmark's last load step
    if plastic_4096 is not None:
        L = 4096
        vm = pms.device_mask(L, 0.3, 0)
        clusters.analyze(vm, plastic_4096)
        torch.cuda.synchronize()
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            lab, st = clusters.analyze(vm, plastic_4096)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        tm = sorted(times)[len(times) // 2]
        out["clusters"] = {"workload": "L=4096 void mask f=0.3 with the plastic mask of the benchmark's last "
                                       "timed load step", "ms": 1e3 * tm, "pixels_per_s": L * L / tm,
                           "stats": st, "indicators": clusters.indicators(st, L)}
        print(f"# clusters done: {1e3 * tm:.2f} ms", file=sys.stderr, flush=True)
    out["method_iterations"] = method_comparison()
    print("# methods done", file=sys.stderr, flush=True)
    out["fig1_strain_maps"] = fig1_strain_maps()
    print("# fig. 1 maps done", file=sys.stderr, flush=True)
    out["cluster_path_dg2"] = cluster_path()
    # the same curve run to the tolerance: FP64 (the FP32 primal residual
    # has a floor above 1e-6 at small loads), on a grid whose 50 steps all
    # converge within the iteration limit
    out["cluster_path_dg2_converged"] = cluster_path(L=256, max_iter=20000, precision="fp64", tick_iters=64)
    print("# cluster path done", file=sys.stderr, flush=True)
    out["percolation_check"] = percolation_check()
    print("# percolation check done", file=sys.stderr, flush=True)
    return out


def method_comparison(L=128, tol=1e-6, max_iter=20000):
    """Iterations of each Green operator of Sec. 2 to a tolerance, on a
    Bernoulli grid and on the single circular void (equibiaxial load step 1,
    FP64, soft reference medium).  The tensor of eq. 3, each DG2 variant and
    CG1 stop on all three indicators, the equilibrium one taken with the
    method's own divergence (the variant's differences; the continuum
    divergence for CG1).  DG1 is not a projection and has no equilibrium of
    its own, so every method is also timed by the change and constraint
    indicators alone (the common criterion)."""
    from paper_0802_2488_amd import dg2
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    c0 = synth.C0_SOFT
    E1 = synth.load_path("equibiaxial", 10, 3.0)[0]
    import torch
    geoms = {"bernoulli f=0.1 (seed 0)": pms.device_mask(L, 0.1, 0),
             "one circular void f=0.1": torch.tensor(synth.circular_void(L, 0.1), device="cuda")}
    res = {}
    for gname, m in geoms.items():
        its = {}
        for name, v in (("DG eq.3", 0), ("DG1", 4), ("CG1", 5)):
            row = {}
            for crit, eta_eq in (("all three indicators", tol), ("change and constraint", 1e30)):
                if crit == "all three indicators" and v == 4:
                    continue
                q = pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=tol, eta_eq=eta_eq,
                                    max_iter=max_iter, precision="fp64", green_variant=v)
                s = pms.Solver(m, q)
                r = s.step(E1, fields=False)
                s.close()
                row[crit] = {"iters": r.iters, "converged": r.converged, "res_eq": r.res_eq}
            its[name] = row
        q = pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=tol, max_iter=max_iter,
                            precision="fp64")
        st = dg2.solve_path(m, q, [E1], fields=False)[0]
        its["DG2 (all three, own differences)"] = {"iters_per_variant": [r.iters for r in st.records],
                                                   "converged": all(r.status == 1 for r in st.records)}
        res[gname] = its
    return {"workload": f"L={L}, equibiaxial load step 1 of 10 (e = 0.3), reference medium {c0} x matrix, "
                        f"tolerance {tol}, FP64, max_iter {max_iter}", **res}


def fig1_strain_maps(L=256, f=0.1, nsteps=4, e_end=0.5, c0=0.1, max_iter=3000):
    """The comparison of Fig. 1: one centred circular void (f = 0.1), the
    paper's moduli (K = 1, mu = 0.4, Y = 0.5), equibiaxial ramp; the strain
    maps of CG1, CG2 (five-point average of CG1), DG1 and DG2 (average of the
    four variants) measured by the library: checkerboard index, sharpness,
    mean and maximum equivalent strain on the matrix pixels."""
    import torch

    from paper_0802_2488_amd import dg2, maps
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    K, mu, Y = 1.0, 0.4, 0.5
    lam = K - 2.0 * mu / 3.0
    vm = torch.tensor(synth.circular_void(L, f), device="cuda")
    path = synth.load_path("equibiaxial", nsteps, e_end)

    def params(v, eta_eq=1e-6):
        return pms.make_params(L, mu=mu, lam=lam, Y=Y, mu0=c0 * mu, lam0=c0 * lam, tol=1e-6, eta_eq=eta_eq,
                               max_iter=max_iter, precision="fp64", green_variant=v)

    res = {}
    for name, v, eta_eq in (("CG1", 5, 1e-6), ("DG1", 4, 1e30)):
        s = pms.Solver(vm, params(v, eta_eq))
        recs = [s.step(E) for E in path]
        s.close()
        r = recs[-1]
        res[name] = dict(maps.strain_map_metrics(r.eps, vm), iters=[x.iters for x in recs],
                         converged=[x.converged for x in recs])
        if name == "CG1":
            res["CG2"] = dict(maps.strain_map_metrics(maps.five_point_average(r.eps), vm),
                              note="five-point average of the CG1 strain")
    steps = dg2.solve_path(vm, params(0), path)
    res["DG2"] = dict(maps.strain_map_metrics(steps[-1].eps, vm),
                      iters=[[x.iters for x in st.records] for st in steps],
                      converged=[all(x.status == 1 for x in st.records) for st in steps])
    torch.cuda.synchronize()
    return {"workload": f"L={L}, one circular void f={f}, K=1, mu=0.4, Y=0.5, equibiaxial ramp of {nsteps} steps "
                        f"to e={e_end}, FP64, reference medium {c0} x matrix, tolerance 1e-6 (DG1: change and "
                        f"constraint), max_iter {max_iter}; measures of the last step's strain", **res}


def cluster_path(L=1024, f=0.2, nsteps=50, max_iter=1500, precision="fp32", tick_iters=16):
    """Sec. 3 indicators along the curve-and-masks workload solved with DG2
    (the paper's method for Sec. 3): per load step the cluster counts of the
    DG2 plastic mask, eps0 = <(eps11 + eps22) / 2>, sigma0 = <(sigma11 +
    sigma22) / 2> (stress of the average strain), and from them r = dn/d eps0
    and -d2 sigma0 / d eps0^2 (library finite differences)."""
    import torch

    from paper_0802_2488_amd import clusters, dg2
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    c0 = synth.C0_SOFT
    vm = pms.device_mask(L, f, 0)
    path = synth.load_path("equibiaxial", nsteps, synth.default_emax("equibiaxial", 1.0, 1.0))
    p = pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=1e-6, max_iter=max_iter,
                        precision=precision)
    t0 = time.perf_counter()
    steps = dg2.solve_path(vm, p, path, tick_iters=tick_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eps0, sig0, n, vmax, spans, iters, conv = [], [], [], [], [], [], []
    for st in steps:
        _, cs = clusters.analyze(vm, st.plastic)
        ind = clusters.indicators(cs, L)
        eps0.append(0.5 * (st.eps_mean[0] + st.eps_mean[1]))
        sig0.append(0.5 * (st.sigma_of_avg_mean[0] + st.sigma_of_avg_mean[1]))
        n.append(ind["n"])
        vmax.append(ind["v_max"])
        spans.append(bool(cs["spans_x1"] and cs["spans_x2"]))
        iters.append([r.iters for r in st.records])
        conv.append(all(r.status == 1 for r in st.records))
    pi = clusters.path_indicators(np.array(eps0), np.array(n), np.array(sig0))
    k = int(np.argmax(pi["r"]))
    return {"workload": f"DG2, L={L}, f={f} (seed 0), equibiaxial, {nsteps} load steps to 3Y/mu, tol 1e-6, "
                        f"{precision.upper()}, "
                        f"reference medium {c0} x matrix, max_iter {max_iter}; clusters of every step's DG2 plastic "
                        f"mask", "seconds": dt, "iters_per_step_and_variant": iters,
            "converged_step_fraction": sum(conv) / len(conv),
            "eps0": eps0, "sigma0": sig0, "n": n, "v_max": vmax,
            "r": pi["r"].tolist(), "minus_d2sigma0": pi["minus_d2sigma0"].tolist(),
            "eps0_at_max_r": eps0[k],
            "eps0_first_spanning": next((e for e, sp in zip(eps0, spans) if sp), None)}


def percolation_check(L=1024, f=0.1, nsteps=30, e_end=1.5, max_iter=20000, precision="fp64", tick_iters=64):
    """The one number Sec. 3 gives for the clusters (Fig. 3): with the paper's
    moduli (K = 1, mu = 0.4, Y = 0.5; lambda = K - 2 mu / 3) and f = 0.1, the
    largest void-plastic cluster of the DG2 solution percolates near an
    equibiaxial eps0 of 0.9.  Reports the first eps0 of the ramp at which
    the largest cluster spans both axes."""
    import torch

    from paper_0802_2488_amd import clusters, dg2
    from paper_0802_2488_amd import solver as pms
    from paper_0802_2488_amd import synth

    K, mu, Y = 1.0, 0.4, 0.5
    lam = K - 2.0 * mu / 3.0
    c0 = synth.C0_SOFT
    vm = pms.device_mask(L, f, 3)
    path = synth.load_path("equibiaxial", nsteps, e_end)
    p = pms.make_params(L, mu=mu, lam=lam, Y=Y, mu0=c0 * mu, lam0=c0 * lam, tol=1e-6, max_iter=max_iter,
                        precision=precision)
    t0 = time.perf_counter()
    steps = dg2.solve_path(vm, p, path, tick_iters=tick_iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eps0, vmax, spans, conv, iters = [], [], [], [], []
    for st in steps:
        _, cs = clusters.analyze(vm, st.plastic)
        eps0.append(0.5 * (st.eps_mean[0] + st.eps_mean[1]))
        vmax.append(clusters.indicators(cs, L)["v_max"])
        spans.append(bool(cs["spans_x1"] and cs["spans_x2"]))
        conv.append(all(r.status == 1 for r in st.records))
        iters.append(max(r.iters for r in st.records))
    return {"workload": f"DG2, L={L}, f={f} (seed 3), K=1, mu=0.4, Y=0.5, equibiaxial ramp of {nsteps} steps to "
                        f"eps0={e_end}, tol 1e-6, {precision.upper()}, reference medium {c0} x matrix, "
                        f"max_iter {max_iter}",
            "paper_eps0_at_percolation": 0.9, "seconds": dt,
            "eps0_first_spanning": next((e for e, sp in zip(eps0, spans) if sp), None),
            "eps0": eps0, "v_max": vmax, "max_iters_per_step": iters,
            "converged_step_fraction": sum(conv) / len(conv)}


def cpu_baseline(L):
    """The FP64 oracle on this host: one iteration of the first load step."""
    import numpy as np

    from oracle import alm
    from paper_0802_2488_amd import synth

    host_cores = len(os.sched_getaffinity(0))
    mask = synth.bernoulli_mask(L, 0.3, 0)
    E = synth.load_path("shear", 40, 4.0)[0]
    s = alm.Solver(mask, alm.Params(L=L))
    s.start(E)
    n = 3
    t0 = time.perf_counter()
    for _ in range(n):
        s.iterate(E)
    dt = time.perf_counter() - t0
    del s
    return dict(value=L * L * n / dt, unit="pixel-iters/s", cores=alm.fft_workers(L), host_cores=host_cores,
                kind="oracle",
                sample=f"{n} augmented-Lagrangian iterations of load step 1 at L={L} (FP64; scipy.fft on "
                       f"{alm.fft_workers(L)} threads, pointwise numpy single-threaded; Green tensor setup "
                       f"excluded), {dt:.1f} s")


def main():
    a = parse()
    if a.copy_ref:
        copy_reference()
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 "
                                   "(independent solves shard by placing whole realizations on different GPUs, "
                                   "one process each)"}))
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "bench needs a GPU"
    L = a.L
    tuned = {"fp32": autotune_sizes((L,), "fp32")[str(L)]}
    if not a.no_fp64:
        tuned["fp64"] = autotune_sizes((L,), "fp64")[str(L)]
    copy = copy_bandwidth()
    r32 = run_gpu(L, "fp32", a.steps, a.warmup, a.max_iter, fp64_check=not a.no_fp64)
    print(f"# fp32 done: {r32['value']:.4e} px-iter/s over {r32['iters']} iterations", file=sys.stderr, flush=True)
    row_b, col_b = algorithmic_bytes(L, 4)
    tm = r32["timing"]
    row_avg_ms = tm["row_ms"] / max(tm["row_launches"], 1)
    col_avg_ms = tm["col_ms"] / max(tm["col_launches"], 1)
    row_gbs = row_b / (row_avg_ms * 1e-3) / 1e9
    col_gbs = col_b / (col_avg_ms * 1e-3) / 1e9
    r64 = None
    if not a.no_fp64:
        r64 = run_gpu(L, "fp64", min(a.steps, 2), 1, min(a.max_iter, 200))
        print(f"# fp64 done: {r64['value']:.4e} px-iter/s", file=sys.stderr, flush=True)
    nxt = None if a.no_next else next_rows_section(r32.get("last_plastic"))
    r32.pop("last_plastic", None)
    batched = None if a.no_batch else batched_section(a)
    serving = None if a.no_serve else serving_section(a)
    cpu = None if a.no_cpu else cpu_baseline(L)
    ms_per_step = 1e3 * r32["seconds"] / a.steps
    traffic = measured_traffic() if L == 4096 else None
    out = {
        "metric": "pixel-iters/s at L=4096 FP32 vs FP64; batched p50/p99 solve latency",
        "value": r32["value"],
        "unit": "pixel-iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Bernoulli void mask)",
        "config": {"workload": f"single realization L={L}, f=0.3, simple shear to 4Y/mu over 40 load steps, "
                               f"tol 1e-6, FP32 fields + FP64 norms, reference medium 0.01 x matrix; step = one "
                               f"load step (max_iter {a.max_iter})",
                   "L": L, "f": 0.3, "seed": 0, "load_steps_timed": list(range(a.warmup + 1, a.warmup + a.steps + 1)),
                   "reductions": "f64 partial sums and norms", "parallelism": "1 GPU",
                   "autotuned_variants": tuned},
        "roofline": {"bound": "hbm", "kernel": "k_row (inverse row FFT + pointwise step + forward row FFT)",
                     "achieved": row_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": row_gbs / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["k_row"],
                     "algorithmic_bytes_per_launch": row_b, "avg_launch_ms": row_avg_ms,
                     "measured_copy_GBs": copy["GBs"], "frac_of_copy": row_gbs / copy["GBs"]},
        # whole solve against the byte floor of the two-pass design (row pass
        # + column pass bytes per pixel-iteration), at the peak and at the copy rate
        "method_floor": {"bytes_per_px_iter": (row_b + col_b) / (L * L),
                         "ceiling_px_iter_s": HBM_PEAK_GBS * 1e9 * L * L / (row_b + col_b),
                         "frac_of_ceiling": r32["value"] * (row_b + col_b) / (L * L) / (HBM_PEAK_GBS * 1e9),
                         "ceiling_at_copy_px_iter_s": copy["GBs"] * 1e9 * L * L / (row_b + col_b),
                         "frac_of_ceiling_at_copy": r32["value"] * (row_b + col_b) / (L * L) / (copy["GBs"] * 1e9)},
        "kernels": {
            "k_column": {"achieved_GBs": col_gbs, "frac": col_gbs / HBM_PEAK_GBS,
                         "frac_of_copy": col_gbs / copy["GBs"], "avg_launch_ms": col_avg_ms,
                         "algorithmic_bytes_per_launch": col_b,
                         "traffic": None if traffic is None else traffic["k_column"]},
            "reductions_ms_per_iter": tm["other_ms"] / max(tm["iterations"], 1),
        },
        "iterations": r32["info"],
        "fp64": None if r64 is None else {"value": r64["value"], "unit": "pixel-iters/s",
                                          "iters_per_step": r64["info"]["iters_per_step"]},
        "copy_bandwidth": copy,
        "next_rows": nxt,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
