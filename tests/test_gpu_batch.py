"""GPU: the batch / serving engine through the C ABI.

A slot of a batch runs the same kernels and fixed-order reductions as a
single solver, so its step records and fields must be bitwise identical to a
pm_solver driven through the same ramp, whatever else shares the batch; an
FP64 slot is also checked against the oracle, iteration-locked.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import alm  # noqa: E402
from paper_0802_2488_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0802_2488_amd import batch as pmb  # noqa: E402
from paper_0802_2488_amd import solver as pms  # noqa: E402
from paper_0802_2488_amd._lib import PmError  # noqa: E402


def params(L, precision, tol=1e-6, max_iter=400, c0=2.0):
    return pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=tol, max_iter=max_iter,
                           precision=precision)


def mixed_jobs():
    """Different grid sizes, precisions, load types, void fractions, ramp lengths."""
    spec = [(16, "fp64", "equibiaxial", 0.1, 3), (32, "fp32", "shear", 0.3, 4), (64, "fp32", "equibiaxial", 0.2, 3),
            (32, "fp64", "shear", 0.05, 2), (16, "fp32", "shear", 0.4, 5), (64, "fp64", "equibiaxial", 0.25, 2),
            (128, "fp32", "shear", 0.15, 2), (16, "fp32", "shear", 0.0, 3), (8, "fp64", "equibiaxial", 0.05, 2)]
    jobs = []
    for k, (L, prec, kind, f, n) in enumerate(spec):
        mask = torch.tensor(synth.bernoulli_mask(L, f, 100 + k), device="cuda")
        path = synth.load_path(kind, 10, synth.default_emax(kind, 1.0, 1.0))[:n]
        # a cap low enough that stopped steps occur next to converged ones
        # (the homogeneous grid converges in two iterations, the small one
        # well within the cap)
        max_iter = 3000 if L == 8 else 300
        jobs.append((mask, params(L, prec, tol=1e-6 if prec == "fp32" else 1e-9, max_iter=max_iter), path))
    return jobs


def single(job):
    mask, p, path = job
    s = pms.Solver(mask, p)
    out = [s.step(E) for E in path]
    s.close()
    return out


def assert_record_equals(rec, r):
    assert rec.iters == r.iters
    assert rec.status == {0: 1, -4: 2, -5: 3}[r.status]
    assert np.array_equal(rec.sigma_mean, r.sigma_mean)
    assert np.array_equal(rec.eps_mean, r.eps_mean)
    assert rec.res_mac == r.res_mac or (np.isinf(rec.res_mac) and np.isinf(r.res_mac))
    assert rec.res_cmp == r.res_cmp
    assert rec.res_eq == r.res_eq


def tick_until_done(b, iters, max_ticks):
    for _ in range(max_ticks):
        if b.tick(iters) == 0:
            return
    raise AssertionError(f"slots still running after {max_ticks} ticks")


def pool_for(jobs, max_slots):
    need = pmb.overhead_bytes(max_slots)
    for _, p, path in jobs:
        need += pmb.slot_bytes(p, len(path))
    return need


@pytest.mark.parametrize("tick_iters", [1, 7, 64])
def test_batch_bitwise_equals_single_solver(tick_iters):
    jobs = mixed_jobs()
    b = pmb.Batch(pool_for(jobs, 16), max_slots=16)
    finals = {}

    def grab(i, s):
        sig, eps, pl, out = b.fetch(s)
        finals[i] = (sig.clone(), eps.clone(), pl.clone())

    recs = pmb.run_all(b, jobs, tick_iters=tick_iters, on_finish=grab)
    b.close()
    saw = set()
    for i, job in enumerate(jobs):
        ref = single(job)
        assert len(recs[i]) == len(ref)
        for rec, r in zip(recs[i], ref):
            assert_record_equals(rec, r)
            saw.add(rec.status)
        sig, eps, pl = finals[i]
        assert torch.equal(sig, ref[-1].sigma)
        assert torch.equal(eps, ref[-1].eps)
        assert torch.equal(pl, ref[-1].plastic)
    assert saw == {1, 2}


def test_streamed_state_batch_equals_cached_single_solves():
    """Three L = 2048 FP32 realizations in one batch hold 192 MiB of stress
    state, above the 128 MiB from which the iteration streams the state with
    the non-temporal hint; each alone holds 64 MiB and keeps the default
    cache policy.  The hint changes no arithmetic: records and final fields
    are bitwise equal."""
    L = 2048
    jobs = []
    for k in range(3):
        mask = torch.tensor(synth.bernoulli_mask(L, 0.2, 40 + k), device="cuda")
        path = synth.load_path("shear" if k % 2 else "equibiaxial", 10, 3.0)[:2]
        jobs.append((mask, params(L, "fp32", tol=0.0, max_iter=12, c0=0.01), path))
    b = pmb.Batch(pool_for(jobs, 4), max_slots=4)
    finals = {}

    def grab(i, s):
        sig, eps, pl, out = b.fetch(s)
        finals[i] = (sig.clone(), eps.clone(), pl.clone())

    recs = pmb.run_all(b, jobs, tick_iters=5, on_finish=grab)
    b.close()
    for i, job in enumerate(jobs):
        ref = single(job)
        for rec, r in zip(recs[i], ref):
            assert rec.iters == 12
            assert_record_equals(rec, r)
        sig, eps, pl = finals[i]
        assert torch.equal(sig, ref[-1].sigma)
        assert torch.equal(eps, ref[-1].eps)
        assert torch.equal(pl, ref[-1].plastic)


def test_graph_replays_match_eager_ticks():
    """Ticks replayed from a captured graph give the same records as eager
    ticks; admissions and releases between replays force recaptures."""
    jobs = mixed_jobs()
    out = []
    for graphs in (False, True):
        b = pmb.Batch(pool_for(jobs, 3), max_slots=3)      # fewer slots than jobs: slots turn over
        b.set_graphs(graphs)
        out.append(pmb.run_all(b, jobs, tick_iters=5))
        b.close()
    for ra, rb in zip(*out):
        assert len(ra) == len(rb)
        for x, y in zip(ra, rb):
            assert x.iters == y.iters and x.status == y.status
            assert np.array_equal(x.sigma_mean, y.sigma_mean) and np.array_equal(x.eps_mean, y.eps_mean)


def test_batch_fp64_slot_matches_oracle_iteration_locked():
    L, iters = 32, 9
    mask = synth.bernoulli_mask(L, 0.2, 7)
    path = [(0.3, 0.3, 0.0), (0.5, 0.45, 0.05), (0.2, 0.6, 0.1)]
    p = params(L, "fp64", tol=0.0, max_iter=iters)
    other = (torch.tensor(synth.bernoulli_mask(64, 0.3, 8), device="cuda"), params(64, "fp64", tol=0.0, max_iter=5),
             [(0.0, 0.0, 0.2)] * 4)
    jobs = [other, (torch.tensor(mask, device="cuda"), p, path)]
    b = pmb.Batch(pool_for(jobs, 4), max_slots=4)
    finals = {}
    recs = pmb.run_all(b, jobs, tick_iters=4, on_finish=lambda i, s: finals.__setitem__(i, b.fetch(s)))
    b.close()
    o = alm.Solver(mask, alm.Params(L=L, mu=1.0, lam=2.0, Y=1.0, mu0=2.0, lam0=4.0))
    for E, rec in zip(path, recs[1]):
        ro = o.step(E, fixed_iters=iters)
        assert rec.iters == iters and rec.status == 2
        np.testing.assert_allclose(rec.sigma_mean, alm.voigt4(ro.sigma_mean), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(rec.eps_mean, alm.voigt4(ro.eps_mean), rtol=1e-10, atol=1e-12)
        assert abs(rec.res_eq - ro.res_eq) <= 1e-8 * ro.res_eq
    sig = alm.from_voigt4(np.moveaxis(finals[1][0].cpu().double().numpy(), 0, -1))
    assert np.linalg.norm(sig - ro.sigma) <= 1e-10 * np.linalg.norm(ro.sigma)


def test_admission_busy_release_and_reuse():
    L = 32
    p = params(L, "fp32", tol=0.0, max_iter=6)
    path = [(0.0, 0.0, 0.1), (0.0, 0.0, 0.2)]
    mask = torch.tensor(synth.bernoulli_mask(L, 0.2, 3), device="cuda")
    one = pmb.slot_bytes(p, len(path))
    b = pmb.Batch(pmb.overhead_bytes(2) + one + one // 2, max_slots=2)
    s0 = b.admit(mask, p, path)
    assert s0 is not None
    assert b.admit(mask, p, path) is None             # pool full
    tick_until_done(b, 4, 10)
    info = b.poll(s0)
    assert info["finished"] == 1 and info["steps_done"] == 2
    first = b.records(s0)
    b.release(s0)
    s1 = b.admit(mask, p, path)                        # the range and id are free again
    assert s1 == s0
    tick_until_done(b, 5, 10)
    again = b.records(s1)
    for a, c in zip(first, again):
        assert np.array_equal(a.sigma_mean, c.sigma_mean) and a.iters == c.iters
    b.release(s1)
    # slot table full
    b2 = pmb.Batch(pmb.overhead_bytes(1) + 4 * one, max_slots=1)
    assert b2.admit(mask, p, path) is not None
    assert b2.admit(mask, p, path) is None
    b2.close()
    b.close()


def test_release_of_a_running_slot_leaves_others_unchanged():
    jobs = mixed_jobs()[:3]
    ref = [single(j) for j in jobs]
    b = pmb.Batch(pool_for(jobs, 4) + pmb.slot_bytes(jobs[0][1], 3), max_slots=4)
    slots = [b.admit(*j) for j in jobs]
    b.tick(3)
    b.release(slots[1])                                # stopped mid-ramp
    tick_until_done(b, 16, 200)
    for k in (0, 2):
        recs = b.records(slots[k])
        for rec, r in zip(recs, ref[k]):
            assert_record_equals(rec, r)
    b.close()


def test_batch_invalid_arguments():
    L = 16
    p = params(L, "fp32")
    mask = torch.zeros((L, L), dtype=torch.uint8, device="cuda")
    b = pmb.Batch(pmb.overhead_bytes(2) + 2 * pmb.slot_bytes(p, 4), max_slots=2)
    with pytest.raises(PmError):
        b.admit(mask, p, np.zeros((2, 3)))              # zero load step
    with pytest.raises(PmError):
        b.admit(mask, p, np.full((1, 3), np.nan))
    with pytest.raises(PmError):
        b.admit(mask, p, np.zeros((0, 3)))
    with pytest.raises(PmError):
        b.poll(1)
    with pytest.raises(PmError):
        b.release(-1)
    s = b.admit(mask, p, [(0.1, 0.1, 0.0)])
    with pytest.raises(PmError):
        b.records(s, 0, 1)                             # nothing finished yet
    with pytest.raises(PmError):
        b.tick(0)
    for v in (4, 5):                                   # DG1 / CG1 run in the single solver
        q = params(L, "fp32")
        q.green_variant = v
        with pytest.raises(PmError):
            b.admit(mask, q, [(0.1, 0.1, 0.0)])
    b.close()
    with pytest.raises(PmError):
        pmb.Batch(1024, max_slots=4)                   # smaller than the fixed part
