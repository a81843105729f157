"""GPU parity at the workload sizes, in the launch configuration the benchmark
times (FP32 fields, FP64 norms, default kernels).

L = 1024 (the curve-and-masks workload) is compared with the FP64 oracle
iteration-locked over its first five load steps, L = 4096 (the benchmark
workload) over 20 iterations of its first step against a stored oracle run
(sampled pixels), in FP32 (<= 1e-4) and in FP64 (<= 1e-10).  At L = 8192, the largest size the
library accepts, the checks are properties that hold at any size: exact
uniform fields in a homogeneous medium, zero stress in voids and the Mises
cap, and FP32 against the library's own FP64 path (which the smaller-size
tests pin to the oracle).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import alm, hencky  # noqa: E402
from paper_0802_2488_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0802_2488_amd import solver as pms  # noqa: E402


def t33(planes):
    return alm.from_voigt4(np.moveaxis(planes.detach().cpu().double().numpy(), 0, -1))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def params(L, precision, max_iter, tol=0.0, c0=2.0):
    return pms.make_params(L, mu=1.0, lam=2.0, Y=1.0, mu0=c0, lam0=2.0 * c0, tol=tol, max_iter=max_iter,
                           precision=precision)


def test_curve_workload_first_five_steps_iteration_locked():
    """L = 1024, f = 0.2, equibiaxial (the curve-and-masks workload, its
    reference medium): FP32 (<= 1e-4, plastic mask outside the band) and FP64
    (<= 1e-10) against one oracle run over the first five load steps."""
    w = synth.WORKLOADS["fp32_L1024"]
    L, iters, c0 = w["L"], 4, w["c0"]
    mask = synth.bernoulli_mask(L, w["f"], 0)
    path = synth.load_path(w["kind"], w["steps"], synth.default_emax(w["kind"], 1.0, 1.0))[:5]
    tm = torch.tensor(mask, device="cuda")
    g32 = pms.Solver(tm, params(L, "fp32", iters, c0=c0))
    g64 = pms.Solver(tm, params(L, "fp64", iters, c0=c0))
    o = alm.Solver(mask, alm.Params(L=L, mu0=c0, lam0=2.0 * c0))
    for E in path:
        ro = o.step(E, fixed_iters=iters)
        rg = g32.step(E)
        assert rg.iters == iters
        assert rel(t33(rg.sigma), ro.sigma) <= 1e-4
        band = np.abs(ro.margin) <= 1e-5
        assert np.array_equal(rg.plastic.cpu().numpy().astype(bool)[~band], ro.plastic[~band])
        np.testing.assert_allclose(rg.sigma_mean, alm.voigt4(ro.sigma_mean), rtol=1e-4, atol=1e-6)
        del rg
        rd = g64.step(E)
        assert rd.iters == iters
        assert rel(t33(rd.sigma), ro.sigma) <= 1e-10
        assert rel(t33(rd.eps), ro.eps) <= 1e-10
        np.testing.assert_array_equal(rd.plastic.cpu().numpy().astype(bool)[~band], ro.plastic[~band])
        del rd, ro
    g32.close()
    g64.close()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_L4096_shear_step1.npz")


@pytest.mark.parametrize("precision,rv,cv", [("fp32", 0, 0), ("fp32", 1, 1), ("fp64", 0, 0)])
def test_benchmark_workload_against_stored_oracle(precision, rv, cv):
    """L = 4096, f = 0.3, shear, first load step, 20 iterations (written by
    tests/golden/make_fullsize_reference.py from the FP64 oracle): the
    stress at the stored sample of pixels (relative L2 <= 1e-4 in FP32,
    <= 1e-10 in FP64), the plastic mask there outside the 1e-5 Y band, and
    the mean stress and strain."""
    ref = np.load(GOLDEN, allow_pickle=False)
    L, iters, c0 = int(ref["L"]), int(ref["iters"]), float(ref["c0"])
    w = synth.WORKLOADS["fp32_L4096_shear"]
    assert (L, float(ref["f"]), c0) == (w["L"], w["f"], w["c0"])
    mask = synth.bernoulli_mask(L, float(ref["f"]), int(ref["seed"]))
    idx = torch.tensor(ref["idx"], device="cuda")
    saved = pms.get_tuning(L, precision)
    pms.set_tuning(L, precision, rv, cv)
    try:
        g = pms.Solver(torch.tensor(mask, device="cuda"), params(L, precision, iters, c0=c0))
        r = g.step(tuple(ref["E"]))
        assert r.iters == iters
        sig = r.sigma.reshape(4, -1)[:, idx].T.double().cpu().numpy()
        pl = r.plastic.reshape(-1)[idx].cpu().numpy().astype(bool)
        g.close()
    finally:
        pms.set_tuning(L, precision, *saved)
    bound = 1e-4 if precision == "fp32" else 1e-10
    w4 = np.array([1.0, 1.0, 1.0, np.sqrt(2.0)])           # Frobenius weights of (11, 22, 33, 12)
    assert np.linalg.norm((sig - ref["sigma"]) * w4) <= bound * np.linalg.norm(ref["sigma"] * w4)
    band = np.abs(ref["margin"]) <= 1e-5
    assert np.array_equal(pl[~band], ref["plastic"][~band])
    np.testing.assert_allclose(r.sigma_mean, ref["sigma_mean"], rtol=bound, atol=bound * 1e-2)
    np.testing.assert_allclose(r.eps_mean, ref["eps_mean"], rtol=bound, atol=bound * 1e-2)
    assert abs(r.res_cmp - float(ref["res_cmp"])) <= (1e-3 if precision == "fp32" else 1e-8) * float(ref["res_cmp"])


def test_max_size_homogeneous_medium_exact():
    L = 8192
    g = pms.Solver(torch.zeros((L, L), dtype=torch.uint8, device="cuda"), params(L, "fp32", 50, tol=1e-6))
    E = (0.7, 0.2, 0.1)
    r = g.step(E)
    assert r.converged and r.iters == 2
    ref = alm.voigt4(hencky.stress(alm.tensor_from_voigt(E), 1.0, 2.0, 1.0))
    s = r.sigma
    for c in range(4):
        assert float((s[c] - ref[c]).abs().max()) <= 1e-6 * np.abs(ref).max()
    g.close()


def test_max_size_porous_fp32_against_fp64_and_invariants():
    L = 8192
    mask = synth.bernoulli_mask(L, 0.3, 1)
    tm = torch.tensor(mask, device="cuda")
    E = (0.0, 0.0, 0.1)
    r32 = pms.Solver(tm, params(L, "fp32", 4)).step(E)
    s32 = r32.sigma.double()
    del r32
    r64 = pms.Solver(tm, params(L, "fp64", 4)).step(E)
    s64 = r64.sigma
    assert float(torch.linalg.vector_norm(s32 - s64) / torch.linalg.vector_norm(s64)) <= 1e-4
    void = tm.bool()
    assert float(s64[:, void].abs().max()) == 0.0
    # Mises norm of the stress deviator never exceeds the yield stress
    tr = (s64[0] + s64[1] + s64[2]) / 3.0
    d2 = (s64[0] - tr) ** 2 + (s64[1] - tr) ** 2 + (s64[2] - tr) ** 2 + 2.0 * s64[3] ** 2
    assert float(torch.sqrt(1.5 * d2).max()) <= 1.0 + 1e-12
    assert not bool(r64.plastic[void].any())
