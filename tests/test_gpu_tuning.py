"""GPU: the autotuner and the kernel variants it chooses between.

Every variant pair of the iteration kernels must satisfy the same parity
bar against the oracle; the autotuner must time all four pairs and put a
valid one into effect; and batched solves stay bitwise equal to single
solves under a non-default tuning.
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


def t33(planes):
    return alm.from_voigt4(np.moveaxis(planes.detach().cpu().double().numpy(), 0, -1))


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(autouse=True)
def restore_tuning():
    saved = {(L, p): pms.get_tuning(L, p) for L in (64, 128, 256, 512, 2048, 4096) for p in ("fp32", "fp64")}
    yield
    for (L, p), (r, c) in saved.items():
        pms.set_tuning(L, p, r, c)


def run_gpu(L, precision, iters, rv, cv):
    pms.set_tuning(L, precision, rv, cv)
    assert pms.get_tuning(L, precision) == (rv, cv)
    mask = synth.bernoulli_mask(L, 0.25, 3)
    g = pms.Solver(torch.tensor(mask, device="cuda"),
                   pms.make_params(L, tol=0.0, max_iter=iters, precision=precision)).step((0.2, 0.1, 0.15))
    assert g.iters == iters
    return mask, g


@pytest.mark.parametrize("rv,cv", [(0, 0), (1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("L,precision,tol", [(64, "fp64", 1e-10), (2048, "fp64", 1e-10), (256, "fp32", 1e-4)])
def test_every_variant_pair_meets_parity(L, precision, tol, rv, cv):
    iters = 2 if L >= 2048 else 12
    mask, g = run_gpu(L, precision, iters, rv, cv)
    o = alm.Solver(mask, alm.Params(L=L)).step((0.2, 0.1, 0.15), fixed_iters=iters)
    assert rel(t33(g.sigma), o.sigma) <= tol
    np.testing.assert_allclose(g.sigma_mean, alm.voigt4(o.sigma_mean), rtol=tol, atol=tol * 1e-2)


@pytest.mark.parametrize("rv,cv", [(1, 0), (0, 1), (1, 1)])
def test_variant_pairs_at_the_benchmark_size(rv, cv):
    """L = 4096 FP32: every pair against the default pair, which the
    full-size tests compare with the oracle."""
    _, ref = run_gpu(4096, "fp32", 3, 0, 0)
    _, g = run_gpu(4096, "fp32", 3, rv, cv)
    d = float(torch.linalg.vector_norm(g.sigma.double() - ref.sigma.double())
              / torch.linalg.vector_norm(ref.sigma.double()))
    assert d <= 1e-5


def test_autotune_times_all_pairs_and_sets_one():
    res = pms.autotune(512, "fp32", iters=5)
    ms = np.array(res["ms_per_iteration"])
    assert ms.shape == (2, 2) and np.all(ms > 0)
    r, c = res["row_variant"], res["col_variant"]
    assert ms[r, c] == ms.min()
    assert pms.get_tuning(512, "fp32") == (r, c)
    with pytest.raises(PmError):
        pms.set_tuning(512, "fp32", 2, 0)
    with pytest.raises(PmError):
        pms.autotune(48, "fp32")


def test_batch_equals_single_under_a_non_default_tuning():
    L = 128
    pms.set_tuning(L, "fp32", 1, 1)
    mask = torch.tensor(synth.bernoulli_mask(L, 0.2, 9), device="cuda")
    p = pms.make_params(L, tol=1e-6, max_iter=150, precision="fp32")
    path = synth.load_path("shear", 10, 4.0)[:3]
    s = pms.Solver(mask, p)
    ref = [s.step(E) for E in path]
    s.close()
    b = pmb.Batch(pmb.overhead_bytes(1) + pmb.slot_bytes(p, 3), max_slots=1)
    recs = pmb.run_all(b, [(mask, p, path)], tick_iters=16)[0]
    b.close()
    for rec, r in zip(recs, ref):
        assert rec.iters == r.iters and np.array_equal(rec.sigma_mean, r.sigma_mean)
