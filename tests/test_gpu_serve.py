"""GPU: the arrival-driven serving loop (continuous batching over the batch
engine) gives every request the same step records as when it is served
alone on a single solver, bit for bit: the same iteration counts, status and
FP64 means, whatever else shares the device while it runs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_0802_2488_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_0802_2488_amd import serve  # noqa: E402


def small_trace(n=14, rate=40.0):
    """The serving trace's draws with small grids and short ramps, so the
    whole trace runs in seconds; arrivals overlap at this rate."""
    tr = synth.serving_trace(n, 11, rate)
    for r in tr:
        r["L"] = {64: 64, 256: 128, 1024: 256, 2048: 64}[r["L"]]
        r["steps"] = 2 + r["steps"] % 3
    return tr


@pytest.mark.parametrize("tick", [5, 16])
def test_each_request_same_alone_and_in_the_mix(tick):
    tr = small_trace()
    mixed, alone = {}, {}
    lat, work, wall, iters = serve.serve_batched(tr, pool_bytes=256 << 20, tick_iters=tick, max_iter=60,
                                                 records=mixed)
    _, work_f, _, iters_f = serve.serve_fifo(tr, max_iter=60, ignore_arrivals=True, records=alone)
    assert sorted(mixed) == list(range(len(tr))) == sorted(alone)
    assert np.all(np.isfinite(lat)) and np.all(lat >= 0)
    assert iters == iters_f and work == work_f
    for i in range(len(tr)):
        a, b = mixed[i], alone[i]
        assert len(a) == len(b) == tr[i]["steps"]
        for ra, rb in zip(a, b):
            assert ra.iters == rb.iters
            assert ra.status == {0: 1, -4: 2, -5: 3}[rb.status]
            assert np.array_equal(ra.sigma_mean, rb.sigma_mean)
            assert np.array_equal(ra.eps_mean, rb.eps_mean)
            assert (ra.res_eq, ra.res_mac, ra.res_cmp) == (rb.res_eq, rb.res_mac, rb.res_cmp)


def test_small_pool_queues_requests():
    """A pool that holds about two requests at a time (besides the engine's
    tables) still serves all of them, each with its alone-records."""
    tr = small_trace(8, rate=200.0)
    mixed, alone = {}, {}
    serve.serve_batched(tr, pool_bytes=(1 << 20) + 2 * 1845248, tick_iters=8, max_iter=40, records=mixed)
    serve.serve_fifo(tr, max_iter=40, ignore_arrivals=True, records=alone)
    for i in range(len(tr)):
        assert [r.iters for r in mixed[i]] == [r.iters for r in alone[i]]
        assert all(np.array_equal(a.sigma_mean, b.sigma_mean) for a, b in zip(mixed[i], alone[i]))
