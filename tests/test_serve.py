"""The serving scheduler: admission, continuous batching and failure isolation
(CPU, with a fake executor), and bitwise alone-vs-mix results on the GPU."""
import threading
import time

import numpy as np
import pytest

from paper_2109_09817_amd.serve import Executor, Server, latency_summary


class FakeExecutor(Executor):
    """Row-wise deterministic 'prediction' with an injected device latency."""

    def __init__(self, slots=2, max_rows=64, latency=0.004, poison=None):
        self.slots = slots
        self.max_rows = max_rows
        self.latency = latency
        self.poison = poison
        self.done_at = [None] * slots
        self.Z = [None] * slots
        self.launched = []
        self.max_concurrent = 0
        self.lock = threading.Lock()

    def batch_bytes(self, m):
        return 1000 * m

    def launch(self, slot, Z):
        if self.poison is not None and np.any(Z == self.poison):
            raise RuntimeError("poisoned batch")
        self.Z[slot] = Z.copy()
        self.done_at[slot] = time.perf_counter() + self.latency
        self.launched.append(Z.shape[0])
        busy = sum(1 for t in self.done_at if t is not None)
        self.max_concurrent = max(self.max_concurrent, busy)

    def ready(self, slot):
        return self.done_at[slot] is not None and time.perf_counter() >= self.done_at[slot]

    def fetch(self, slot, m):
        Z = self.Z[slot]
        self.done_at[slot] = None
        return Z.sum(axis=1), (Z * Z).sum(axis=1)


def test_all_requests_complete_with_rowwise_results():
    ex = FakeExecutor()
    srv = Server(ex, d=3)
    rng = np.random.default_rng(0)
    reqs = [rng.standard_normal((int(rng.integers(1, 20)), 3)) for _ in range(200)]
    futs = [srv.submit(z) for z in reqs]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    for z, r in zip(reqs, res):
        np.testing.assert_array_equal(r.mean, z.sum(axis=1))
        np.testing.assert_array_equal(r.var, (z * z).sum(axis=1))
    assert max(ex.launched) <= ex.max_rows
    # continuous batching: several requests share a batch, and batches overlap on the slots
    assert len(ex.launched) < len(reqs)
    assert ex.max_concurrent == 2
    s = latency_summary(res, 1.0)
    assert s["requests"] == 200 and s["p99_ms"] >= s["p50_ms"] > 0


def test_requests_arriving_during_a_batch_join_the_next_one():
    ex = FakeExecutor(slots=1, latency=0.05)
    srv = Server(ex, d=2)
    f0 = srv.submit(np.ones((4, 2)))
    time.sleep(0.01)  # batch 0 is on the device
    later = [srv.submit(np.full((3, 2), float(i))) for i in range(5)]
    assert not f0.done()
    for f in later:
        assert f.result(timeout=5).batch_rows == 15  # all five went together
    srv.close()


def test_bad_requests_fail_alone():
    ex = FakeExecutor(poison=-777.0)
    srv = Server(ex, d=2)
    good = srv.submit(np.ones((2, 2)))
    nan = srv.submit(np.array([[1.0, np.nan]]))
    shape = srv.submit(np.ones((2, 5)))
    big = srv.submit(np.ones((1000, 2)))
    assert isinstance(nan.exception(timeout=5), ValueError)
    assert isinstance(shape.exception(timeout=5), ValueError)
    assert isinstance(big.exception(timeout=5), ValueError)
    np.testing.assert_array_equal(good.result(timeout=5).mean, [2.0, 2.0])
    time.sleep(0.02)
    poisoned = srv.submit(np.array([[-777.0, 0.0]]))
    assert isinstance(poisoned.exception(timeout=5), RuntimeError)
    after = srv.submit(np.ones((1, 2)))
    np.testing.assert_array_equal(after.result(timeout=5).mean, [2.0])
    srv.close()


class FailingFetchExecutor(FakeExecutor):
    """The device work of batches holding the poison value fails when their results are fetched."""

    def fetch(self, slot, m):
        Z = self.Z[slot]
        self.done_at[slot] = None
        if np.any(Z == -7.5):
            raise RuntimeError("device error surfaced at fetch")
        return Z.sum(axis=1), (Z * Z).sum(axis=1)


def test_failed_fetch_fails_its_batch_and_serving_continues():
    ex = FailingFetchExecutor(slots=1, latency=0.002)
    srv = Server(ex, d=2)
    bad = srv.submit(np.full((3, 2), -7.5))
    bad.exception(timeout=10)  # resolved, not hanging
    good = [srv.submit(np.ones((2, 2)) * i) for i in range(20)]
    res = [f.result(timeout=10) for f in good]
    srv.close()
    assert isinstance(bad.exception(), RuntimeError)
    assert [float(r.mean[0]) for r in res] == [2.0 * i for i in range(20)]
    assert srv.used == 0


class DyingExecutor(FakeExecutor):
    """ready() raises: the scheduler thread itself cannot continue."""

    def ready(self, slot):
        raise MemoryError("scheduler-level failure")


def test_scheduler_failure_resolves_every_pending_request():
    ex = DyingExecutor(slots=1, latency=10.0)
    srv = Server(ex, d=2)
    futs = [srv.submit(np.ones((1, 2))) for _ in range(5)]
    for f in futs:
        assert isinstance(f.exception(timeout=10), RuntimeError)
    srv.thread.join(timeout=10)
    assert not srv.thread.is_alive()
    late = srv.submit(np.ones((1, 2)))
    assert isinstance(late.exception(timeout=1), RuntimeError)
    with pytest.raises(RuntimeError) as ei:
        srv.close()
    assert isinstance(ei.value.__cause__, MemoryError)


def test_memory_budget_limits_inflight_batches():
    ex = FakeExecutor(slots=4, latency=0.02)
    srv = Server(ex, d=2, hbm_budget=1000 * 64)  # exactly one full batch fits
    futs = [srv.submit(np.ones((64, 2))) for _ in range(6)]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    assert ex.max_concurrent == 1


@pytest.mark.gpu
def test_gpu_serving_alone_equals_in_mix():
    import torch
    import synth
    from _helpers import dev
    from paper_2109_09817_amd import gp
    from paper_2109_09817_amd.serve import GpuExecutor
    n, d, kc = 20000, 48, 32
    p = synth.make_problem("c5", n=n, cond_variant=True)
    k = gp.Kernel(p.ell, p.sf, p.noise)
    X = dev(p.X)
    rng = np.random.default_rng(0)
    model = gp.PredictModel(k, X, dev(rng.standard_normal(n)), dev(rng.standard_normal((kc, n)) * 0.01))
    q = synth.query_molecule("c5", 117, seed=42)
    alone_srv = Server(GpuExecutor(model, slots=2, max_rows=1024), d=d)
    alone = alone_srv.submit(q).result(timeout=60)
    alone_srv.close()
    mix_srv = Server(GpuExecutor(model, slots=2, max_rows=1024), d=d)
    others = [synth.query_molecule("c5", int(m), seed=int(s)) for s, m in enumerate(rng.integers(10, 300, 20))]
    with mix_srv.cv:  # hold the scheduler so that all requests are queued together
        futs = [mix_srv.submit(z) for z in others[:7]] + [mix_srv.submit(q)] + [mix_srv.submit(z) for z in others[7:]]
    res = [f.result(timeout=60) for f in futs]
    mix_srv.close()
    mine = res[7]
    assert mine.batch_rows > q.shape[0]  # it really shared a batch
    np.testing.assert_array_equal(mine.mean, alone.mean)
    np.testing.assert_array_equal(mine.var, alone.var)
    torch.cuda.synchronize()
