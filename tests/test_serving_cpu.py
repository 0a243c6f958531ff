"""Admission and batching logic of the serving loop, with a host-side double
for the GPU launch (no device needed)."""
import time

from paper_1905_04356_amd import serving as S


class FakeEvent:
    def __init__(self, done):
        self.done = done

    def query(self):
        return time.perf_counter() >= self.done


def fake_pool(footprints):
    return [S.PoolItem(4, 4, 4, 32, None, None, None, None, fp) for fp in footprints]


def run(footprints, arrivals, items, budget, slots, service_s, max_batch=256):
    launches = []

    def launcher(si, its):
        launches.append((si, [it.footprint for it in its]))
        return FakeEvent(time.perf_counter() + service_s), [None] * len(its)

    srv = S.Server(0, fake_pool(footprints), budget, streams=slots, max_batch=max_batch,
                   launcher=launcher)
    stats = srv.run(arrivals, items)
    return srv, stats, launches


def test_all_requests_complete_in_fifo_admission_order():
    arrivals = [0.001 * i for i in range(200)]
    items = [i % 3 for i in range(200)]
    srv, stats, launches = run([10, 20, 30], arrivals, items, budget=10 ** 9, slots=2,
                               service_s=0.003)
    assert stats["requests"] == 200
    assert srv.admitted == list(range(200))
    assert stats["batches"] == len(launches) < 200   # requests were batched
    assert stats["p50_ms"] >= 0


def test_budget_is_never_exceeded_and_backpressure_waits():
    arrivals = [0.0] * 50
    items = [0] * 50
    srv, stats, launches = run([100], arrivals, items, budget=350, slots=4, service_s=0.002)
    assert srv.peak_used <= 350
    assert all(sum(fps) <= 350 for _, fps in launches)
    assert stats["requests"] == 50


def test_oversized_request_runs_alone_when_idle():
    arrivals = [0.0, 0.0, 0.0]
    items = [0, 1, 0]
    srv, stats, launches = run([10, 1000], arrivals, items, budget=100, slots=2,
                               service_s=0.001)
    assert stats["requests"] == 3
    assert [1000] in [fps for _, fps in launches]


def test_max_batch_respected():
    arrivals = [0.0] * 40
    items = [0] * 40
    srv, stats, launches = run([1], arrivals, items, budget=10 ** 6, slots=1, service_s=0.001,
                               max_batch=8)
    assert max(len(fps) for _, fps in launches) <= 8


def test_large_requests_run_alone_in_fifo_order():
    big = S.PoolItem(128, 128, 128, 6000, None, None, None, None, 10)    # 3 128^2 2^14
    pool = fake_pool([10, 10]) + [big]
    assert big.work >= 1 << 25 > pool[0].work
    launches = []

    def launcher(si, its):
        launches.append([it.m for it in its])
        return FakeEvent(time.perf_counter() + 0.002), [None] * len(its)

    arrivals = [0.0005 * i for i in range(120)]
    items = [2 if i % 7 == 3 else i % 2 for i in range(120)]
    srv = S.Server(0, pool, 10 ** 9, streams=2, launcher=launcher)
    stats = srv.run(arrivals, items)
    assert stats["requests"] == 120
    assert srv.admitted == list(range(120))
    assert all(len(b) == 1 for b in launches if 128 in b)
    assert any(len(b) > 1 for b in launches)            # the small ones still batch
