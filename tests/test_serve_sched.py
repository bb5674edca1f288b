"""Scheduling of the serving loop with a fake executor (no GPU): arrival
order, memory admission, overlap of lanes, oversized requests, and the
request pool's distribution."""
import threading
import time

import numpy as np

from paper_1906_08148_amd import serve


class FakeLane:
    """Runs a batch by sleeping; records the peak footprint it was given."""

    def __init__(self, budget, per_req=0.02):
        self.budget = budget
        self.per_req = per_req
        self.batches = []
        self.peak = 0
        self.lock = threading.Lock()

    def run(self, specs):
        fp = sum(s.footprint() for s in specs)
        with self.lock:
            self.peak = max(self.peak, fp)
            self.batches.append([s.rid for s in specs])
        time.sleep(self.per_req * len(specs) ** 0.5)
        return [{"stats": {"flops": 1.0, "rid": s.rid}} for s in specs]


def spec(rid, n=2048, kind="1d"):
    return serve.RequestSpec(serve.MatrixSpec(kind, n, 0.5, rid), 1e-6, 1, rid=rid)


def test_every_request_completes_in_order_of_batches():
    lanes = [FakeLane(10 << 30)]
    s = serve.Scheduler(lanes, max_batch=4)
    hs = [s.submit(spec(i)) for i in range(10)]
    for h in hs:
        assert h.done.wait(5)
    s.close()
    assert [h.result.rid for h in hs] == list(range(10))
    flat = [r for b in lanes[0].batches for r in b]
    assert sorted(flat) == list(range(10))
    assert all(len(b) <= 4 for b in lanes[0].batches)
    # arrival order is kept inside the single lane
    assert flat == sorted(flat)


def test_admission_respects_lane_budget():
    big = spec(0, 65536, "3d")
    budget = big.footprint() + spec(1, 4096, "3d").footprint() // 2
    lanes = [FakeLane(budget), FakeLane(budget)]
    s = serve.Scheduler(lanes, max_batch=16)
    hs = [s.submit(spec(i, 65536 if i % 3 == 0 else 4096, "3d")) for i in range(12)]
    for h in hs:
        assert h.done.wait(10)
    s.close()
    for l in lanes:
        assert l.peak <= budget
    assert all(not h.result.error for h in hs)


def test_oversized_request_fails_fast():
    lanes = [FakeLane(1 << 20)]
    s = serve.Scheduler(lanes)
    h = s.submit(spec(0, 65536, "3d"))
    assert h.done.wait(1)
    assert h.result.error
    s.close()


def test_two_lanes_overlap():
    lanes = [FakeLane(10 << 30, per_req=0.2), FakeLane(10 << 30, per_req=0.2)]
    s = serve.Scheduler(lanes, max_batch=1)
    t0 = time.perf_counter()
    hs = [s.submit(spec(i)) for i in range(4)]
    for h in hs:
        h.done.wait(5)
    dt = time.perf_counter() - t0
    s.close()
    assert dt < 0.7  # 4 x 0.2 s serially would take 0.8 s
    assert {h.result.lane for h in hs} == {0, 1}


def test_requests_arriving_during_a_batch_join_the_next():
    lanes = [FakeLane(10 << 30, per_req=0.1)]
    s = serve.Scheduler(lanes, max_batch=16)
    h0 = s.submit(spec(0))
    time.sleep(0.02)  # the first batch is running
    hs = [s.submit(spec(i)) for i in range(1, 6)]
    for h in [h0] + hs:
        h.done.wait(5)
    s.close()
    assert lanes[0].batches[0] == [0]
    assert lanes[0].batches[1] == [1, 2, 3, 4, 5]


def test_poisson_stream_and_summary():
    lanes = [FakeLane(10 << 30, per_req=0.005)]
    s = serve.Scheduler(lanes, max_batch=8)
    res = serve.run_stream(s, [spec(i) for i in range(20)], rate=400.0)
    s.close()
    summ = serve.summarize(res)
    assert summ["completed"] == 20 and summ["p99_s"] >= summ["p50_s"] > 0


def test_request_pool_distribution():
    pool = serve.request_pool(512)
    ns = np.array([r.mat.n for r in pool])
    assert ns.min() >= 2048 and ns.max() <= 65536 and np.all(ns % 2048 == 0)
    assert 0.4 < np.mean([r.mat.kind == "1d" for r in pool]) < 0.6
    al = np.array([r.mat.alpha for r in pool])
    assert al.min() >= 0.2 and al.max() <= 1.0
    lt = np.log10([r.tau for r in pool])
    assert lt.min() >= -8 and lt.max() <= -4
    assert set(r.mode for r in pool) == {0, 1, 2}
    assert serve.request_pool(512)[17].mat == pool[17].mat  # seeded
