"""Host logic of the serving loop: admission by HBM footprint, FIFO hand-out,
batch caps, workspace release, oversized requests and error propagation.
The slots are fakes that only hold a simulated workspace, so everything
here runs on the CPU."""
import threading
import time

import numpy as np
import pytest

from paper_2009_03707_amd import serve

BPV = 10


class Ledger:
    """Workspace each fake slot really holds, checked at every launch."""

    def __init__(self, budget):
        self.budget = budget
        self.lock = threading.Lock()
        self.held = {}
        self.peak = 0
        self.violations = []
        self.running = 0
        self.max_running = 0


class FakeSlot:
    def __init__(self, ledger, idx, delay_per_voxel=2e-6, fail_on=None):
        self.ledger, self.idx, self.d, self.fail_on = ledger, idx, delay_per_voxel, fail_on
        self.ws = 0
        self.released = 0

    def run(self, batch):
        vox = sum(r.voxels for r in batch)
        with self.ledger.lock:
            self.ws = max(self.ws, BPV * vox)
            self.ledger.held[self.idx] = self.ws
            total = sum(self.ledger.held.values())
            self.ledger.peak = max(self.ledger.peak, total)
            alone = len(batch) == 1 and BPV * vox > self.ledger.budget
            if total > self.ledger.budget and not alone:
                self.ledger.violations.append((self.idx, total))
            self.ledger.running += 1
            self.ledger.max_running = max(self.ledger.max_running, self.ledger.running)
        try:
            if self.fail_on is not None and any(r.rid == self.fail_on for r in batch):
                raise RuntimeError("simulated launch failure")
            time.sleep(1e-3 + self.d * vox)
            for r in batch:
                r.counts = [r.rid, len(batch), 0, 0]
        finally:
            with self.ledger.lock:
                self.ledger.running -= 1

    def workspace_bytes(self):
        with self.ledger.lock:
            return self.ws

    def release(self):
        with self.ledger.lock:
            self.ws = 0
            self.ledger.held[self.idx] = 0
        self.released += 1

    def close(self):
        pass


def make_requests(n, lo, hi, seed=0, spread=0.0):
    rng = np.random.default_rng(seed)
    return [serve.Request(rid=i, arrival=float(i) * spread, nvox=int(rng.integers(lo, hi + 1))) for i in range(n)]


def run(slots=3, budget=3000, n=60, lo=10, hi=100, max_batch=64, max_batch_voxels=1 << 30, time_scale=0.0,
        spread=0.0, fail_on=None):
    led = Ledger(budget)
    fakes = [FakeSlot(led, i, fail_on=fail_on) for i in range(slots)]
    srv = serve.Server(fakes, hbm_budget=budget, max_batch=max_batch, max_batch_voxels=max_batch_voxels,
                       bytes_per_voxel=BPV)
    reqs = make_requests(n, lo, hi, spread=spread)
    try:
        summ = serve.run_stream(srv, reqs, time_scale=time_scale, timeout_s=60)
    finally:
        srv.close()
    return summ, srv, reqs, led, fakes


def test_all_complete_within_budget_under_pressure():
    # budget 3000 B = 300 voxels; requests 10..100 voxels, 3 slots
    summ, srv, reqs, led, fakes = run()
    assert all(r.done >= r.arrival >= 0 for r in reqs)
    assert all(r.counts[0] == r.rid for r in reqs)
    assert not led.violations, led.violations
    assert led.peak <= 3000
    assert srv.admission_waits > 0        # the small budget forced queueing
    assert summ["requests"] == 60 and summ["p99_ms"] >= summ["p50_ms"] >= 0


def test_fifo_hand_out():
    _, srv, reqs, _, _ = run(budget=2000, n=80)
    order = [r.order for r in sorted(reqs, key=lambda r: r.rid)]
    assert order == list(range(80))


def test_batches_respect_caps():
    _, srv, reqs, _, _ = run(budget=10 ** 9, n=100, max_batch=7, max_batch_voxels=400)
    for (_, size, vox, _, _) in srv.batches:
        assert size <= 7
        assert vox <= 400 or size == 1
    assert sum(b[1] for b in srv.batches) == 100
    assert max(b[1] for b in srv.batches) > 1  # requests were batched


def test_generous_budget_overlaps_slots():
    _, _, _, led, _ = run(budget=10 ** 9, n=40, max_batch=2)
    assert led.max_running >= 2


def test_idle_workspaces_released_for_large_request():
    # small requests first leave workspace in several slots; a request that
    # only fits once they are dropped must trigger releases, not starve
    led = Ledger(1000)
    fakes = [FakeSlot(led, i) for i in range(3)]
    srv = serve.Server(fakes, hbm_budget=1000, max_batch=1, bytes_per_voxel=BPV)
    reqs = [serve.Request(rid=i, arrival=0.0, nvox=40) for i in range(6)]
    reqs.append(serve.Request(rid=6, arrival=0.05, nvox=90))
    try:
        serve.run_stream(srv, reqs, time_scale=1.0, timeout_s=30)
    finally:
        srv.close()
    assert all(r.done > 0 for r in reqs)
    assert srv.releases > 0 and sum(f.released for f in fakes) > 0
    assert not led.violations


def test_oversized_request_runs_alone():
    big = serve.Request(rid=99, arrival=0.0, nvox=100)  # 1000 B > budget
    led2 = Ledger(500)
    fakes = [FakeSlot(led2, i) for i in range(2)]
    srv2 = serve.Server(fakes, hbm_budget=500, bytes_per_voxel=BPV)
    rs = [serve.Request(rid=i, arrival=0.0, nvox=20) for i in range(4)] + [big]
    try:
        serve.run_stream(srv2, rs, time_scale=0.0, timeout_s=30)
    finally:
        srv2.close()
    assert big.done > 0 and big.batch_size == 1
    assert not led2.violations


def test_launch_error_propagates():
    with pytest.raises(RuntimeError, match="simulated launch failure"):
        run(n=20, fail_on=5)


def test_latency_summary_fields():
    reqs = [serve.Request(rid=i, arrival=0.1 * i, nvox=10) for i in range(5)]
    for i, r in enumerate(reqs):
        r.done = r.arrival + 0.01 * (i + 1)
        r.batch_size = 1
    s = serve.summarize(reqs)
    assert s["requests"] == 5 and s["voxels"] == 50
    assert s["p50_ms"] == pytest.approx(30.0)
    assert s["max_ms"] == pytest.approx(50.0)
    assert s["makespan_s"] == pytest.approx(0.45)
