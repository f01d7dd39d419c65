"""Serving loop on the GPU: every request served in the mix (continuous
batching over several slots, with and without HBM pressure) is
byte-identical to the same field run alone, and a timestep and an ad-hoc
request equal the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stream():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_03707_amd import serve
    base = torch.from_numpy(fields.grf_field((40, 36, 24), seed=0)).cuda()
    reqs = serve.stream_requests(base, steps=12, step_hz=50.0, rate=60.0, seed=7, lo=8, hi=36, workers=1)
    assert len(reqs) > 12  # some ad-hoc requests arrived
    return base, reqs


def _serve(base, reqs, budget, slots=3, max_batch=64):
    from paper_2009_03707_amd import serve
    rs = [serve.Request(rid=r.rid, arrival=r.arrival, field=r.field, kind=r.kind, nvox=r.nvox) for r in reqs]
    srv = serve.Server([serve.GpuSlot(keep_results=True) for _ in range(slots)], hbm_budget=budget,
                       max_batch=max_batch)
    try:
        summ = serve.run_stream(srv, rs, produce=serve.roll_producer(base), time_scale=1.0, timeout_s=120)
    finally:
        srv.close()
    return rs, summ, srv


def _check_alone(rs):
    from gpu_util import same_complex
    from paper_2009_03707_amd import msc
    ctx = msc.Context()
    try:
        for r in rs:
            assert r.done >= r.arrival
            same_complex(r.result, msc.complex_(r.field, ctx))
    finally:
        ctx.close()


def test_served_equals_alone(stream):
    base, reqs = stream
    rs, summ, srv = _serve(base, reqs, budget=1 << 40)
    assert summ["requests"] == len(reqs)
    _check_alone(rs)


class WatchedSlot:
    """A GPU slot that records, after every batch and release, the device
    memory all watched slots' contexts really hold (their own figures)."""
    peak = 0
    slots = []

    def __init__(self):
        from paper_2009_03707_amd import serve
        self.inner = serve.GpuSlot(keep_results=True)
        WatchedSlot.slots.append(self)

    def _note(self):
        WatchedSlot.peak = max(WatchedSlot.peak, sum(s.inner.workspace_bytes() for s in WatchedSlot.slots))

    def run(self, batch):
        self.inner.run(batch)
        self._note()

    def release(self):
        self.inner.release()
        self._note()

    def workspace_bytes(self):
        return self.inner.workspace_bytes()

    def close(self):
        self.inner.close()


def test_served_under_hbm_pressure_equals_alone(stream):
    from paper_2009_03707_amd import serve
    base, reqs = stream
    # measure what the largest request really needs on an empty context
    bigf = max([base] + [r.field for r in reqs if r.field is not None], key=lambda t: t.numel())
    probe = serve.GpuSlot()
    probe.run([serve.Request(rid=-1, arrival=0.0, field=bigf, kind="probe")])
    need = probe.workspace_bytes()
    probe.close()
    # room for about two of the largest requests: slots must queue and release;
    # the per-voxel estimate is calibrated on that field, as a deployment would
    budget = 2 * need + need // 2
    WatchedSlot.peak, WatchedSlot.slots = 0, []
    slots = [WatchedSlot() for _ in range(3)]

    def fresh():
        return [serve.Request(rid=r.rid, arrival=r.arrival, field=r.field, kind=r.kind, nvox=r.nvox) for r in reqs]

    # a first pass calibrates the per-voxel estimate on this stream (as the
    # benchmark warms its slots); the second pass is the one checked
    bpv = -(-need // int(bigf.numel()))
    for rep in range(2):
        WatchedSlot.peak = 0
        rs = fresh()
        srv = serve.Server(slots, hbm_budget=budget, bytes_per_voxel=bpv, close_slots=False)
        try:
            serve.run_stream(srv, rs, produce=serve.roll_producer(base), time_scale=1.0, timeout_s=120)
        finally:
            srv.close()
        bpv = srv.bpv
    for sl in slots:
        sl.close()
    assert srv.admission_waits + srv.releases > 0, "the budget should have forced queueing or releases"
    assert WatchedSlot.peak <= budget, (WatchedSlot.peak, budget, srv.estimate_raises)
    assert srv.max_resident <= budget
    _check_alone(rs)


def test_served_timestep_and_request_equal_oracle(stream):
    from gpu_util import csr_np, u32
    base, reqs = stream
    rs, _, _ = _serve(base, reqs, budget=1 << 40, slots=2)
    picks = [r for r in rs if r.kind == "timestep5"] + [next(r for r in rs if not r.kind.startswith("timestep"))]
    for r in picks:
        f = r.field.cpu().numpy()
        if r.kind == "timestep5":
            np.testing.assert_array_equal(f, fields.advected_step(base.cpu().numpy(), 5))
        ref = O.complex_(f)
        np.testing.assert_array_equal(u32(r.result.grad).reshape(f.shape), ref.grad)
        assert r.result.count == ref.crit.count.tolist()
        rp, col, val = ref.p.csr()
        g = csr_np(r.result.m21t)
        np.testing.assert_array_equal(g[0], rp)
        np.testing.assert_array_equal(g[1], col)
        np.testing.assert_array_equal(g[2], val)
