"""Continuous-batching server for time-varying fields.

Requests (advected timesteps arriving at a fixed rate, ad-hoc fields
arriving as a Poisson process) enter one FIFO queue.  A fixed set of slots
-- each a host thread with its own HIP stream and library context -- pulls
work: whenever a slot is free it takes the waiting requests, in arrival
order, that fit the HBM budget, the per-launch voxel cap and the batch-size
cap, and runs them as one batched launch (ms_complex_batch; a single request
uses ms_complex).  Requests that arrive while others are on the GPU are
admitted as soon as a slot and memory free up, so the work of different
slots overlaps on the device.  Inputs stay on the device: the base field is
resident in HBM and each timestep is formed there.

HBM admission.  A context keeps its workspace between calls (it only grows),
and reports exactly how much device memory it holds (workspace_bytes of
ms_ctx_get_timing); the server reads that after every batch and release.
The need of a batch not yet run is estimated as ``bytes_per_voxel * voxels``
with a per-voxel figure measured at the high-water mark of the densest
inputs.  A slot may take a batch only if the other slots' real holdings plus
max(its own real holding, the batch's estimate) stay within the budget; if
the slot then holds more than that reservation, the per-voxel estimate is
scaled up by the overshoot (batches hold per-field copies of their outputs,
so they need more per voxel than single fields do).
When nothing fits, the workspaces of idle slots are released first; a
request larger than the whole budget runs alone once every other slot is
idle.

Latency of a request = completion time - arrival time.  A request's result
is identical to running it alone: a batched launch is byte-identical per
field to single-field runs.
"""
from __future__ import annotations

import collections
import json
import threading
import time
from dataclasses import dataclass, field as dc_field

import numpy as np

# Device bytes per voxel that a context holds after a call, growth headroom
# of its buffers included: 343 at the high-water mark of the densest inputs
# measured (512^3 noise-dominated blobs: 0.41 critical cells and 4.6 closure
# entries of the 1-saddle/2-saddle DAG per vertex), rounded up.  It is an
# estimate, not a bound (the closure is data dependent); the server raises
# it when a slot is seen to hold more.
BYTES_PER_VOXEL = 400


@dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the stream
    field: object = None        # device float32 tensor (nz, ny, nx), or a size for fakes
    kind: str = "request"
    nvox: int = 0
    start: float = -1.0         # when its launch began
    done: float = -1.0          # when its launch completed
    batch_size: int = 0
    slot: int = -1
    order: int = -1             # position in which the queue handed it out
    transient: bool = False     # input formed on arrival; dropped once served
    result: object = None       # msc.Complex when results are kept
    counts: list = dc_field(default_factory=list)

    @property
    def voxels(self) -> int:
        return self.nvox if self.nvox else int(self.field.numel())


class GpuSlot:
    """Runs batches through one library context on its own stream."""

    def __init__(self, options: dict | None = None, keep_results: bool = False):
        import torch
        from . import msc
        self._msc = msc
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.ctx = msc.Context()
        if options:
            from . import autotune
            autotune.apply(self.ctx, dict(autotune.DEFAULT, **options))
        self.keep_results = keep_results

    def run(self, batch):
        import torch
        with torch.cuda.stream(self.stream):
            fs = [r.field for r in batch]
            rs = [self.ctx.complex_raw(fs[0])] if len(fs) == 1 else self.ctx.complex_batch_raw(fs)
            for r, res in zip(batch, rs):
                r.counts = list(res.count)
                if self.keep_results:
                    r.result = self._msc._to_complex(res, r.field)
            self.stream.synchronize()
        if not self.keep_results:
            for r in batch:
                if r.transient:
                    r.field = None

    def release(self):
        self.ctx.release()

    def workspace_bytes(self) -> int:
        """Device memory the slot's context holds now (exact)."""
        return int(self.ctx.timing()["workspace_bytes"])

    def start_counting(self):
        self.ctx.set_timing(True)

    def counters(self) -> dict:
        t = self.ctx.timing()
        return {"allocations": t["allocations"], "workspace_gb": round(t["workspace_bytes"] / 1e9, 2),
                "busy_s": round(t["total_ms"] / 1e3, 3), "calls": t["calls"]}

    def close(self):
        self.ctx.close()


class Server:
    """Slots pull batches from the queue; see the module docstring."""

    def __init__(self, slots, hbm_budget: int, max_batch_voxels: int = 192 << 20, max_batch: int = 64,
                 bytes_per_voxel: int = BYTES_PER_VOXEL, close_slots: bool = True):
        self.close_slots = close_slots
        self.hbm_budget = int(hbm_budget)
        self.max_batch_voxels = int(max_batch_voxels)
        self.max_batch = int(max_batch)
        self.bpv = int(bytes_per_voxel)
        self._slots = list(slots)
        n = len(self._slots)
        self._cv = threading.Condition()
        self._pending = collections.deque()
        self._busy = [False] * n
        # what each slot's context reported holding (at start, after its last
        # batch or release), and that or the reservation of its running batch
        self._real = [int(sl.workspace_bytes()) for sl in self._slots]
        self._resident = list(self._real)
        self._reserved = [0] * n      # what admission reserved for each slot's running batch
        self.estimate_raises = 0      # times a batch needed more than its reservation
        self._release = [False] * n   # asked to drop its workspace before the next batch
        self._stop = False
        self._handed = 0
        self._t0 = time.perf_counter()
        self.batches = []             # (slot, size, voxels, start, done)
        self.admission_waits = 0      # times a free slot found nothing that fits
        self.releases = 0
        self.max_resident = 0         # largest sum of what the slots' contexts reported holding
        self.errors = []
        self._threads = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(n)]
        for t in self._threads:
            t.start()

    # -- clock ---------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self._t0

    def start_clock(self):
        self._t0 = time.perf_counter()

    # -- queue ---------------------------------------------------------------
    def submit(self, req: Request):
        with self._cv:
            self._pending.append(req)
            self._cv.notify_all()

    def footprint(self, req: Request) -> int:
        return self.bpv * req.voxels

    def _take(self, s: int):
        """With the lock held: the next batch slot s may run, or None."""
        n = len(self._slots)
        if not self._pending or any(self._release[o] for o in range(n) if o != s):
            return None  # releases still in progress free memory first
        others = sum(self._resident[o] for o in range(n) if o != s)
        batch, vox, fp = [], 0, 0
        for r in self._pending:
            if batch and (len(batch) >= self.max_batch or vox + r.voxels > self.max_batch_voxels):
                break
            nfp = fp + self.footprint(r)
            if others + max(self._resident[s], nfp) > self.hbm_budget:
                break
            batch.append(r)
            vox += r.voxels
            fp = nfp
        if not batch:
            idle = [o for o in range(n) if o != s and not self._busy[o] and self._resident[o]]
            if idle:
                # nothing fits: idle slots drop their workspaces, then retry
                for o in idle:
                    self._release[o] = True
                    self._resident[o] = 0
                    self.releases += 1
                self._cv.notify_all()
                return None
            if any(self._busy[o] for o in range(n) if o != s):
                self.admission_waits += 1
                return None
            # every other slot is idle and empty: an oversized request runs alone
            batch, fp = [self._pending[0]], self.footprint(self._pending[0])
        for r in batch:
            self._pending.popleft()
            r.order = self._handed
            self._handed += 1
        self._busy[s] = True
        self._resident[s] = max(self._resident[s], fp)  # reserved until the real figure is read
        self._reserved[s] = self._resident[s]
        return batch

    def _worker(self, s: int):
        slot = self._slots[s]
        while True:
            release, batch = False, None
            with self._cv:
                while not self._stop:
                    if self._release[s]:
                        release = True
                        break
                    batch = self._take(s)
                    if batch:
                        break
                    self._cv.wait()
                if not release and not batch:
                    return
            if release:
                slot.release()
                held = slot.workspace_bytes()
                with self._cv:
                    self._real[s] = held
                    self._resident[s] = held
                    self._release[s] = False
                    self._cv.notify_all()
                continue
            t_start = self.now()
            try:
                slot.run(batch)
            except Exception as e:  # recorded; these requests stay unfinished
                self.errors.append(repr(e))
                t_done = -1.0
            else:
                t_done = self.now()
            for r in batch:
                r.start, r.done, r.batch_size, r.slot = t_start, t_done, len(batch), s
            held = slot.workspace_bytes()
            vox = sum(r.voxels for r in batch)
            with self._cv:
                self._busy[s] = False
                if held > self._reserved[s] > 0:
                    # the batch needed more than admission reserved for it:
                    # scale the per-voxel estimate by the overshoot
                    self.bpv = -(-self.bpv * held // self._reserved[s])
                    self.estimate_raises += 1
                self._real[s] = held
                self._resident[s] = held
                self.max_resident = max(self.max_resident, sum(self._real))
                self.batches.append((s, len(batch), vox, t_start, t_done))
                self._cv.notify_all()

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for t in self._threads:
            t.join()
        if self.close_slots:
            for sl in self._slots:
                sl.close()


def run_stream(server: Server, requests, produce=None, time_scale: float = 1.0, timeout_s: float = 600.0):
    """Submits `requests` at arrival * time_scale seconds after the start
    (time_scale 0: all at once) and waits for all of them; returns the
    latency summary.  `produce(req)`, if given, runs on the caller's thread
    right before submission (e.g. forms a timestep on the device) and must
    leave the request's field ready."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    server.start_clock()
    for r in reqs:
        r.arrival = r.arrival * time_scale
        delay = r.arrival - server.now()
        if delay > 0:
            time.sleep(delay)
        if produce is not None:
            produce(r)
        server.submit(r)
    deadline = time.perf_counter() + timeout_s
    while any(r.done < 0 for r in reqs):
        if server.errors:
            raise RuntimeError(f"serving failed: {server.errors[0]}")
        if time.perf_counter() > deadline:
            raise TimeoutError("requests not completed in time")
        time.sleep(0.002)
    return summarize(reqs)


def summarize(reqs) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs]) * 1e3
    vox = sum(r.voxels for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {
        "requests": len(reqs),
        "voxels": int(vox),
        "makespan_s": round(span, 4),
        "throughput_mvox_s": round(vox / span / 1e6, 2) if span > 0 else None,
        "p50_ms": round(float(np.percentile(lat, 50)), 2),
        "p99_ms": round(float(np.percentile(lat, 99)), 2),
        "max_ms": round(float(lat.max()), 2),
        "mean_batch": round(float(np.mean([r.batch_size for r in reqs])), 2),
    }


# -- the advected-field workload ------------------------------------------------

def stream_requests(base, steps: int = 200, step_hz: float = 10.0, rate: float = 20.0, seed: int = 7,
                    lo: int = 64, hi: int = 256, workers: int = 0):
    """Timestep requests t = 0..steps-1 arriving at t / step_hz (their fields
    are formed from the resident base when they arrive), plus the Poisson
    ad-hoc requests over the same duration, cubic with side U{lo..hi},
    alternating GRF and blob fields, moved to the device up front."""
    import torch
    from . import fields
    duration = steps / step_hz
    reqs = [Request(rid=t, arrival=t / step_hz, kind=f"timestep{t}", nvox=int(base.numel())) for t in range(steps)]
    arr = fields.request_arrivals(duration, rate=rate, seed=seed, lo=lo, hi=hi)
    specs = [fields.BatchItem(dims=(side, side, side), kind=kind, seed=s) for _, side, kind, s in arr]
    host = fields.make_batch(specs, workers=workers)
    for i, ((ta, side, kind, s), h) in enumerate(zip(arr, host)):
        reqs.append(Request(rid=steps + i, arrival=ta, field=torch.from_numpy(h).cuda(), kind=kind, nvox=h.size))
    return reqs


def roll_producer(base):
    """Forms timestep t on the device from the resident base (shifted by t
    voxels along x, periodic), just before the timestep is submitted."""
    import torch

    def produce(r: Request):
        if r.kind.startswith("timestep"):
            t = int(r.kind[len("timestep"):])
            r.field = torch.roll(base, shifts=t, dims=2)
            r.transient = True
            torch.cuda.current_stream().synchronize()
    return produce


def run_plain(requests, produce=None, options: dict | None = None) -> float:
    """The same requests one at a time through one context, in arrival
    order, with no batching and no overlap; returns seconds."""
    import torch
    slot = GpuSlot(options)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in sorted(requests, key=lambda r: r.arrival):
            if produce is not None:
                produce(r)
            slot.run([r])
        torch.cuda.synchronize()
        return time.perf_counter() - t0
    finally:
        slot.close()


def serve_benchmark(steps: int = 200, slots: int = 3, options: dict | None = None, log=print,
                    nx: int = 384, ny: int = 384, nz: int = 256) -> dict:
    """The advected GRF stream (periodic k^-3 base of nx x ny x nz, seed 0,
    `steps` timesteps at 10 Hz) plus Poisson requests at 20/s: served in real
    time (latency), the same requests served all at once (capacity), and
    the plain sequential path over the same requests."""
    import torch
    from . import fields
    base = torch.from_numpy(fields.grf_field((nx, ny, nz), seed=0)).cuda()
    produce = roll_producer(base)
    t0 = time.perf_counter()
    reqs = stream_requests(base, steps=steps)
    log(f"serve: {len(reqs)} requests generated in {time.perf_counter() - t0:.1f} s")
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.8)

    def fresh():
        return [Request(rid=r.rid, arrival=r.arrival, field=r.field, kind=r.kind, nvox=r.nvox) for r in reqs]

    torch.cuda.synchronize()
    slot_set = [GpuSlot(options) for _ in range(slots)]

    def serve(time_scale):
        for sl in slot_set:
            sl.start_counting()
        srv = Server(slot_set, hbm_budget=budget, close_slots=False)
        try:
            summ = run_stream(srv, fresh(), produce=produce, time_scale=time_scale)
        finally:
            srv.close()
        summ["slots"] = [sl.counters() for sl in slot_set]
        return summ, srv

    try:
        _, warm = serve(0.0)  # warm the slots' workspaces on the whole stream
        torch.cuda.synchronize()
        # device memory the contexts hold (their own exact figures) against
        # the largest batch each slot ran
        lib_bytes = sum(sl.workspace_bytes() for sl in slot_set)
        slot_vox = [max([b[2] for b in warm.batches if b[0] == i] or [0]) for i in range(slots)]
        rt, srv = serve(1.0)
        log(f"serve realtime: {json.dumps(rt)}")
        cap, srv2 = serve(0.0)
        log(f"serve all-at-once: {json.dumps(cap)}")
    finally:
        for sl in slot_set:
            sl.close()
    torch.cuda.empty_cache()  # the plain path starts from the same free memory as the slots did
    plain_s = run_plain(fresh(), produce=produce, options=options)
    vox = sum(r.voxels for r in reqs)
    out = {
        "workload": f"advected grf {nx}x{ny}x{nz}, {steps} steps at 10 Hz + Poisson 20/s sides 64..256",
        "slots": slots, "hbm_budget_gb": round(budget / 1e9, 1), "bytes_per_voxel": BYTES_PER_VOXEL,
        "bytes_per_voxel_learned": max(srv.bpv, srv2.bpv), "max_resident_gb": round(max(srv.max_resident,
                                                                                       srv2.max_resident) / 1e9, 2),
        "workspace_gb": round(lib_bytes / 1e9, 2),
        "measured_bytes_per_voxel": round(lib_bytes / max(sum(slot_vox), 1), 1),
        "realtime": rt, "all_at_once": cap,
        "plain_s": round(plain_s, 4), "plain_mvox_s": round(vox / plain_s / 1e6, 2),
        "served_vs_plain": round(cap["throughput_mvox_s"] / (vox / plain_s / 1e6), 3),
        "admission_waits": srv.admission_waits + srv2.admission_waits,
    }
    del base
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="serve the advected-field stream and report latency and throughput")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--slots", type=int, default=3)
    a = ap.parse_args()
    print(json.dumps(serve_benchmark(steps=a.steps, slots=a.slots)))
