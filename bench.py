#!/usr/bin/env python
"""Benchmark of the Morse-Smale hot path on one MI355X.

A step is one ms_complex call (gradient, critical cells, saddle-extremum
arcs, saddle-saddle reachability, DAG minor, path counting and every arc
matrix with its transpose) on a field already resident in HBM; results stay
in HBM.  Prints one JSON line.

Default workload: 512^3 float32 sum of 2000 seeded anisotropic Gaussian blobs
plus N(0, 0.01) noise (the densest critical-point configuration).
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CSRC = os.path.join(ROOT, "paper_2009_03707_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def make_workload(name):
    from paper_2009_03707_amd import fields
    if name == "blobs512":
        f = fields.blob_field((512, 512, 512), nblobs=2000, seed=0)
        desc = ("blobs512: 512x512x512 float32, sum of 2000 anisotropic Gaussian blobs (amplitude U[-1,1], "
                "sigma U[2,20] per axis, seed 0) plus N(0,0.01) noise")
    elif name == "grf256":
        f = fields.grf_field((256, 256, 256), seed=0)
        desc = "grf256: 256x256x256 float32 Gaussian random field, power spectrum k^-3, seed 0"
    elif name == "sine32":
        f = fields.sine_field(32, seed=0)
        desc = "sine32: 32^3 float32 sin(3x)+sin(5y)+sin(7z) plus U(-1e-3,1e-3) noise, seed 0"
    else:
        raise SystemExit(f"unknown workload {name}")
    return f, desc


def cpu_baseline(f, side):
    """The oracle, unmodified, on a side^3 crop of the same field (one core)."""
    import numpy as np
    from oracle import oracle as O
    crop = np.ascontiguousarray(f[:side, :side, :side])
    t0 = time.perf_counter()
    O.complex_(crop)
    dt = time.perf_counter() - t0
    n = crop.size
    return {"value": round(n / dt / 1e6, 4), "unit": "Mvoxels/s", "cores": 1, "kind": "oracle",
            "sample": f"{side}^3 corner crop of the benchmark field ({n} voxels), whole hot path, "
                      f"{dt:.1f} s on one core of {cpu_model()} (host has {os.cpu_count()} logical CPUs)"}


def measured_traffic(kernel, source):
    """HBM bytes per launch of `kernel` from its committed counter summary
    (profiles/<kernel>_blobs512_traffic.txt: FETCH_SIZE and WRITE_SIZE,
    scaled by a plain copy of known size), or None when the kernel's source
    file has changed since it was measured."""
    import hashlib
    try:
        lines = open(os.path.join(PROFILES, f"{kernel}_blobs512_traffic.txt")).read().splitlines()
    except OSError:
        return None
    kv = dict(l.split(":", 1) for l in lines if ":" in l and not l.startswith("#"))
    src = hashlib.sha256(open(os.path.join(CSRC, source), "rb").read()).hexdigest()
    if kv.get("source_sha256", "").strip() != src:
        return None
    try:
        return int(kv["traffic_bytes_per_launch"].strip())
    except (KeyError, ValueError):
        return None


def valu_profile(kernel, source):
    """VALU counters of `kernel` from its committed summary
    (profiles/<kernel>_blobs512_valu.txt), or None when the kernel's source
    has changed since they were taken."""
    import hashlib
    try:
        lines = open(os.path.join(PROFILES, f"{kernel}_blobs512_valu.txt")).read().splitlines()
    except OSError:
        return None
    kv = dict((a.strip(), b.strip()) for a, b in (l.split(":", 1) for l in lines if ":" in l and not l.startswith("#")))
    src = hashlib.sha256(open(os.path.join(CSRC, source), "rb").read()).hexdigest()
    if kv.get("source_sha256") != src:
        return None
    return {k: float(v) for k, v in kv.items() if k not in ("kernel", "source", "source_sha256")}


# MI355X vector ALU: 256 compute units at 2.4 GHz, each issuing one wave64
# VALU instruction per cycle across its four SIMDs (a SIMD takes four cycles
# for a wave64 instruction on 16 lanes) = 64 lane-operations per CU-cycle.
VALU_PEAK_LANE_OPS = 256 * 2.4e9 * 64


def roofline(kernel, source, bytes_per_launch, avg_launch_ms):
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    return {"kernel": kernel, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel, source),
            "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_launch_ms, 4)}


def copy_bandwidth(torch, mib=1024, reps=5):
    """GB/s of a plain device-to-device copy (bytes read + bytes written)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * 4 * n / (ms / 1e3) / 1e9


def transfer_bench(ctx, f, torch, msc, reps=3):
    """The same call with the field copied in from pinned host memory and the
    critical list and the six arc matrices copied back (the gradient stays on
    the device): whole-job rate including PCIe, for context only."""
    import ctypes as C
    fh = torch.from_numpy(f).pin_memory()
    fd = torch.empty(fh.shape, dtype=fh.dtype, device="cuda")
    fd.copy_(fh, non_blocking=True)
    r = ctx.complex_raw(fd)
    torch.cuda.synchronize()

    def outputs(r):
        n = int(sum(r.count))
        out = [(r.crit.id, 4 * n), (r.crit.index, n), (r.crit.value, 4 * n), (r.crit.vmax, 4 * n)]
        for name in ("m10", "m10t", "m21", "m21t", "m32", "m32t"):
            m = getattr(r.arcs, name)
            out += [(m.rowptr, 8 * (m.nrows + 1)), (m.col, 4 * m.nnz), (m.val, 8 * m.nnz)]
        return [(p, b) for p, b in out if p and b > 0]

    d2h = sum(b for _, b in outputs(r))
    host = torch.empty(d2h, dtype=torch.uint8, pin_memory=True)
    hip = msc._hip_rt()
    t0 = time.perf_counter()
    for _ in range(reps):
        fd.copy_(fh, non_blocking=True)
        r = ctx.complex_raw(fd)
        o = 0
        for p, b in outputs(r):
            rc = hip.hipMemcpyAsync(C.c_void_p(host.data_ptr() + o), C.c_void_p(p), b, 2, msc._stream_handle())
            if rc != 0:
                raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
            o += b
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    return {"ms_per_step": round(ms, 2), "mvox_s": round(f.size / ms / 1e3, 2), "h2d_bytes": int(fh.numel() * 4),
            "d2h_bytes": int(d2h)}


def out_of_core_bench(ctx, f, torch, msc, slab=64, reps=2):
    """ms_gradient_critical_chunked on the benchmark field held in host
    memory, streamed in z-slabs (copies of the next slab overlap the current
    slab's kernels); whole-job rate including the host-to-device traffic.
    Then ms_manifolds_chunked on the same field and slabs."""
    import numpy as np
    f = np.ascontiguousarray(f)
    ctx.gradient_critical_chunked(f, slab, want_grad=False)  # warm
    t0 = time.perf_counter()
    for _ in range(reps):
        _, cid, idx, val, vmax, cnt = ctx.gradient_critical_chunked(f, slab, want_grad=False)
    ms = (time.perf_counter() - t0) / reps * 1e3
    del cid, idx, val, vmax
    # the manifold labels of the same field, stitched across the slabs
    ctx.manifolds_chunked(f, slab)  # warm (pinned label staging)
    t0 = time.perf_counter()
    for _ in range(reps):
        lo, hi, cnt_l = ctx.manifolds_chunked(f, slab)
        del lo, hi
    ms_l = (time.perf_counter() - t0) / reps * 1e3
    if cnt_l != cnt:
        raise SystemExit(f"out-of-core label counts {cnt_l} differ from {cnt}")
    return {"slab_rows": slab, "ms_per_call": round(ms, 2), "mvox_s": round(f.size / ms / 1e3, 2),
            "h2d_gbs": round(4 * f.size * (slab + 3) / slab / (ms / 1e3) / 1e9, 2), "critical_counts": cnt,
            "labels_ms_per_call": round(ms_l, 2), "labels_mvox_s": round(f.size / ms_l / 1e3, 2),
            "note": "host field in, critical list out (64-bit ids); counts equal the in-HBM run's; labels: "
                    "ms_manifolds_chunked, both 64-bit label arrays out (16 bytes per vertex)"}


def graph_bench(torch, msc, nthreads=16):
    """Host MS-complex graph of the 256^3 GRF (build from the device result)
    and its simplification, serial and by the paper's subgrid schedule."""
    from paper_2009_03707_amd import fields
    f = fields.grf_field((256, 256, 256), seed=0)
    fd = torch.from_numpy(f).cuda()
    ctx = msc.Context()
    r = ctx.complex_raw(fd)
    torch.cuda.synchronize()
    out = {"workload": "grf256 (256^3 k^-3 GRF, seed 0)", "nodes": int(sum(r.count)), "threads": nthreads}
    t0 = time.perf_counter()
    g = msc.Graph.from_result(ctx, r, (256, 256, 256), nthreads=nthreads)
    out["build_s"] = round(time.perf_counter() - t0, 3)
    out["arcs"] = g.counts()[1]
    thr = 0.05  # in units of the field's standard deviation (the GRF is normalised)
    t0 = time.perf_counter()
    n = g.simplify(thr, msc.MS_SIMPLIFY_SERIAL, 1)
    out["serial"] = {"threshold": thr, "cancellations": n, "s": round(time.perf_counter() - t0, 3),
                     "alive": g.counts()[0]}
    g.close()
    for k in (2, nthreads):  # the paper's two subgrids per round, and one per host thread
        g = msc.Graph.from_result(ctx, r, (256, 256, 256), nthreads=nthreads)
        t0 = time.perf_counter()
        n = g.simplify(thr, msc.MS_SIMPLIFY_SUBGRID, k)
        out[f"subgrid{k}"] = {"threshold": thr, "cancellations": n, "s": round(time.perf_counter() - t0, 3),
                              "alive": g.counts()[0]}
        g.close()
    ctx.close()
    return out


def batch_bench(args, torch, msc):
    """The same kernels on the uneven 64-field batch: one field per call in
    sequence (plain) versus one ms_complex_batch call (batched)."""
    from paper_2009_03707_amd import fields
    specs = fields.batch_specs(args.batch)
    log(f"generating the {args.batch}-field batch")
    hs = fields.make_batch(specs)
    fs = [torch.from_numpy(h).cuda() for h in hs]
    del hs
    nvox = sum(int(f.numel()) for f in fs)
    ctx = msc.Context()
    tuned = None
    if not args.no_autotune:
        from paper_2009_03707_amd import autotune
        tuned = autotune.tune(ctx, fs, log=log)
    for f in fs:  # warm every per-field shape
        ctx.complex_raw(f)
    ctx.complex_batch_raw(fs)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(reps):
        for f in fs:
            ctx.complex_raw(f)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) / reps * 1e3
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.complex_batch_raw(fs)
    torch.cuda.synchronize()
    batch_ms = (time.perf_counter() - t0) / reps * 1e3
    log(f"batch of {len(fs)}: plain {plain_ms:.1f} ms, batched {batch_ms:.1f} ms")
    ctx.close()
    return {"workload": f"batch{len(fs)}: {len(fs)} float32 fields, sides U{{64..320}} per axis (seeds 1000+i), "
                        "even i k^-3 GRF, odd i blobs (2000 scaled by volume) + N(0,0.01)",
            "fields": len(fs), "voxels": nvox, "reps": reps,
            "plain_ms": round(plain_ms, 2), "batched_ms": round(batch_ms, 2),
            "plain_mvox_s": round(nvox / plain_ms / 1e3, 2), "batched_mvox_s": round(nvox / batch_ms / 1e3, 2),
            "speedup": round(plain_ms / batch_ms, 3), "launch_params": tuned}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="blobs512")
    ap.add_argument("--cpu-sample", type=int, default=160, help="side of the oracle crop (0 = skip)")
    ap.add_argument("--batch", type=int, default=64, help="fields in the batched comparison (0 = skip)")
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch parameters")
    ap.add_argument("--params", default=None,
                    help='fixed launch parameters instead of autotuning, e.g. \'{"tile": 5, "schedule": 2}\'')
    ap.add_argument("--serve-steps", type=int, default=200,
                    help="timesteps of the served advected-field stream (0 = skip)")
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--no-transfers", dest="transfers", action="store_false",
                    help="skip the run that includes the host-device copies")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="skip the out-of-core run and the host graph / simplification timings")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device-to-device copy of this many MiB (a known-size kernel for "
                         "scaling hardware traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the hot path is measured on a single MI355X "
              f"(asked for --gpus {args.gpus}); multi-GPU sharding is a design note, not a run.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_03707_amd import msc

    if args.calibrate_copy > 0:
        n_el = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n_el, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {4 * n_el} bytes read and written once")
        del src, dst

    log(f"generating {args.workload}")
    f, desc = make_workload(args.workload)
    n = int(f.size)
    fd = torch.from_numpy(f).cuda()
    ctx = msc.Context()
    tuned = None
    if args.params:
        from paper_2009_03707_amd import autotune
        tuned = dict(autotune.DEFAULT, **json.loads(args.params))
        autotune.apply(ctx, tuned)
    elif not args.no_autotune:
        from paper_2009_03707_amd import autotune
        tuned = autotune.tune(ctx, [fd], log=log)
    for i in range(args.warmup):
        r = ctx.complex_raw(fd)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ctx.complex_raw(fd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed {args.steps} steps in {t1 - t0:.3f} s")
    # stage and per-launch times come from further steps with the library's
    # event timing on (its events sit between launches, so they are kept out
    # of the timed steps above)
    prof_steps = max(1, min(args.steps, 3))
    ctx.set_timing(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(prof_steps):
        r = ctx.complex_raw(fd)
    torch.cuda.synchronize()
    instrumented_ms = (time.perf_counter() - tp0) / prof_steps * 1e3
    tm = ctx.timing()
    stats = {k: int(getattr(r.arcs.stats, k)) for k, _ in msc.Stats._fields_}
    counts = list(r.count)
    ms_per_step = (t1 - t0) / args.steps * 1e3
    value = n / (ms_per_step / 1e3) / 1e6
    calls = max(tm["calls"], 1)
    grad_ms = tm["gradient_ms"] / calls
    grad_bytes = 8 * n  # 4 B field read + 4 B gradient word written per vertex
    grad_roof = roofline("grad_lowerstar", "gradient.hip", grad_bytes, grad_ms)
    vp = valu_profile("grad_lowerstar", "gradient.hip")
    if vp:
        # the gradient is bound by the vector ALU: active lane-operations
        # (VALU instructions x the lanes each had active, from the counters)
        # per second against the VALU peak; issue_frac counts every
        # instruction as 64 lanes (the issue slots the kernel used)
        lane_ops = vp["thread_cycles_valu_per_launch"]
        issued = vp["valu_insts_per_launch"] * 64
        grad_roof.update({"bound": "alu", "hbm_gbs": grad_roof["achieved"], "hbm_frac": grad_roof["frac"],
                          "achieved": round(lane_ops / (grad_ms / 1e3) / 1e12, 2),
                          "peak": round(VALU_PEAK_LANE_OPS / 1e12, 2), "unit": "T lane-ops/s",
                          "frac": round(lane_ops / (grad_ms / 1e3) / VALU_PEAK_LANE_OPS, 4),
                          "issue_frac": round(issued / (grad_ms / 1e3) / VALU_PEAK_LANE_OPS, 4),
                          "lane_ops_per_launch": int(lane_ops), "valu_insts_per_launch": int(vp["valu_insts_per_launch"])})
    # critical-cell stage: every gradient word read once, 13 B written per
    # critical cell (id, index, value, highest vertex)
    crit_ms = tm["critical_ms"] / calls
    ncrit = int(sum(r.count))
    crit_roof = roofline("crit_count+crit_scatter", "critical.hip", 4 * n + 13 * ncrit, crit_ms)
    tc, ts = measured_traffic("crit_count", "critical.hip"), measured_traffic("crit_scatter", "critical.hip")
    crit_roof["traffic"] = tc + ts if tc is not None and ts is not None else None
    crit_roof["note"] = "whole critical stage (both passes, scan, count readback), per call"
    if tm["rank_launches"] > 0:
        # path-count ranking: per input entry 4 B row + 8 B count read and a
        # 1 B head flag + 8 B scaled count written at its merged position;
        # per run head its 4 B row written
        rank_bytes = 21 * tm["rank_entries"] + 4 * tm["rank_heads"]
        main_roof = roofline("k_entry_rank", "paths.hip", rank_bytes / tm["rank_launches"],
                             tm["rank_ms"] / tm["rank_launches"])
        main_roof["launches_per_step"] = tm["rank_launches"] // calls
        main_roof["entries_per_step"] = tm["rank_entries"] // calls
        main_roof["heads_per_step"] = tm["rank_heads"] // calls
    else:
        main_roof = grad_roof
    stages = {k.replace("_ms", ""): round(v / calls, 3) for k, v in tm.items() if k.endswith("_ms") and k != "rank_ms"}
    ctx.set_timing(False)
    copy_gbs = copy_bandwidth(torch)
    for roof in (main_roof, crit_roof):
        roof["copy_gbs"] = round(copy_gbs, 1)
        roof["frac_of_copy"] = round(roof["achieved"] / copy_gbs, 4)
    log(f"device copy bandwidth {copy_gbs:.0f} GB/s")
    transfers = transfer_bench(ctx, f, torch, msc) if args.transfers else None
    ooc = None
    if args.extras:
        log("out-of-core run of the same field from host memory")
        ooc = out_of_core_bench(ctx, f, torch, msc)
        if ooc["critical_counts"] != counts:
            raise SystemExit(f"out-of-core counts {ooc['critical_counts']} differ from the in-HBM run's {counts}")
    out = {
        "metric": "MS-complex Mvoxels/s at 512^3 (plain vs batched), %HBM peak; p50/p99 latency",
        "value": round(value, 2),
        "unit": "Mvoxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64",
        "data": "synthetic",
        "config": {"workload": desc, "method": "plain (one field per call)", "voxels": n,
                   "critical_counts": counts},
        "roofline": main_roof,
        "roofline_gradient": grad_roof,
        "roofline_critical": crit_roof,
        "stages_ms": stages,
        "instrumented": {"steps": prof_steps, "ms_per_step": round(instrumented_ms, 3),
                         "note": "stages_ms and the rooflines' durations come from these steps, run with event "
                                 "timing after the timed ones"},
        "stats": stats,
        "launch_params": tuned,
    }
    if transfers:
        out["with_transfers"] = transfers
    if ooc:
        out["out_of_core"] = ooc
    ctx.close()
    del fd
    torch.cuda.empty_cache()
    if args.batch > 0:
        out["batched"] = batch_bench(args, torch, msc)
        torch.cuda.empty_cache()  # the batch's workspace goes back to the device before serving
    if args.serve_steps > 0:
        from paper_2009_03707_amd import serve
        out["served"] = serve.serve_benchmark(steps=args.serve_steps, slots=args.serve_slots, options=tuned,
                                              log=log)
        torch.cuda.empty_cache()
    if args.extras:
        log("host MS-complex graph and simplification of grf256")
        out["graph"] = graph_bench(torch, msc)
    if args.cpu_sample > 0:
        log(f"timing the oracle on a {args.cpu_sample}^3 crop")
        out["cpu_baseline"] = cpu_baseline(f, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
