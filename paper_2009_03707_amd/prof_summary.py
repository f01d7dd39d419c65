"""Summarise rocprofv3 output into short per-kernel tables.

Kernel trace (rocpd SQLite, written by
`rocprofv3 --kernel-trace --stats -d DIR -o run -- <command>`): calls, total
ms, average us, share of GPU kernel time.

    python -m paper_2009_03707_amd.prof_summary DIR/run_results.db [N]

Counters (CSV, written by `rocprofv3 --pmc C1 C2 ... --output-format csv -d
DIR -o run -- <command>`): per kernel and counter, the dispatch count and the
mean value per dispatch.  With --copy-bytes B, the kernel whose name contains
"copy" is taken as a plain copy of B bytes read and B bytes written, and each
counter's bytes-per-KiB scale factor (B / (1024 * mean)) is printed.

    python -m paper_2009_03707_amd.prof_summary DIR/run_counter_collection.csv [N] [--copy-bytes B]

Traffic of one kernel (per launch, in bytes) from a FETCH_SIZE run and a
WRITE_SIZE run of the same command, each scaled by what the counter reads
for the run's first plain copy dispatch of B bytes (bench.py
--calibrate-copy issues it before anything else); the kernel's source file
is hashed so that a later change of the kernel invalidates the figure.

    python -m paper_2009_03707_amd.prof_summary traffic FETCH.csv WRITE.csv KERNEL SOURCE B

VALU counters of one kernel per launch (SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU,
SQ_THREAD_CYCLES_VALU, SQ_BUSY_CU_CYCLES, GRBM_GUI_ACTIVE in one --pmc run),
with the kernel's source hash:

    python -m paper_2009_03707_amd.prof_summary valu COUNTERS.csv KERNEL SOURCE

SQ instruction counters of one kernel per launch (SQ_INSTS_VALU,
SQ_INSTS_SALU, SQ_WAVE_CYCLES, SQ_BUSY_CYCLES in one --pmc run), with the
instructions per 64 entries when the entries per launch are given:

    python -m paper_2009_03707_amd.prof_summary sq COUNTERS.csv KERNEL SOURCE [ENTRIES]
"""
import collections
import csv
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = name.replace("msc::(anonymous namespace)::", "").replace("void ", "")
    depth, out = 0, []
    for ch in name:  # drop the argument list, keep template arguments
        if ch == "(":
            depth += 1
        if depth == 0:
            out.append(ch)
        if ch == ")":
            depth -= 1
    return re.sub(r"\s+", " ", "".join(out)).strip()


def counters(path, n, copy_bytes):
    acc = collections.defaultdict(lambda: [0, 0.0])
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            key = (short(row["Kernel_Name"]), row["Counter_Name"])
            acc[key][0] += 1
            acc[key][1] += float(row["Counter_Value"])
    rows = sorted(acc.items(), key=lambda kv: -kv[1][1])
    print(f"{'kernel':44s} {'counter':>12s} {'dispatches':>10s} {'mean/dispatch':>14s}")
    for (k, c), (cnt, tot) in rows[:n]:
        print(f"{k[:44]:44s} {c:>12s} {cnt:10d} {tot / cnt:14.1f}")
    if copy_bytes:
        for (k, c), (cnt, tot) in rows:
            if "copy" in k.lower():
                mean = tot / cnt
                print(f"copy calibration: {k[:44]} {c} mean {mean:.1f} per dispatch for {copy_bytes} B "
                      f"-> {copy_bytes / (1024.0 * mean):.4f} bytes per counted KiB / 1024")


def _dispatches(path, counter):
    with open(path, newline="") as fh:
        rows = [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def traffic(fetch_csv, write_csv, kernel, source, copy_bytes):
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    src = hashlib.sha256(open(os.path.join(here, "csrc", source), "rb").read()).hexdigest()
    out = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = _dispatches(path, name)
        cal = next(r for r in rows if "copyBuffer" in r["Kernel_Name"])
        factor = copy_bytes / (1024.0 * float(cal["Counter_Value"]))  # bytes per counted byte
        ks = [float(r["Counter_Value"]) for r in rows if short(r["Kernel_Name"]).startswith(kernel)]
        out[name] = (factor, float(cal["Counter_Value"]), len(ks), sum(ks) * 1024.0 * factor / max(len(ks), 1))
    f_fac, f_cal, n, f_b = out["FETCH_SIZE"]
    w_fac, w_cal, _, w_b = out["WRITE_SIZE"]
    print(f"# {kernel}: HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch)")
    print(f"# calibration: first plain copy of {copy_bytes} B reads FETCH_SIZE {f_cal:.1f} KiB "
          f"(x{f_fac:.4f}) and WRITE_SIZE {w_cal:.1f} KiB (x{w_fac:.4f})")
    print(f"kernel: {kernel}")
    print(f"source: {source}")
    print(f"source_sha256: {src}")
    print(f"launches: {n}")
    print(f"fetch_bytes_per_launch: {int(f_b)}")
    print(f"write_bytes_per_launch: {int(w_b)}")
    print(f"traffic_bytes_per_launch: {int(f_b + w_b)}")


def valu(csv_path, kernel, source, cus=256):
    """VALU counters of one kernel per launch, from a --pmc run with
    SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_THREAD_CYCLES_VALU,
    SQ_BUSY_CU_CYCLES and GRBM_GUI_ACTIVE (each summed over the shader
    engines / dies by rocprofv3)."""
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    src = hashlib.sha256(open(os.path.join(here, "csrc", source), "rb").read()).hexdigest()
    acc = collections.defaultdict(float)
    disp = set()
    with open(csv_path, newline="") as fh:
        for row in csv.DictReader(fh):
            if not short(row["Kernel_Name"]).startswith(kernel):
                continue
            disp.add(row["Dispatch_Id"])
            acc[row["Counter_Name"]] += float(row["Counter_Value"])
    n = max(len(disp), 1)
    per = {k: v / n for k, v in acc.items()}
    print(f"# {kernel}: VALU counters per launch (rocprofv3 --pmc, summed over shader engines and dies)")
    print("# valu_busy_pct follows rocprofv3's VALUBusy: 100 * SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE, with"
          " GRBM_GUI_ACTIVE taken per die (summed value / 8)")
    print(f"kernel: {kernel}")
    print(f"source: {source}")
    print(f"source_sha256: {src}")
    print(f"launches: {len(disp)}")
    print(f"valu_insts_per_launch: {per.get('SQ_INSTS_VALU', 0):.0f}")
    print(f"active_inst_valu_per_launch: {per.get('SQ_ACTIVE_INST_VALU', 0):.0f}")
    print(f"thread_cycles_valu_per_launch: {per.get('SQ_THREAD_CYCLES_VALU', 0):.0f}")
    print(f"busy_cu_cycles_per_launch: {per.get('SQ_BUSY_CU_CYCLES', 0):.0f}")
    print(f"gui_active_per_launch: {per.get('GRBM_GUI_ACTIVE', 0):.0f}")
    gui = per.get("GRBM_GUI_ACTIVE", 0) / 8.0
    if gui > 0:
        print(f"valu_busy_pct: {100.0 * per.get('SQ_ACTIVE_INST_VALU', 0) / cus / gui:.2f}")
    if per.get("SQ_ACTIVE_INST_VALU", 0) > 0:
        print(f"lanes_per_valu_inst: {per.get('SQ_THREAD_CYCLES_VALU', 0) / per['SQ_ACTIVE_INST_VALU']:.2f}")


def sq(csv_path, kernel, source, entries_per_launch=0):
    """SQ instruction and cycle counters of one kernel per launch, from a
    --pmc run with SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_WAVE_CYCLES and
    SQ_BUSY_CYCLES; with the entries one launch ranks, the instructions per
    64 entries (one wave's worth)."""
    import hashlib
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    src = hashlib.sha256(open(os.path.join(here, "csrc", source), "rb").read()).hexdigest()
    acc = collections.defaultdict(float)
    disp = set()
    with open(csv_path, newline="") as fh:
        for row in csv.DictReader(fh):
            if not short(row["Kernel_Name"]).startswith(kernel):
                continue
            disp.add(row["Dispatch_Id"])
            acc[row["Counter_Name"]] += float(row["Counter_Value"])
    n = max(len(disp), 1)
    per = {k: v / n for k, v in acc.items()}
    print(f"# {kernel}: SQ counters per launch, mean over the launches (summed over shader engines and dies)")
    print(f"kernel: {kernel}")
    print(f"source: {source}")
    print(f"source_sha256: {src}")
    print(f"launches: {len(disp)}")
    for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES"):
        print(f"{c.lower()}_per_launch: {per.get(c, 0):.0f}")
    if entries_per_launch:
        print(f"entries_per_launch: {entries_per_launch}")
        for c in ("SQ_INSTS_VALU", "SQ_INSTS_SALU"):
            print(f"{c[9:].lower()}_insts_per_64_entries: {64.0 * per.get(c, 0) / entries_per_launch:.1f}")


def main():
    if sys.argv[1] == "sq":
        sq(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]) if len(sys.argv) > 5 else 0)
        return
    if sys.argv[1] == "valu":
        valu(sys.argv[2], sys.argv[3], sys.argv[4])
        return
    if sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], int(sys.argv[6]))
        return
    if sys.argv[1].endswith(".csv"):
        args = [a for a in sys.argv[2:] if not a.startswith("--")]
        cb = 0
        if "--copy-bytes" in sys.argv:
            cb = int(sys.argv[sys.argv.index("--copy-bytes") + 1])
            args = [a for a in args if a != str(cb)]
        counters(sys.argv[1], int(args[0]) if args else 40, cb)
        return
    db = sys.argv[1]
    n = int(sys.argv[2]) if len(sys.argv) > 2 else 25
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    total = sum(r[2] for r in rows)
    print(f"{'kernel':44s} {'calls':>7s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
    for r in rows[:n]:
        print(f"{short(r[0])[:44]:44s} {r[1]:7d} {r[2] / 1000:10.2f} {r[3]:10.1f} {r[4]:6.1f}")
    print(f"{'(all kernels)':44s} {sum(r[1] for r in rows):7d} {total / 1000:10.2f}")


if __name__ == "__main__":
    main()
