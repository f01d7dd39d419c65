"""Writes tests/golden/fullsize_digests.json: SHA-256 digests of every output
of the oracle on the full-size benchmark configurations.

Run on a CPU host (no GPU needed); it calls only the oracle (oracle/) and the
seeded input generators (paper_2009_03707_amd/fields.py), never the HIP path:

    python tests/golden/make_fullsize_digests.py [--workers 5] [--only NAME ...]

Cases: the 256^3 k^-3 GRF, the 512^3 blob field, all 64 fields of the
uneven batch, and of the served stream the timesteps 0, 1 and 199 of the
advected 384x384x256 GRF plus its first 20 Poisson requests.  Each case
records the input's digest (so a generator difference is told apart from a
result difference), the critical counts, matrix sizes, and the digest of the
exact bytes of every output array in the layout of include/msc.h: gradient
words (uint32), the critical list (uint32 ids, uint8 index, float32 value
bits, uint32 highest vertex), the six arc matrices as CSR (int64 rowptr,
uint32 col, uint64 val) and the two manifold label arrays (uint32).  Results
are merged into the JSON file as cases finish, so an interrupted run resumes
where it stopped.  The 512^3 case needs about 20 GB of memory and 20-30
minutes of one core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "fullsize_digests.json")

SERVE_DIMS = (384, 384, 256)
SERVE_STEPS = 200
SERVE_TIMESTEPS = (0, 1, 199)
SERVE_REQUESTS = 20


def case_names():
    names = ["grf256", "blobs512"]
    names += [f"batch64/{i}" for i in range(64)]
    names += [f"serve/timestep{t}" for t in SERVE_TIMESTEPS]
    names += [f"serve/request{i}" for i in range(SERVE_REQUESTS)]
    return names


def make_field(name: str) -> np.ndarray:
    """The input of a case, from the shared seeded generators."""
    from paper_2009_03707_amd import fields
    if name == "grf256":
        return fields.grf_field((256, 256, 256), seed=0)
    if name == "blobs512":
        return fields.blob_field((512, 512, 512), nblobs=2000, seed=0)
    if name.startswith("batch64/"):
        return fields.make_batch_field(fields.batch_specs(64)[int(name.split("/")[1])])
    if name.startswith("serve/timestep"):
        base = fields.grf_field(SERVE_DIMS, seed=0)
        return fields.advected_step(base, int(name[len("serve/timestep"):]))
    if name.startswith("serve/request"):
        i = int(name[len("serve/request"):])
        arr = fields.request_arrivals(SERVE_STEPS / 10.0)
        _, side, kind, seed = arr[i]
        return fields.make_batch_field(fields.BatchItem(dims=(side, side, side), kind=kind, seed=seed))
    raise KeyError(name)


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def csr_digests(rowptr, col, val):
    return {"rowptr": digest(rowptr.astype(np.int64)), "col": digest(col.astype(np.uint32)),
            "val": digest(val.astype(np.uint64)), "nnz": int(len(col))}


def coo_csr(row, col, val, nrows):
    """CSR of COO entries already sorted by (row, col)."""
    rowptr = np.zeros(nrows + 1, dtype=np.int64)
    np.add.at(rowptr, row.astype(np.int64) + 1, 1)
    return np.cumsum(rowptr), col, val


def coo_digests(coo):
    """Digests of the matrix and of its transpose (both canonical CSR)."""
    nr, nc = coo.shape
    a = csr_digests(*coo_csr(coo.row, coo.col, coo.val, nr))
    order = np.lexsort((coo.row, coo.col))
    t = csr_digests(*coo_csr(coo.col[order], coo.row[order], coo.val[order], nc))
    return a, t


def run_case(name: str) -> dict:
    from oracle import oracle as O
    t0 = time.perf_counter()
    f = make_field(name)
    nz, ny, nx = f.shape
    rec = {"dims": [int(nx), int(ny), int(nz)], "input": digest(f)}
    t1 = time.perf_counter()
    g = O.gradient(f)
    rec["grad"] = digest(g)
    cr = O.critical(f, g)
    rec["counts"] = [int(c) for c in cr.count]
    rec["crit"] = {"id": digest(cr.id.astype(np.uint32)), "index": digest(cr.index.astype(np.uint8)),
                   "value": digest(cr.value.astype(np.float32).view(np.uint32)),
                   "vmax": digest(cr.vmax.astype(np.uint32))}
    m10, m32 = O.se_arcs(f, g, cr)
    rec["m10"], rec["m10t"] = coo_digests(m10)
    rec["m32"], rec["m32t"] = coo_digests(m32)
    del m10, m32
    lo, hi = O.manifolds(f, g, cr)
    rec["min_label"], rec["max_label"] = digest(lo), digest(hi)
    del lo, hi
    p = O.ss_paths(f, g, cr)
    rec["m21t"], rec["m21"] = coo_digests(p)
    rec["n_saturated"] = int((p.val == np.uint64(2 ** 64 - 1)).sum())
    rec["oracle_s"] = round(time.perf_counter() - t1, 1)
    rec["total_s"] = round(time.perf_counter() - t0, 1)
    return rec


def _worker(name):
    try:
        return name, run_case(name), None
    except Exception as e:  # noqa: BLE001 - reported and the case left out
        return name, None, repr(e)


def load():
    if os.path.exists(OUT):
        with open(OUT) as fh:
            return json.load(fh)
    return {"about": "oracle output digests at the benchmark sizes (tests/golden/make_fullsize_digests.py)",
            "cases": {}}


def save(doc):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(doc, fh, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=5)
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--redo", action="store_true", help="recompute cases already in the file")
    a = ap.parse_args()
    doc = load()
    names = a.only or case_names()
    todo = [n for n in names if a.redo or n not in doc["cases"]]
    # largest first, so the long cases overlap the many short ones
    weight = {"blobs512": 0, "grf256": 2}
    todo.sort(key=lambda n: weight.get(n, 1 if n.startswith("serve/timestep") else 3))
    doc["host"] = {"cpu": platform.processor() or platform.machine(), "python": platform.python_version(),
                   "numpy": np.__version__, "logical_cpus": os.cpu_count()}
    print(f"{len(todo)} cases to run with {a.workers} workers", flush=True)
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(a.workers, maxtasksperchild=1) as pool:
        for name, rec, err in pool.imap_unordered(_worker, todo):
            if err:
                print(f"FAILED {name}: {err}", flush=True)
                continue
            doc["cases"][name] = rec
            save(doc)
            print(f"done {name} {rec['dims']} counts={rec['counts']} in {rec['total_s']} s", flush=True)


if __name__ == "__main__":
    main()
