"""Python front end of the serial CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It marshals numpy arrays into the plain C oracle (msc_oracle.c) and
assembles its outputs into simple numpy structures.  It shares no code with
the GPU library.

All outputs follow the contract conventions stated at the top of
msc_oracle.c (vertex order with id tie-break, word-major cell ids, nibble
encoding, critical list sorted by (index, id), saturating u64 path counts).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

ORC_OK, ORC_ERR_ARG, ORC_ERR_NONFINITE, ORC_ERR_OOM, ORC_ERR_INTERNAL = 0, 1, 2, 3, 4

_p = np.ctypeslib.ndpointer


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        i64 = C.c_int64
        L.orc_gradient.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, _p(np.uint32, flags="C")]
        L.orc_critical_counts.argtypes = [_p(np.uint32, flags="C"), i64, i64, i64, _p(np.int64, flags="C")]
        L.orc_critical_fill.argtypes = [_p(np.float32, flags="C"), _p(np.uint32, flags="C"), i64, i64, i64,
                                        _p(np.uint32, flags="C"), _p(np.uint8, flags="C"),
                                        _p(np.float32, flags="C"), _p(np.uint32, flags="C")]
        L.orc_se_arcs.argtypes = [_p(np.uint32, flags="C"), i64, i64, i64, _p(np.uint32, flags="C"),
                                  _p(np.int64, flags="C"),
                                  _p(np.int64, flags="C"), _p(np.int64, flags="C"), _p(np.uint64, flags="C"),
                                  C.POINTER(i64),
                                  _p(np.int64, flags="C"), _p(np.int64, flags="C"), _p(np.uint64, flags="C"),
                                  C.POINTER(i64)]
        L.orc_ss_paths.argtypes = [_p(np.uint32, flags="C"), i64, i64, i64, _p(np.uint32, flags="C"),
                                   _p(np.int64, flags="C"), C.POINTER(C.c_void_p)]
        L.orc_ss_rows_lazy.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, _p(np.int64, flags="C"), i64,
                                       C.POINTER(C.c_void_p)]
        L.orc_manifolds.argtypes = [_p(np.uint32, flags="C"), i64, i64, i64, _p(np.uint32, flags="C"),
                                    _p(np.int64, flags="C"), _p(np.uint32, flags="C"), _p(np.uint32, flags="C")]
        L.orc_coo_free.argtypes = [C.c_void_p]
        L.orc_coo_nnz.argtypes = [C.c_void_p]
        L.orc_coo_nnz.restype = i64
        L.orc_coo_copy.argtypes = [C.c_void_p, _p(np.int64, flags="C"), _p(np.int64, flags="C"),
                                   _p(np.uint64, flags="C")]
        L.orc_nibble_lazy.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, i64]
        L.orc_nibble_lazy.restype = C.c_uint32
        L.orc_m10_row_lazy.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, i64, _p(np.int64, flags="C")]
        L.orc_m32_col_lazy.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, i64, _p(np.int64, flags="C")]
        L.orc_lower_star.argtypes = [_p(np.float32, flags="C"), i64, i64, i64, i64,
                                     _p(np.int64, flags="C"), _p(np.uint32, flags="C")]
        _LIB = L
    return _LIB


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _dims(f):
    nz, ny, nx = f.shape
    return int(nx), int(ny), int(nz)


def _check(rc, what):
    if rc != ORC_OK:
        raise OracleError(rc, what)


def gradient(f: np.ndarray) -> np.ndarray:
    """Gradient words, shape (nz, ny, nx) uint32 (one word per vertex)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    g = np.zeros(f.shape, dtype=np.uint32)
    _check(lib().orc_gradient(f, *_dims(f), g), "gradient")
    return g


@dataclass
class Critical:
    id: np.ndarray      # uint32 cell ids, sorted by (index, id)
    index: np.ndarray   # uint8
    value: np.ndarray   # float32 f(highest vertex)
    vmax: np.ndarray    # uint32 id of highest vertex
    count: np.ndarray   # int64[4]

    def of_index(self, k):
        o = int(self.count[:k].sum())
        return self.id[o:o + int(self.count[k])]


def critical(f: np.ndarray, grad: np.ndarray) -> Critical:
    f = np.ascontiguousarray(f, dtype=np.float32)
    grad = np.ascontiguousarray(grad, dtype=np.uint32)
    cnt = np.zeros(4, dtype=np.int64)
    _check(lib().orc_critical_counts(grad, *_dims(f), cnt), "critical_counts")
    n = int(cnt.sum())
    ids = np.zeros(max(n, 1), np.uint32)
    idx = np.zeros(max(n, 1), np.uint8)
    val = np.zeros(max(n, 1), np.float32)
    vm = np.zeros(max(n, 1), np.uint32)
    _check(lib().orc_critical_fill(f, grad, *_dims(f), ids, idx, val, vm), "critical_fill")
    return Critical(ids[:n], idx[:n], val[:n], vm[:n], cnt)


@dataclass
class Coo:
    row: np.ndarray
    col: np.ndarray
    val: np.ndarray   # uint64 multiplicities / path counts
    shape: tuple

    def dense(self):
        d = np.zeros(self.shape, dtype=np.uint64)
        d[self.row, self.col] = self.val
        return d

    def csr(self):
        """(rowptr int64, col uint32, val uint64) -- rows ascending, columns
        ascending within a row (the COO is already sorted that way)."""
        rowptr = np.zeros(self.shape[0] + 1, dtype=np.int64)
        np.add.at(rowptr, self.row + 1, 1)
        return np.cumsum(rowptr), self.col.astype(np.uint32), self.val.astype(np.uint64)


def se_arcs(f: np.ndarray, grad: np.ndarray, crit: Critical):
    """(M10, M32): M10 rows are 1-saddle ranks and columns minimum ranks; M32
    rows are maximum ranks and columns 2-saddle ranks."""
    grad = np.ascontiguousarray(grad, dtype=np.uint32)
    cnt = crit.count.astype(np.int64)
    c1, c2 = int(cnt[1]), int(cnt[2])
    a = [np.zeros(max(2 * c1, 1), t) for t in (np.int64, np.int64, np.uint64)]
    b = [np.zeros(max(2 * c2, 1), t) for t in (np.int64, np.int64, np.uint64)]
    na, nb = C.c_int64(0), C.c_int64(0)
    ids = np.ascontiguousarray(crit.id if len(crit.id) else np.zeros(1, np.uint32))
    _check(lib().orc_se_arcs(grad, *_dims(f), ids, cnt, a[0], a[1], a[2], C.byref(na),
                             b[0], b[1], b[2], C.byref(nb)), "se_arcs")
    m10 = Coo(a[0][:na.value], a[1][:na.value], a[2][:na.value], (c1, int(cnt[0])))
    m32 = Coo(b[0][:nb.value], b[1][:nb.value], b[2][:nb.value], (int(cnt[3]), c2))
    return m10, m32


NO_LABEL = 0xFFFFFFFF


def manifolds(f: np.ndarray, grad: np.ndarray, crit: Critical):
    """(min_label, max_label), both uint32 of shape (nz, ny, nx).

    min_label[v]: rank of the minimum whose ascending manifold holds vertex v.
    max_label[w]: rank of the maximum whose descending manifold holds the cube
    with lowest corner w, or NO_LABEL (no such cube, or its path leaves the
    box)."""
    grad = np.ascontiguousarray(grad, dtype=np.uint32)
    cnt = crit.count.astype(np.int64)
    lo = np.zeros(grad.shape, np.uint32)
    hi = np.zeros(grad.shape, np.uint32)
    ids = np.ascontiguousarray(crit.id if len(crit.id) else np.zeros(1, np.uint32))
    _check(lib().orc_manifolds(grad, *_dims(grad), ids, cnt, lo, hi), "manifolds")
    return lo, hi


def _take_coo(h, shape):
    L = lib()
    n = L.orc_coo_nnz(h)
    r = np.zeros(max(n, 1), np.int64)
    c = np.zeros(max(n, 1), np.int64)
    v = np.zeros(max(n, 1), np.uint64)
    L.orc_coo_copy(h, r, c, v)
    L.orc_coo_free(h)
    return Coo(r[:n], c[:n], v[:n], shape)


def ss_paths(f: np.ndarray, grad: np.ndarray, crit: Critical) -> Coo:
    """P: rows 1-saddle ranks, columns 2-saddle ranks, values = number of
    gradient paths (saturating at 2^64-1)."""
    grad = np.ascontiguousarray(grad, dtype=np.uint32)
    cnt = crit.count.astype(np.int64)
    h = C.c_void_p()
    ids = np.ascontiguousarray(crit.id if len(crit.id) else np.zeros(1, np.uint32))
    _check(lib().orc_ss_paths(grad, *_dims(f), ids, cnt, C.byref(h)), "ss_paths")
    return _take_coo(h, (int(cnt[1]), int(cnt[2])))


@dataclass
class Complex:
    grad: np.ndarray
    crit: Critical
    m10: Coo
    m32: Coo
    p: Coo           # 1-saddle x 2-saddle path counts; M21 is its transpose
    min_label: np.ndarray = None   # ascending manifolds of minima (per vertex)
    max_label: np.ndarray = None   # descending manifolds of maxima (per cube)


def complex_(f: np.ndarray, labels: bool = True) -> Complex:
    g = gradient(f)
    cr = critical(f, g)
    m10, m32 = se_arcs(f, g, cr)
    p = ss_paths(f, g, cr)
    lo, hi = manifolds(f, g, cr) if labels else (None, None)
    return Complex(g, cr, m10, m32, p, lo, hi)


# ---- lazy accessors (work from f alone; for sampled checks at large sizes) ----

def nibble_lazy(f: np.ndarray, cell_id: int) -> int:
    f = np.ascontiguousarray(f, dtype=np.float32)
    return int(lib().orc_nibble_lazy(f, *_dims(f), int(cell_id)))


def word_lazy(f: np.ndarray, vid: int) -> int:
    w = 0
    for k in range(8):
        w |= nibble_lazy(f, 8 * int(vid) + k) << (4 * k)
    return w


def lower_star(f: np.ndarray, vid: int):
    f = np.ascontiguousarray(f, dtype=np.float32)
    ids = np.zeros(27, np.int64)
    nib = np.zeros(27, np.uint32)
    n = lib().orc_lower_star(f, *_dims(f), int(vid), ids, nib)
    if n < 0:
        raise OracleError(n, "lower_star")
    return ids[:n], nib[:n]


def m10_row_lazy(f: np.ndarray, s1_cell: int):
    f = np.ascontiguousarray(f, dtype=np.float32)
    out = np.zeros(2, np.int64)
    _check(lib().orc_m10_row_lazy(f, *_dims(f), int(s1_cell), out), "m10_row_lazy")
    return out


def m32_col_lazy(f: np.ndarray, s2_cell: int):
    f = np.ascontiguousarray(f, dtype=np.float32)
    out = np.zeros(2, np.int64)
    _check(lib().orc_m32_col_lazy(f, *_dims(f), int(s2_cell), out), "m32_col_lazy")
    return out


def ss_rows_lazy(f: np.ndarray, s1_cells) -> Coo:
    """Path counts for the given 1-saddles; rows and columns are cell ids."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    src = np.ascontiguousarray(np.asarray(s1_cells, dtype=np.int64))
    h = C.c_void_p()
    _check(lib().orc_ss_rows_lazy(f, *_dims(f), src if len(src) else np.zeros(1, np.int64), len(src),
                                  C.byref(h)), "ss_rows_lazy")
    return _take_coo(h, (0, 0))
