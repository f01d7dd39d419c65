"""Thin Python binding of libmsc.so (include/msc.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch supplies device memory (tensors) and the stream
(``torch.cuda.current_stream()``).  If the library is not built, or there is
no GPU, calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsc.so")

MS_OK, MS_ERR_INVALID_ARG, MS_ERR_NONFINITE, MS_ERR_TOO_LARGE, MS_ERR_CAPACITY, MS_ERR_OOM, MS_ERR_HIP, \
    MS_ERR_INTERNAL = range(8)

EXPORTED = ["ms_ctx_create", "ms_ctx_destroy", "ms_ctx_set_stream", "ms_last_error", "ms_gradient",
            "ms_critical", "ms_connect", "ms_complex", "ms_ctx_set_timing", "ms_ctx_get_timing",
            "ms_ctx_set_option", "ms_complex_batch", "ms_ctx_release", "ms_critical_noalloc",
            "ms_graph_build", "ms_graph_build_host", "ms_graph_destroy", "ms_graph_num_nodes", "ms_graph_last_error",
            "ms_graph_node", "ms_graph_find", "ms_graph_arcs", "ms_graph_counts", "ms_graph_simplify",
            "ms_graph_num_cancellations", "ms_graph_cancellations", "ms_gradient_critical_chunked",
            "ms_manifolds_chunked", "ms_extremum_arcs_host", "ms_csr64_transpose_host"]
LABEL_EXIT64 = 0xFFFFFFFFFFFFFFFF
MS_DOWN, MS_UP = 0, 1
MS_SIMPLIFY_SERIAL, MS_SIMPLIFY_SUBGRID = 0, 1

(MS_OPT_PATH_SCHEDULE, MS_OPT_MERGE_LIGHT, MS_OPT_MERGE_CHUNK, MS_OPT_GRADIENT_TILE, MS_OPT_BATCH_GRAPH,
 MS_OPT_TRANSPOSE_PACK) = 1, 2, 3, 4, 5, 6
MS_PATHS_READY, MS_PATHS_POWER, MS_PATHS_ENTRY = 0, 1, 2


class MscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libmsc status {status}: {msg}")
        self.status = status


class Dims(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64)]


class Crit(C.Structure):
    _fields_ = [("id", C.c_void_p), ("index", C.c_void_p), ("value", C.c_void_p), ("vmax", C.c_void_p),
                ("capacity", C.c_int64)]


class Csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p)]


class Crit64(C.Structure):
    _fields_ = [("id", C.c_void_p), ("index", C.c_void_p), ("value", C.c_void_p), ("vmax", C.c_void_p),
                ("capacity", C.c_int64)]


class Csr64Host(C.Structure):
    _fields_ = [("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p), ("capacity", C.c_int64),
                ("nnz", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("pj_rounds_vertex", "pj_rounds_cube", "bfs_levels", "reachable",
                                         "junctions", "nnz_a", "nnz_b", "nnz_bstar", "nnz_d", "spgemm_iters",
                                         "nnz_astar", "products", "nnz_p")]


class Arcs(C.Structure):
    _fields_ = [("m10", Csr), ("m10t", Csr), ("m21", Csr), ("m21t", Csr), ("m32", Csr), ("m32t", Csr),
                ("n_saturated", C.c_int64), ("stats", Stats), ("min_label", C.c_void_p),
                ("max_label", C.c_void_p)]


class Timing(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gradient_ms", "critical_ms", "extrema_ms", "bfs_ms", "minor_ms",
                                          "paths_ms", "total_ms")] + [("calls", C.c_int64),
                                                                      ("allocations", C.c_int64),
                                                                      ("workspace_bytes", C.c_int64),
                                                                      ("rank_ms", C.c_double),
                                                                      ("rank_launches", C.c_int64),
                                                                      ("rank_entries", C.c_int64),
                                                                      ("rank_heads", C.c_int64),
                                                                      ("graph_captures", C.c_int64),
                                                                      ("graph_replays", C.c_int64),
                                                                      ("side_ms", C.c_double)]


class Result(C.Structure):
    _fields_ = [("grad", C.c_void_p), ("crit", Crit), ("count", C.c_int64 * 4), ("arcs", Arcs)]


class Node(C.Structure):
    _fields_ = [("cell", C.c_uint32), ("index", C.c_uint8), ("alive", C.c_uint8), ("value", C.c_float),
                ("vmax", C.c_uint32)]


class Cancellation(C.Structure):
    _fields_ = [("upper", C.c_int64), ("lower", C.c_int64), ("persistence", C.c_double)]


# ms_alloc_fn / ms_free_fn (include/msc.h)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


def _torch_alloc(user, nbytes, stream):
    """Workspace block from torch's caching allocator on the context's
    stream (`user` carries the device ordinal); NULL when torch cannot."""
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(user or 0), int(stream or 0))
    except Exception:  # noqa: BLE001 - any failure is reported to the library as NULL (MS_ERR_OOM)
        return None


def _torch_free(user, ptr, nbytes, stream):
    torch.cuda.caching_allocator_delete(int(ptr))


# kept alive for the life of the module: the library holds these pointers
TORCH_ALLOCATOR = (ALLOC_FN(_torch_alloc), FREE_FN(_torch_free))

_LIB = None


def lib():
    """Loads libmsc.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.ms_ctx_create.argtypes = [C.POINTER(vp), vp, ALLOC_FN, FREE_FN, vp]
        L.ms_ctx_destroy.argtypes = [vp]
        L.ms_ctx_destroy.restype = None
        L.ms_ctx_set_stream.argtypes = [vp, vp]
        L.ms_last_error.argtypes = [vp]
        L.ms_last_error.restype = C.c_char_p
        L.ms_gradient.argtypes = [vp, vp, Dims, vp]
        L.ms_critical.argtypes = [vp, vp, vp, Dims, C.POINTER(Crit), C.POINTER(i64)]
        L.ms_critical_noalloc.argtypes = [vp, vp, vp, Dims, C.POINTER(Crit), C.POINTER(i64)]
        L.ms_connect.argtypes = [vp, vp, Dims, vp, C.POINTER(i64), C.POINTER(Arcs)]
        L.ms_complex.argtypes = [vp, vp, Dims, C.POINTER(Result)]
        L.ms_ctx_set_timing.argtypes = [vp, C.c_int]
        L.ms_ctx_get_timing.argtypes = [vp, C.POINTER(Timing)]
        L.ms_ctx_set_option.argtypes = [vp, C.c_int, C.c_int64]
        L.ms_complex_batch.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(Dims), C.POINTER(Result)]
        L.ms_ctx_release.argtypes = [vp]
        L.ms_gradient_critical_chunked.argtypes = [vp, vp, Dims, i64, vp, C.POINTER(Crit64), C.POINTER(i64)]
        L.ms_manifolds_chunked.argtypes = [vp, vp, Dims, i64, vp, vp, C.POINTER(i64)]
        L.ms_extremum_arcs_host.argtypes = [Dims, vp, vp, vp, i64, vp, i64, C.POINTER(Csr64Host),
                                            C.POINTER(Csr64Host)]
        L.ms_csr64_transpose_host.argtypes = [C.POINTER(Csr64Host), i64, i64, C.POINTER(Csr64Host)]
        L.ms_graph_build.argtypes = [vp, C.POINTER(Result), Dims, C.c_int, C.POINTER(vp)]
        L.ms_graph_build_host.argtypes = [C.POINTER(Result), Dims, C.c_int, C.POINTER(vp)]
        L.ms_graph_destroy.argtypes = [vp]
        L.ms_graph_destroy.restype = None
        L.ms_graph_num_nodes.argtypes = [vp]
        L.ms_graph_num_nodes.restype = i64
        L.ms_graph_last_error.argtypes = [vp]
        L.ms_graph_last_error.restype = C.c_char_p
        L.ms_graph_node.argtypes = [vp, i64, C.POINTER(Node)]
        L.ms_graph_find.argtypes = [vp, C.c_uint32, C.POINTER(i64)]
        L.ms_graph_arcs.argtypes = [vp, i64, C.c_int, vp, vp, i64, C.POINTER(i64)]
        L.ms_graph_counts.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.ms_graph_simplify.argtypes = [vp, C.c_double, C.c_int, C.c_int, C.POINTER(i64)]
        L.ms_graph_num_cancellations.argtypes = [vp]
        L.ms_graph_num_cancellations.restype = i64
        L.ms_graph_cancellations.argtypes = [vp, i64, i64, C.POINTER(Cancellation)]
        for n in EXPORTED:
            getattr(L, n)
        _LIB = L
    return _LIB


_hip = None


def extremum_arcs_host(dims, min_label, max_label, s1_id, s2_id):
    """ms_extremum_arcs_host: (M10, M32^T) of a field from its 64-bit labels
    (host numpy, e.g. Context.manifolds_chunked) and its 1- and 2-saddle
    ids (host numpy uint64, e.g. from Context.gradient_critical_chunked);
    each matrix as (rowptr int64, col uint64, val uint64).  dims = (nx, ny,
    nz)."""
    import numpy as np
    out = []
    mats = []
    keep = []
    for ids, lab in ((s1_id, min_label), (s2_id, max_label)):
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        lab = np.ascontiguousarray(lab, dtype=np.uint64)
        cap = max(2 * len(ids), 1)
        arrs = (np.zeros(len(ids) + 1, np.int64), np.empty(cap, np.uint64), np.empty(cap, np.uint64))
        keep.append((ids, lab))
        mats.append(Csr64Host(arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data, cap, 0))
        out.append(arrs)
    (i1, l1), (i2, l2) = keep
    st = lib().ms_extremum_arcs_host(Dims(*[int(x) for x in dims]), l1.ctypes.data, l2.ctypes.data,
                                     i1.ctypes.data, len(i1), i2.ctypes.data, len(i2), C.byref(mats[0]),
                                     C.byref(mats[1]))
    if st != MS_OK:
        raise MscError(st, "ms_extremum_arcs_host")
    return tuple((rp, col[:m.nnz], val[:m.nnz]) for (rp, col, val), m in zip(out, mats))


def csr64_transpose_host(csr, ncols: int):
    """ms_csr64_transpose_host of a host CSR (rowptr int64, col uint64, val
    uint64) with `ncols` columns; returns the transpose in the same form."""
    import numpy as np
    rp, col, val = (np.ascontiguousarray(csr[0], np.int64), np.ascontiguousarray(csr[1], np.uint64),
                    np.ascontiguousarray(csr[2], np.uint64))
    nnz = int(rp[-1])
    out = (np.zeros(int(ncols) + 1, np.int64), np.empty(max(nnz, 1), np.uint64), np.empty(max(nnz, 1), np.uint64))
    src = Csr64Host(rp.ctypes.data, col.ctypes.data, val.ctypes.data, len(col), nnz)
    dst = Csr64Host(out[0].ctypes.data, out[1].ctypes.data, out[2].ctypes.data, max(nnz, 1), 0)
    st = lib().ms_csr64_transpose_host(C.byref(src), len(rp) - 1, int(ncols), C.byref(dst))
    if st != MS_OK:
        raise MscError(st, "ms_csr64_transpose_host")
    return out[0], out[1][:nnz], out[2][:nnz]


def _hip_rt():
    global _hip
    if _hip is None:
        h = C.CDLL("libamdhip64.so")
        h.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        h.hipMemcpyAsync.restype = C.c_int
        _hip = h
    return _hip


def _dims(f: torch.Tensor) -> Dims:
    if f.dim() != 3:
        raise ValueError("field must be a 3D tensor of shape (nz, ny, nx)")
    nz, ny, nx = f.shape
    return Dims(nx, ny, nz)


def _check_field(f: torch.Tensor):
    if not f.is_cuda or f.dtype != torch.float32 or not f.is_contiguous():
        raise ValueError("field must be a contiguous float32 CUDA/HIP tensor")


def _stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One ms_ctx bound to the current torch stream of the current device.

    allocator: "torch" (default) takes the workspace from torch's caching
    allocator; "hip" lets the library call hipMalloc / hipFree; or a pair
    (alloc, free) of ALLOC_FN / FREE_FN callbacks, which the caller keeps
    alive, with `user` passed through to them."""

    def __init__(self, allocator="torch", user=None):
        self._h = C.c_void_p()
        if allocator == "torch":
            fns, user = TORCH_ALLOCATOR, torch.cuda.current_device()
        elif allocator == "hip":
            fns = (ALLOC_FN(), FREE_FN())
        else:
            fns = allocator
        self._fns = fns
        st = lib().ms_ctx_create(C.byref(self._h), _stream_handle(), fns[0], fns[1],
                                 C.c_void_p(user) if user else None)
        if st != MS_OK:
            raise MscError(st, "ms_ctx_create failed")

    def close(self):
        if self._h:
            lib().ms_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        lib().ms_ctx_set_stream(self._h, _stream_handle())

    def _raise(self, st, what):
        if st != MS_OK:
            msg = lib().ms_last_error(self._h)
            raise MscError(st, f"{what}: {msg.decode() if msg else ''}")

    def set_path_schedule(self, schedule: int):
        """MS_PATHS_READY (default), MS_PATHS_POWER (the paper's iteration) or
        MS_PATHS_ENTRY (ready frontier with entry-parallel merges)."""
        self._raise(lib().ms_ctx_set_option(self._h, MS_OPT_PATH_SCHEDULE, int(schedule)), "ms_ctx_set_option")

    def release(self):
        """Frees the context's workspace (outputs of earlier calls become invalid)."""
        self._raise(lib().ms_ctx_release(self._h), "ms_ctx_release")

    def set_option(self, option: int, value: int):
        self._raise(lib().ms_ctx_set_option(self._h, int(option), int(value)), "ms_ctx_set_option")

    def set_timing(self, on: bool):
        self._raise(lib().ms_ctx_set_timing(self._h, 1 if on else 0), "ms_ctx_set_timing")

    def timing(self) -> dict:
        t = Timing()
        self._raise(lib().ms_ctx_get_timing(self._h, C.byref(t)), "ms_ctx_get_timing")
        return {k: getattr(t, k) for k, _ in Timing._fields_}

    # -- entry points -------------------------------------------------------
    def gradient(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_field(f)
        self._sync_stream()
        g = out if out is not None else torch.empty(f.shape, dtype=torch.int32, device=f.device)
        st = lib().ms_gradient(self._h, C.c_void_p(f.data_ptr()), _dims(f), C.c_void_p(g.data_ptr()))
        self._raise(st, "ms_gradient")
        return g

    def critical(self, f: torch.Tensor, grad: torch.Tensor):
        """Returns (id int32[N], index uint8[N], value float32[N], vmax int32[N],
        counts list[4]); ids and vertex ids are uint32 values stored in int32."""
        _check_field(f)
        self._sync_stream()
        cnt = (C.c_int64 * 4)()
        st = lib().ms_critical(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(grad.data_ptr()), _dims(f), None, cnt)
        self._raise(st, "ms_critical (count)")
        n = sum(cnt)
        dev = f.device
        ids = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        idx = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
        val = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
        vm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        cr = Crit(ids.data_ptr(), idx.data_ptr(), val.data_ptr(), vm.data_ptr(), n)
        st = lib().ms_critical(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(grad.data_ptr()), _dims(f),
                               C.byref(cr), cnt)
        self._raise(st, "ms_critical")
        return ids[:n], idx[:n], val[:n], vm[:n], list(cnt)

    def critical_noalloc(self, f: torch.Tensor, grad: torch.Tensor, out=None):
        """ms_critical_noalloc: the library allocates no device memory (its
        scratch is a fixed per-GPU array).  `out` = (id, index, value, vmax)
        tensors to fill (capacity = the shortest), or None to query the counts
        only.  Returns the counts per index; raises MscError (MS_ERR_CAPACITY,
        MS_ERR_TOO_LARGE, ...) like the library."""
        _check_field(f)
        self._sync_stream()
        cnt = (C.c_int64 * 4)()
        cr = None
        if out is not None:
            cap = min(int(t.numel()) for t in out)
            cr = C.byref(Crit(out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), out[3].data_ptr(), cap))
        st = lib().ms_critical_noalloc(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(grad.data_ptr()), _dims(f),
                                       cr, cnt)
        self._raise(st, "ms_critical_noalloc")
        return list(cnt)

    def gradient_critical_chunked(self, f, slab: int, want_grad: bool = True):
        """ms_gradient_critical_chunked on a host numpy float32 field (nz, ny,
        nx): returns (grad uint32 (nz, ny, nx) or None, id uint64[], index
        uint8[], value float32[], vmax uint64[], counts)."""
        import numpy as np
        f = np.ascontiguousarray(f, dtype=np.float32)
        nz, ny, nx = f.shape
        self._sync_stream()
        cnt = (C.c_int64 * 4)()
        grad = np.empty(f.shape, np.uint32) if want_grad else None
        gp = grad.ctypes.data if want_grad else None
        # room for one record per vertex first (only the pages written are
        # touched); a denser field reports its counts and is run again
        cap = max(int(f.size), 1)
        for attempt in range(2):
            arrs = (np.empty(cap, np.uint64), np.empty(cap, np.uint8), np.empty(cap, np.float32),
                    np.empty(cap, np.uint64))
            cr = Crit64(*[a.ctypes.data for a in arrs], cap)
            st = lib().ms_gradient_critical_chunked(self._h, f.ctypes.data, Dims(nx, ny, nz), int(slab), gp,
                                                    C.byref(cr), cnt)
            if st != MS_ERR_CAPACITY or attempt:
                break
            cap = max(int(sum(cnt)), 1)
        self._raise(st, "ms_gradient_critical_chunked")
        n = int(sum(cnt))
        return (grad,) + tuple(a[:n] for a in arrs) + (list(cnt),)

    def manifolds_chunked(self, f, slab: int, want_min: bool = True, want_max: bool = True):
        """ms_manifolds_chunked on a host numpy float32 field (nz, ny, nx):
        returns (min_label uint64 (nz, ny, nx) or None, max_label uint64
        (nz, ny, nx) or None, counts)."""
        import numpy as np
        f = np.ascontiguousarray(f, dtype=np.float32)
        nz, ny, nx = f.shape
        self._sync_stream()
        cnt = (C.c_int64 * 4)()
        lo = np.empty(f.shape, np.uint64) if want_min else None
        hi = np.empty(f.shape, np.uint64) if want_max else None
        st = lib().ms_manifolds_chunked(self._h, f.ctypes.data, Dims(nx, ny, nz), int(slab),
                                        lo.ctypes.data if want_min else None, hi.ctypes.data if want_max else None,
                                        cnt)
        self._raise(st, "ms_manifolds_chunked")
        return lo, hi, list(cnt)

    def connect(self, grad: torch.Tensor, dims, crit_id: torch.Tensor, counts) -> "Arcs":
        self._sync_stream()
        cnt = (C.c_int64 * 4)(*[int(c) for c in counts])
        arcs = Arcs()
        st = lib().ms_connect(self._h, C.c_void_p(grad.data_ptr()), Dims(*dims),
                              C.c_void_p(crit_id.data_ptr() if crit_id.numel() else 0), cnt, C.byref(arcs))
        self._raise(st, "ms_connect")
        return arcs

    def complex_batch_raw(self, fs):
        """ms_complex_batch over a list of field tensors; returns one Result
        per field, pointing at context-owned buffers valid until the next
        call on this context."""
        for f in fs:
            _check_field(f)
        self._sync_stream()
        n = len(fs)
        ptrs = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
        dims = (Dims * n)(*[_dims(f) for f in fs])
        res = (Result * n)()
        st = lib().ms_complex_batch(self._h, n, ptrs, dims, res)
        self._raise(st, "ms_complex_batch")
        return list(res)

    def complex_raw(self, f: torch.Tensor) -> Result:
        """ms_complex; the returned structure points at context-owned device
        buffers valid until the next call on this context."""
        _check_field(f)
        self._sync_stream()
        res = Result()
        st = lib().ms_complex(self._h, C.c_void_p(f.data_ptr()), _dims(f), C.byref(res))
        self._raise(st, "ms_complex")
        return res


# -- copying context-owned outputs into torch tensors ---------------------------

def _copy_dev(ptr: int, nbytes: int, dtype, count: int, device) -> torch.Tensor:
    t = torch.empty(max(count, 1), dtype=dtype, device=device)
    if nbytes > 0:
        rc = _hip_rt().hipMemcpyAsync(C.c_void_p(t.data_ptr()), C.c_void_p(ptr), nbytes, 3, _stream_handle())
        if rc != 0:
            raise MscError(MS_ERR_HIP, f"hipMemcpyAsync failed ({rc})")
    return t[:count]


@dataclass
class CsrT:
    nrows: int
    ncols: int
    rowptr: torch.Tensor  # int64[nrows+1]
    col: torch.Tensor     # int32 (uint32 values)
    val: torch.Tensor     # int64 (uint64 bit patterns)


def csr_to_torch(m: Csr, device) -> CsrT:
    rp = _copy_dev(m.rowptr or 0, 8 * (m.nrows + 1) if m.rowptr else 0, torch.int64, m.nrows + 1, device)
    if not m.rowptr:
        rp.zero_()
    col = _copy_dev(m.col or 0, 4 * m.nnz, torch.int32, m.nnz, device)
    val = _copy_dev(m.val or 0, 8 * m.nnz, torch.int64, m.nnz, device)
    return CsrT(m.nrows, m.ncols, rp, col, val)


@dataclass
class Complex:
    grad: torch.Tensor
    crit_id: torch.Tensor
    crit_index: torch.Tensor
    crit_value: torch.Tensor
    crit_vmax: torch.Tensor
    count: list
    m10: CsrT
    m10t: CsrT
    m21: CsrT
    m21t: CsrT
    m32: CsrT
    m32t: CsrT
    n_saturated: int
    stats: dict
    min_label: torch.Tensor  # int32 (uint32 values), shape of the field: rank of each vertex's minimum
    max_label: torch.Tensor  # int32 (uint32 values): rank of the maximum of the cube at each lowest corner,
    #                          0xFFFFFFFF (-1) when there is none or its path leaves the grid


def _to_complex(r: Result, f: torch.Tensor) -> Complex:
    dev = f.device
    n = sum(r.count)
    nv = f.numel()
    return Complex(
        grad=_copy_dev(r.grad, 4 * nv, torch.int32, nv, dev).view(f.shape),
        crit_id=_copy_dev(r.crit.id, 4 * n, torch.int32, n, dev),
        crit_index=_copy_dev(r.crit.index, n, torch.uint8, n, dev),
        crit_value=_copy_dev(r.crit.value, 4 * n, torch.float32, n, dev),
        crit_vmax=_copy_dev(r.crit.vmax, 4 * n, torch.int32, n, dev),
        count=list(r.count),
        m10=csr_to_torch(r.arcs.m10, dev), m10t=csr_to_torch(r.arcs.m10t, dev),
        m21=csr_to_torch(r.arcs.m21, dev), m21t=csr_to_torch(r.arcs.m21t, dev),
        m32=csr_to_torch(r.arcs.m32, dev), m32t=csr_to_torch(r.arcs.m32t, dev),
        n_saturated=int(r.arcs.n_saturated),
        stats={k: int(getattr(r.arcs.stats, k)) for k, _ in Stats._fields_},
        min_label=_copy_dev(r.arcs.min_label or 0, 4 * nv if r.arcs.min_label else 0, torch.int32, nv,
                            dev).view(f.shape),
        max_label=_copy_dev(r.arcs.max_label or 0, 4 * nv if r.arcs.max_label else 0, torch.int32, nv,
                            dev).view(f.shape),
    )


def complex_(f: torch.Tensor, ctx: Context | None = None) -> Complex:
    """Runs the whole hot path and copies the results into torch tensors."""
    own = ctx is None
    ctx = ctx or Context()
    try:
        out = _to_complex(ctx.complex_raw(f), f)
        torch.cuda.current_stream().synchronize()
        return out
    finally:
        if own:
            ctx.close()


def complex_batch(fs, ctx: Context | None = None):
    """Runs ms_complex_batch (one launch per phase for all fields) and copies
    each field's result into torch tensors."""
    own = ctx is None
    ctx = ctx or Context()
    try:
        rs = ctx.complex_batch_raw(fs)
        out = [_to_complex(r, f) for r, f in zip(rs, fs)]
        torch.cuda.current_stream().synchronize()
        return out
    finally:
        if own:
            ctx.close()


# -- host MS-complex graph and simplification ----------------------------------

class Graph:
    """ms_graph: the 1-skeleton as a host graph (nodes = critical points in
    the order of the critical list, arcs in both directions with
    multiplicities) and its persistence-driven simplification."""

    def __init__(self, handle):
        self._h = handle

    @classmethod
    def from_result(cls, ctx: "Context", result: Result, dims, nthreads: int = 8) -> "Graph":
        """From a (device) result of ms_complex / ms_complex_batch; dims =
        (nx, ny, nz) of the field."""
        h = C.c_void_p()
        ctx._sync_stream()
        st = lib().ms_graph_build(ctx._h, C.byref(result), Dims(*dims), int(nthreads), C.byref(h))
        ctx._raise(st, "ms_graph_build")
        return cls(h)

    @classmethod
    def from_host(cls, result: Result, dims, nthreads: int = 8) -> "Graph":
        """From a result whose critical list and CSR arrays are host memory."""
        h = C.c_void_p()
        st = lib().ms_graph_build_host(C.byref(result), Dims(*dims), int(nthreads), C.byref(h))
        if st != MS_OK:
            raise MscError(st, "ms_graph_build_host")
        return cls(h)

    def close(self):
        if self._h:
            lib().ms_graph_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ok(self, st, what):
        if st != MS_OK:
            msg = lib().ms_graph_last_error(self._h)
            raise MscError(st, f"{what}: {msg.decode() if msg else ''}")

    def num_nodes(self) -> int:
        return int(lib().ms_graph_num_nodes(self._h))

    def node(self, i: int) -> dict:
        n = Node()
        self._ok(lib().ms_graph_node(self._h, int(i), C.byref(n)), "ms_graph_node")
        return {k: getattr(n, k) for k, _ in Node._fields_}

    def find(self, cell: int) -> int:
        out = C.c_int64()
        self._ok(lib().ms_graph_find(self._h, int(cell), C.byref(out)), "ms_graph_find")
        return out.value

    def arcs(self, i: int, direction: int):
        """(neighbour nodes int64[], multiplicities uint64[]) of a node."""
        import numpy as np
        cnt = C.c_int64()
        st = lib().ms_graph_arcs(self._h, int(i), int(direction), None, None, 0, C.byref(cnt))
        if st not in (MS_OK, MS_ERR_CAPACITY):
            self._ok(st, "ms_graph_arcs")
        n = cnt.value
        nbr = np.zeros(max(n, 1), np.int64)
        mult = np.zeros(max(n, 1), np.uint64)
        self._ok(lib().ms_graph_arcs(self._h, int(i), int(direction), nbr.ctypes.data, mult.ctypes.data, n,
                                     C.byref(cnt)), "ms_graph_arcs")
        return nbr[:n], mult[:n]

    def counts(self):
        alive = (C.c_int64 * 4)()
        arcs = (C.c_int64 * 3)()
        self._ok(lib().ms_graph_counts(self._h, alive, arcs), "ms_graph_counts")
        return list(alive), list(arcs)

    def simplify(self, threshold: float, schedule: int = MS_SIMPLIFY_SERIAL, nthreads: int = 1) -> int:
        n = C.c_int64()
        self._ok(lib().ms_graph_simplify(self._h, float(threshold), int(schedule), int(nthreads), C.byref(n)),
                 "ms_graph_simplify")
        return n.value

    def cancellations(self):
        """[(upper, lower, persistence)] in the order they were made."""
        n = int(lib().ms_graph_num_cancellations(self._h))
        buf = (Cancellation * max(n, 1))()
        self._ok(lib().ms_graph_cancellations(self._h, 0, n, buf), "ms_graph_cancellations")
        return [(buf[i].upper, buf[i].lower, buf[i].persistence) for i in range(n)]
