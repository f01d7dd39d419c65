"""ms_extremum_arcs_host (the saddle-extremum arcs of an out-of-core field,
Section 3.5 "Saddle-Extrema arcs", assembled on the host from stitched
labels) runs without a GPU: from the oracle's labels and saddles it must
give the oracle's M10 and the transpose of its M32 entry for entry, and it
must reject ids and labels that are not those of a field of the given dims.
ms_csr64_transpose_host turns them into M10^T and M32, equal to the
oracle's."""
import numpy as np
import pytest

from forest import widen_exit
from oracle import oracle as O
from paper_2009_03707_amd import fields

FIELDS = [("rand", (1, 1, 1), 0), ("rand", (7, 1, 1), 1), ("rand", (1, 9, 4), 2), ("rand", (13, 11, 9), 3),
          ("rand", (16, 5, 23), 1), ("grf", (30, 24, 20), 4), ("blob", (40, 33, 27), 5), ("sine", 24, 0)]


def _field(kind, dims, seed):
    if kind == "rand":
        return fields.random_field(dims, seed=seed, levels=seed % 3)
    if kind == "grf":
        return fields.grf_field(dims, seed=seed)
    if kind == "sine":
        return fields.sine_field(dims)
    return fields.blob_field(dims, nblobs=6, seed=seed)


def _inputs(f):
    ref = O.complex_(f, labels=True)
    off = np.cumsum([0] + ref.crit.count.tolist())
    ids = ref.crit.id.astype(np.uint64)
    nz, ny, nx = f.shape
    return ref, (nx, ny, nz), ref.min_label.astype(np.uint64), widen_exit(ref.max_label), \
        ids[off[1]:off[2]], ids[off[2]:off[3]]


def _csr_t(coo):
    """CSR of the transpose of an oracle COO (rows ascending, columns
    ascending within a row)."""
    order = np.lexsort((coo.row, coo.col))
    rows, cols, vals = coo.col[order], coo.row[order], coo.val[order]
    rp = np.zeros(coo.shape[1] + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols.astype(np.uint64), vals.astype(np.uint64)


@pytest.fixture(scope="module")
def msc():
    from paper_2009_03707_amd import msc as m
    m.lib()
    return m


@pytest.mark.parametrize("kind,dims,seed", FIELDS)
def test_equals_oracle(msc, kind, dims, seed):
    f = _field(kind, dims, seed)
    ref, d, lo, hi, s1, s2 = _inputs(f)
    (rp1, c1, v1), (rp2, c2, v2) = msc.extremum_arcs_host(d, lo, hi, s1, s2)
    w_rp, w_c, w_v = ref.m10.csr()
    np.testing.assert_array_equal(rp1, w_rp)
    np.testing.assert_array_equal(c1, w_c.astype(np.uint64))
    np.testing.assert_array_equal(v1, w_v)
    w_rp, w_c, w_v = _csr_t(ref.m32)
    np.testing.assert_array_equal(rp2, w_rp)
    np.testing.assert_array_equal(c2, w_c)
    np.testing.assert_array_equal(v2, w_v)


@pytest.mark.parametrize("kind,dims,seed", FIELDS)
def test_transposes_equal_oracle(msc, kind, dims, seed):
    """M10^T and M32 by ms_csr64_transpose_host: the oracle's M10 transposed
    and its M32 as they are."""
    f = _field(kind, dims, seed)
    ref, d, lo, hi, s1, s2 = _inputs(f)
    m10, m32t = msc.extremum_arcs_host(d, lo, hi, s1, s2)
    cnt = ref.crit.count.tolist()
    for got, want in ((msc.csr64_transpose_host(m10, cnt[0]), _csr_t(ref.m10)),
                      (msc.csr64_transpose_host(m32t, cnt[3]), ref.m32.csr())):
        for g, w in zip(got, want):
            np.testing.assert_array_equal(g, w.astype(g.dtype))


def test_transpose_errors(msc):
    import ctypes as C
    lib = msc.lib()
    rp = np.array([0, 2, 3], np.int64)
    col = np.array([0, 4, 1], np.uint64)
    val = np.array([1, 1, 2], np.uint64)
    # column 4 beyond ncols = 3
    with pytest.raises(msc.MscError):
        msc.csr64_transpose_host((rp, col, val), 3)
    rp_t, col_t, val_t = msc.csr64_transpose_host((rp, col, val), 5)
    np.testing.assert_array_equal(rp_t, [0, 1, 2, 2, 2, 3])
    np.testing.assert_array_equal(col_t, [0, 1, 0])
    np.testing.assert_array_equal(val_t, [1, 2, 1])
    bad_rp = np.array([0, 2, 1], np.int64)
    with pytest.raises(msc.MscError):
        msc.csr64_transpose_host((bad_rp, col, val), 5)
    out_rp = np.zeros(6, np.int64)
    one = np.empty(1, np.uint64)
    src = msc.Csr64Host(rp.ctypes.data, col.ctypes.data, val.ctypes.data, 3, 3)
    dst = msc.Csr64Host(out_rp.ctypes.data, one.ctypes.data, one.ctypes.data, 1, 0)
    assert lib.ms_csr64_transpose_host(C.byref(src), 2, 5, C.byref(dst)) == msc.MS_ERR_CAPACITY and dst.nnz == 3
    assert lib.ms_csr64_transpose_host(None, 2, 5, C.byref(dst)) == msc.MS_ERR_INVALID_ARG


def test_errors(msc):
    import ctypes as C
    f = _field("grf", (30, 24, 20), 4)
    ref, d, lo, hi, s1, s2 = _inputs(f)
    assert len(s1) and len(s2)
    bad = s1.copy()
    bad[0] = s2[0]  # a quad among the 1-saddles
    with pytest.raises(msc.MscError) as e:
        msc.extremum_arcs_host(d, lo, hi, bad, s2)
    assert e.value.status == msc.MS_ERR_INVALID_ARG
    bad = s1.copy()
    bad[-1] = np.uint64(8 * f.size + 1)  # beyond the grid
    with pytest.raises(msc.MscError):
        msc.extremum_arcs_host(d, lo, hi, bad, s2)
    lo_bad = lo.copy()
    lo_bad.reshape(-1)[int(s1[0]) >> 3] = np.uint64(0xFFFFFFFFFFFFFFFF)
    with pytest.raises(msc.MscError):
        msc.extremum_arcs_host(d, lo_bad, hi, s1, s2)
    # an edge along +x at the last x does not exist
    nx = d[0]
    edge = np.array([8 * (nx - 1) + 1], np.uint64)
    with pytest.raises(msc.MscError):
        msc.extremum_arcs_host(d, lo, hi, edge, s2[:0])
    # capacity: nnz is reported, MS_ERR_CAPACITY returned
    lib = msc.lib()
    rp = np.zeros(len(s1) + 1, np.int64)
    col = np.empty(1, np.uint64)
    val = np.empty(1, np.uint64)
    m10 = msc.Csr64Host(rp.ctypes.data, col.ctypes.data, val.ctypes.data, 1, 0)
    st = lib.ms_extremum_arcs_host(msc.Dims(*d), lo.ctypes.data, None, s1.ctypes.data, len(s1), None, 0,
                                   C.byref(m10), None)
    assert st == msc.MS_ERR_CAPACITY and m10.nnz == len(ref.m10.row)
    # null output pointer where one is asked for
    m10 = msc.Csr64Host(None, col.ctypes.data, val.ctypes.data, 1, 0)
    assert lib.ms_extremum_arcs_host(msc.Dims(*d), lo.ctypes.data, None, s1.ctypes.data, len(s1), None, 0,
                                     C.byref(m10), None) == msc.MS_ERR_INVALID_ARG
    assert lib.ms_extremum_arcs_host(msc.Dims(0, 1, 1), None, None, None, 0, None, 0, None,
                                     None) == msc.MS_ERR_INVALID_ARG


@pytest.mark.parametrize("seed", range(24))
def test_random_small_fields(msc, seed):
    """Small fields of random dims (1..12 per axis), with ties from 0..2
    quantisation levels: all four matrices equal the oracle's."""
    rng = np.random.default_rng(7000 + seed)
    dims = tuple(int(x) for x in rng.integers(1, 13, size=3))
    f = fields.random_field(dims, seed=seed, levels=seed % 3)
    ref, d, lo, hi, s1, s2 = _inputs(f)
    m10, m32t = msc.extremum_arcs_host(d, lo, hi, s1, s2)
    cnt = ref.crit.count.tolist()
    pairs = [(m10, ref.m10.csr()), (m32t, _csr_t(ref.m32)), (msc.csr64_transpose_host(m10, cnt[0]), _csr_t(ref.m10)),
             (msc.csr64_transpose_host(m32t, cnt[3]), ref.m32.csr())]
    for got, want in pairs:
        for g, w in zip(got, want):
            np.testing.assert_array_equal(g, w.astype(g.dtype))
