"""Out-of-core gradient and critical cells (ms_gradient_critical_chunked).

* Small fields, many slab heights (one row up to the whole field): the
  gradient words and the critical list (ids widened to 64 bits) equal the
  oracle's on the whole field, bit for bit -- the slabs' halos make every
  lower star exact and the slabs' lists concatenate in id order.
* A field of 1024 x 1024 x 600 vertices (more than the 2^29 vertices whose
  cell ids fit the 32-bit in-HBM entry points), separable with integer
  values: its critical counts per index are the closed-form count polynomial
  prod_axes (m + M t) (m = 1D minima, M = interior 1D maxima; pinned against
  the oracle in tests/test_oracle_pins.py), its ids strictly increase, and
  each value is the field at the recorded highest vertex.
* Non-finite input and too small an output are reported (and invalid
  arguments and non-finite input to the label call).

ms_manifolds_chunked (labels stitched across slabs, Section 3.4):

* The same small fields and slab heights: both labels equal the oracle's
  (widened to 64 bits, its exit label to all ones) word for word.
* The 512^3 blobs field in slabs of 100 rows: the labels, and the
  saddle-extremum arcs ms_extremum_arcs_host assembles from them, equal
  those of ms_complex on the whole field in HBM.
* The 1024 x 1024 x 600 field above (beyond 32-bit cell ids, so no in-HBM
  run and no oracle run to compare with): the labels form the forest the
  gradient defines -- every minimum and maximum labels itself with its rank,
  every other vertex and cube carries the label of its successor along the
  path (or the exit label where the path leaves the grid) -- which
  determines them uniquely; checked on every vertex, slab by slab."""
import numpy as np
import pytest

from forest import EXIT64, check_forest, widen_exit
from oracle import oracle as O
from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = msc.Context()
    yield c
    c.close()


CASES = [("rand", (9, 8, 7), 0), ("rand", (16, 5, 23), 1), ("rand", (1, 1, 9), 2), ("rand", (13, 1, 6), 3),
         ("grf", (30, 24, 20), 4), ("blob", (40, 33, 27), 5), ("sine", 32, 0)]


def _field(kind, dims, seed):
    if kind == "rand":
        return fields.random_field(dims, seed=seed, levels=seed % 3)
    if kind == "grf":
        return fields.grf_field(dims, seed=seed)
    if kind == "blob":
        return fields.blob_field(dims, nblobs=6, seed=seed)
    return fields.sine_field(dims)


@pytest.mark.parametrize("kind,dims,seed", CASES)
def test_slabs_equal_oracle(ctx, kind, dims, seed):
    f = _field(kind, dims, seed)
    ref_g = O.gradient(f)
    ref = O.critical(f, ref_g)
    nz = f.shape[0]
    for slab in sorted({1, 2, 3, 5, max(1, nz // 2), nz}):
        grad, cid, idx, val, vmax, cnt = ctx.gradient_critical_chunked(f, slab)
        np.testing.assert_array_equal(grad, ref_g, err_msg=f"slab {slab}")
        assert cnt == ref.count.tolist(), slab
        np.testing.assert_array_equal(cid, ref.id.astype(np.uint64))
        np.testing.assert_array_equal(idx, ref.index)
        np.testing.assert_array_equal(val.view(np.uint32), ref.value.view(np.uint32))
        np.testing.assert_array_equal(vmax, ref.vmax.astype(np.uint64))


def _zigzag(n, period, phase):
    """Integer sequence with distinct neighbours and a few extrema:
    |((i + phase) mod period) - period / 2| doubled, plus one for the
    falling half, so neighbours always differ."""
    t = (np.arange(n) + phase) % period
    h = period // 2
    return np.where(t < h, 2 * (h - t) + 1, 2 * (t - h)).astype(np.float64)


def _count_poly_1d(seq):
    n = len(seq)
    m = sum(1 for i in range(n) if (i == 0 or seq[i - 1] > seq[i]) and (i == n - 1 or seq[i + 1] > seq[i]))
    M = sum(1 for i in range(1, n - 1) if seq[i - 1] < seq[i] > seq[i + 1])
    return m, M


def test_beyond_32bit_cell_ids(ctx):
    nx, ny, nz = 1024, 1024, 600
    assert nx * ny * nz > (1 << 29)
    # z minima at 160, 360, 560: the last lies beyond vertex 2^29 (cell id 2^32)
    a, b, c = _zigzag(nx, 300, 7), _zigzag(ny, 410, 100), _zigzag(nz, 200, 140)
    f = np.empty((nz, ny, nx), np.float32)
    ab = (b[:, None] + a[None, :]).astype(np.float32)
    for z in range(nz):
        np.add(ab, np.float32(c[z]), out=f[z])
    print("[chunked] field built", flush=True)
    grad, cid, idx, val, vmax, cnt = ctx.gradient_critical_chunked(f, 120, want_grad=False)
    poly = np.array([1])
    for seq in (a, b, c):
        m, M = _count_poly_1d(list(seq))
        poly = np.polymul(poly, np.array([M, m]))
    want = [int(x) for x in list(poly[::-1]) + [0] * 4][:4]
    assert cnt == want
    off = np.cumsum([0] + cnt)
    for k in range(4):
        ids = cid[off[k]:off[k + 1]]
        assert (np.diff(ids.astype(np.int64)) > 0).all()
        assert (idx[off[k]:off[k + 1]] == k).all()
        assert bin(int(ids[0]) & 7).count("1") == k if len(ids) else True
    assert int(cid.max()) >= (1 << 32)  # cells whose ids do not fit 32 bits
    flat = f.reshape(-1)
    np.testing.assert_array_equal(val, flat[vmax.astype(np.int64)])
    assert ((cid >> np.uint64(3)) <= vmax).all()


def test_errors(ctx):
    from paper_2009_03707_amd import msc
    f = fields.random_field((10, 9, 8), seed=1)
    bad = f.copy()
    bad[5, 3, 2] = np.inf
    with pytest.raises(msc.MscError) as e:
        ctx.gradient_critical_chunked(bad, 2)
    assert e.value.status == msc.MS_ERR_NONFINITE
    lib, C = msc.lib(), msc.C
    cnt = (C.c_int64 * 4)()
    out = msc.Crit64(None, None, None, None, 0)
    st = lib.ms_gradient_critical_chunked(ctx._h, f.ctypes.data, msc.Dims(10, 9, 8), 3, None, C.byref(out), cnt)
    assert st == msc.MS_ERR_CAPACITY and sum(cnt) > 0
    with pytest.raises(msc.MscError) as e:
        ctx.manifolds_chunked(bad, 2)
    assert e.value.status == msc.MS_ERR_NONFINITE
    lo = np.empty(f.shape, np.uint64)
    assert lib.ms_manifolds_chunked(ctx._h, f.ctypes.data, msc.Dims(10, 9, 0), 3, lo.ctypes.data, None,
                                    cnt) == msc.MS_ERR_INVALID_ARG
    assert lib.ms_manifolds_chunked(ctx._h, None, msc.Dims(10, 9, 8), 3, lo.ctypes.data, None,
                                    cnt) == msc.MS_ERR_INVALID_ARG
    # no label output: counts only
    cnt2 = (C.c_int64 * 4)()
    assert lib.ms_manifolds_chunked(ctx._h, f.ctypes.data, msc.Dims(10, 9, 8), 3, None, None, cnt2) == msc.MS_OK
    assert list(cnt2) == O.critical(f, O.gradient(f)).count.tolist()
    # the context still works after the errors
    lo, hi, _ = ctx.manifolds_chunked(f, 3)
    ref_g = O.gradient(f)
    want_lo, want_hi = O.manifolds(f, ref_g, O.critical(f, ref_g))
    np.testing.assert_array_equal(lo, want_lo.astype(np.uint64))
    np.testing.assert_array_equal(hi, widen_exit(want_hi))


@pytest.mark.parametrize("kind,dims,seed", CASES)
def test_labels_equal_oracle(ctx, kind, dims, seed):
    f = _field(kind, dims, seed)
    ref_g = O.gradient(f)
    ref = O.critical(f, ref_g)
    lo_ref, hi_ref = O.manifolds(f, ref_g, ref)
    nz = f.shape[0]
    for slab in sorted({1, 2, 3, 5, max(1, nz // 2), nz}):
        lo, hi, cnt = ctx.manifolds_chunked(f, slab)
        assert cnt == ref.count.tolist(), slab
        np.testing.assert_array_equal(lo, lo_ref.astype(np.uint64), err_msg=f"min labels, slab {slab}")
        np.testing.assert_array_equal(hi, widen_exit(hi_ref), err_msg=f"max labels, slab {slab}")
    lo, hi, _ = ctx.manifolds_chunked(f, 2, want_min=False)
    assert lo is None
    np.testing.assert_array_equal(hi, widen_exit(hi_ref))


def test_labels_after_release_and_regrowth(ctx):
    """Label staging that grows (a taller slab), or is freed between calls
    (ms_ctx_release), gives the same labels."""
    f = fields.grf_field((30, 24, 20), seed=4)
    ref_g = O.gradient(f)
    lo_ref, hi_ref = O.manifolds(f, ref_g, O.critical(f, ref_g))
    for slab in (2, 9, 3):
        lo, hi, _ = ctx.manifolds_chunked(f, slab)
        np.testing.assert_array_equal(lo, lo_ref.astype(np.uint64))
        np.testing.assert_array_equal(hi, widen_exit(hi_ref))
        ctx.release()


def test_labels_equal_in_hbm_512(ctx):
    """Labels and, from them, the saddle-extremum arcs (ms_extremum_arcs_host
    on the out-of-core saddles) equal those of the in-HBM run."""
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    f = fields.blob_field((512, 512, 512), nblobs=64, seed=0)
    print("[chunked] 512^3 labels", flush=True)
    got = msc.complex_(to_dev(f), ctx)
    want_lo = got.min_label.cpu().numpy().view(np.uint32).reshape(f.shape)
    want_hi = got.max_label.cpu().numpy().view(np.uint32).reshape(f.shape)
    want = [(m.rowptr.cpu().numpy(), m.col.cpu().numpy().view(np.uint32), m.val.cpu().numpy().view(np.uint64))
            for m in (got.m10, got.m32t)]
    del got
    lo, hi, cnt = ctx.manifolds_chunked(f, 100)
    np.testing.assert_array_equal(lo, want_lo.astype(np.uint64))
    np.testing.assert_array_equal(hi, widen_exit(want_hi))
    _, cid, _, _, _, cnt2 = ctx.gradient_critical_chunked(f, 100, want_grad=False)
    assert cnt2 == cnt
    off = np.cumsum([0] + cnt)
    arcs = msc.extremum_arcs_host(f.shape[::-1], lo, hi, cid[off[1]:off[2]], cid[off[2]:off[3]])
    for (rp, col, val), (w_rp, w_col, w_val) in zip(arcs, want):
        np.testing.assert_array_equal(rp, w_rp)
        np.testing.assert_array_equal(col, w_col.astype(np.uint64))
        np.testing.assert_array_equal(val, w_val)


def test_labels_beyond_32bit_cell_ids(ctx):
    nx, ny, nz = 1024, 1024, 600
    a, b, c = _zigzag(nx, 300, 7), _zigzag(ny, 410, 100), _zigzag(nz, 200, 140)
    f = np.empty((nz, ny, nx), np.float32)
    ab = (b[:, None] + a[None, :]).astype(np.float32)
    for z in range(nz):
        np.add(ab, np.float32(c[z]), out=f[z])
    print("[chunked] field built", flush=True)
    grad, cid, idx, _, _, cnt = ctx.gradient_critical_chunked(f, 120)
    lo, hi, cnt2 = ctx.manifolds_chunked(f, 120)
    assert cnt2 == cnt
    from paper_2009_03707_amd import msc
    assert msc.LABEL_EXIT64 == int(EXIT64)
    print("[chunked] labels done", flush=True)
    off = np.cumsum([0] + cnt)
    vmin = (cid[off[0]:off[1]] >> np.uint64(3)).astype(np.int64)
    vmax = (cid[off[3]:off[4]] >> np.uint64(3)).astype(np.int64)
    # saddle-extremum arcs: every 1-saddle reaches minima twice, a 2-saddle
    # maxima at most twice, columns ascending within a row
    from paper_2009_03707_amd import msc
    (rp1, c1, v1), (rp2, c2, v2) = msc.extremum_arcs_host((nx, ny, nz), lo, hi, cid[off[1]:off[2]],
                                                          cid[off[2]:off[3]])
    assert (np.add.reduceat(v1, rp1[:-1]) == 2).all() and int(c1.max()) < cnt[0]
    assert (np.diff(rp2) <= 2).all() and (c2 < np.uint64(cnt[3])).all()
    for rp, c in ((rp1, c1), (rp2, c2)):
        two = np.flatnonzero(np.diff(rp) == 2)
        assert (c[rp[two]] < c[rp[two] + 1]).all()
    del cid, idx
    # roots: each extremum labels itself with its rank
    np.testing.assert_array_equal(lo.reshape(-1)[vmin], np.arange(len(vmin), dtype=np.uint64))
    np.testing.assert_array_equal(hi.reshape(-1)[vmax], np.arange(len(vmax), dtype=np.uint64))
    assert int(lo.max()) < cnt[0]
    assert int(hi[hi != EXIT64].max()) < cnt[3]
    for z0 in range(0, nz, 50):  # every row, across the slab boundaries too
        z1 = min(nz, z0 + 50)
        check_forest(grad, lo, vmin, 0, False, z0, z1)
        check_forest(grad, hi, vmax, 7, True, z0, z1, EXIT64)

