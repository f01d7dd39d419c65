"""GPU parity of the whole hot path (ms_complex and the separate entry points)
against the oracle: gradient words, critical lists and all six arc matrices
bit-exact (integer outputs; path counts are exact saturating u64)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["ready", "power", "ready-chunked", "entry", "entry-pack1", "entry-wide",
                                        "ready-pack2", "entry-pack4", "power-pack4"])
def ctx(request):
    """The path-counting schedules: the ready frontier, the paper's power
    iteration and the entry ranking; "ready-chunked" sends every column
    through the workgroup merge with tiny chunks, so that chunk splitting is
    exercised on small fields.  The transposes: "entry-pack1" packs only
    the matrices whose values are all 1 and "ready-pack2" those whose values
    are at most 3 (the others move their values as a separate payload);
    "entry-wide" packs none; "entry-pack4" and "power-pack4" pack four value
    bits, so that every path count of 15 or more is an escape, looked up
    again after the transpose."""
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = msc.Context()
    sched = request.param.split("-")[0]
    c.set_path_schedule({"power": msc.MS_PATHS_POWER, "entry": msc.MS_PATHS_ENTRY}.get(sched, msc.MS_PATHS_READY))
    if request.param == "ready-chunked":
        c.set_option(msc.MS_OPT_MERGE_LIGHT, 0)
        c.set_option(msc.MS_OPT_MERGE_CHUNK, 3)
    pack = {"entry-pack1": 1, "entry-wide": 0, "ready-pack2": 2, "entry-pack4": 4, "power-pack4": 4}.get(request.param)
    if pack is not None:
        c.set_option(msc.MS_OPT_TRANSPOSE_PACK, pack)
    yield c
    c.close()


def _transpose(coo):
    order = np.lexsort((coo.row, coo.col))
    t = O.Coo(coo.col[order], coo.row[order], coo.val[order], (coo.shape[1], coo.shape[0]))
    return t


def _eq_csr(got, coo, name):
    from gpu_util import csr_np
    rp, col, val = coo.csr()
    g_rp, g_col, g_val = csr_np(got)
    assert got.nrows == coo.shape[0] and got.ncols == coo.shape[1], (name, got.nrows, got.ncols, coo.shape)
    np.testing.assert_array_equal(g_rp, rp, err_msg=name)
    np.testing.assert_array_equal(g_col, col, err_msg=name)
    np.testing.assert_array_equal(g_val, val, err_msg=name)


def check_complex(ctx, f):
    from gpu_util import to_dev, u32
    from paper_2009_03707_amd import msc
    ref = O.complex_(f)
    got = msc.complex_(to_dev(f), ctx)
    np.testing.assert_array_equal(u32(got.grad).reshape(f.shape), ref.grad)
    assert got.count == ref.crit.count.tolist()
    np.testing.assert_array_equal(u32(got.crit_id), ref.crit.id)
    np.testing.assert_array_equal(got.crit_index.cpu().numpy(), ref.crit.index)
    np.testing.assert_array_equal(got.crit_value.cpu().numpy().view(np.uint32), ref.crit.value.view(np.uint32))
    np.testing.assert_array_equal(u32(got.crit_vmax), ref.crit.vmax)
    _eq_csr(got.m10, ref.m10, "m10")
    _eq_csr(got.m10t, _transpose(ref.m10), "m10t")
    _eq_csr(got.m32, ref.m32, "m32")
    _eq_csr(got.m32t, _transpose(ref.m32), "m32t")
    _eq_csr(got.m21t, ref.p, "m21t")
    _eq_csr(got.m21, _transpose(ref.p), "m21")
    assert got.n_saturated == int((ref.p.val == np.uint64(2 ** 64 - 1)).sum())
    return got, ref


def _cases():
    rng = np.random.default_rng(777)
    out = []
    for i in range(24):
        dims = tuple(int(v) for v in rng.integers(1, 20, size=3))
        out.append(("rand", dims, 200 + i, int(rng.choice([0, 0, 2, 4]))))
    for dims in [(1, 1, 1), (2, 2, 2), (7, 1, 1), (1, 6, 5), (33, 9, 5), (5, 40, 3)]:
        out.append(("rand", dims, 9, 0))
    return out


@pytest.mark.parametrize("kind,dims,seed,levels", _cases())
def test_random_fields(ctx, kind, dims, seed, levels):
    check_complex(ctx, fields.random_field(dims, seed=seed, levels=levels))


@pytest.mark.parametrize("name", ["sine32", "grf48", "blob64", "blob72dense", "monotone", "constant"])
def test_structured_fields(ctx, name):
    if name == "sine32":
        f = fields.sine_field(32)
    elif name == "grf48":
        f = fields.grf_field((48, 44, 40), seed=2)
    elif name == "blob64":
        f = fields.blob_field((64, 64, 64), nblobs=4, seed=0)
    elif name == "blob72dense":
        f = fields.blob_field((72, 70, 66), nblobs=12, seed=5)
    elif name == "monotone":
        f = np.arange(30 * 20 * 10, dtype=np.float32).reshape(10, 20, 30)
    else:
        f = np.zeros((9, 8, 7), np.float32)
    got, ref = check_complex(ctx, f)
    if name == "sine32":
        assert got.count == [192, 472, 386, 105]


def test_separate_entry_points_match_complex(ctx):
    from gpu_util import to_dev, u32, csr_np
    from paper_2009_03707_amd import msc
    f = fields.grf_field((30, 25, 20), seed=4)
    fd = to_dev(f)
    g = ctx.gradient(fd)
    ids, idx, val, vm, cnt = ctx.critical(fd, g)
    arcs = ctx.connect(g, (30, 25, 20), ids, cnt)
    dev = fd.device
    p_sep = msc.csr_to_torch(arcs.m21t, dev)
    m10_sep = msc.csr_to_torch(arcs.m10, dev)
    torch.cuda.synchronize()
    ref = O.complex_(f)
    _eq_csr(p_sep, ref.p, "m21t via ms_connect")
    _eq_csr(m10_sep, ref.m10, "m10 via ms_connect")


def test_deterministic_repeat(ctx):
    from gpu_util import to_dev, u32, csr_np
    from paper_2009_03707_amd import msc
    f = fields.blob_field((40, 36, 32), nblobs=3, seed=1)
    a = msc.complex_(to_dev(f), ctx)
    b = msc.complex_(to_dev(f), ctx)
    for name in ("m10", "m10t", "m21", "m21t", "m32", "m32t"):
        for x, y in zip(csr_np(getattr(a, name)), csr_np(getattr(b, name))):
            np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a.min_label.cpu().numpy(), b.min_label.cpu().numpy())
    np.testing.assert_array_equal(a.max_label.cpu().numpy(), b.max_label.cpu().numpy())
    # every statistic but the pointer-jumping round counts, which depend on
    # how far the in-place rounds see each other's updates
    sa = {k: v for k, v in a.stats.items() if not k.startswith("pj_rounds")}
    sb = {k: v for k, v in b.stats.items() if not k.startswith("pj_rounds")}
    assert sa == sb
    for k in ("pj_rounds_vertex", "pj_rounds_cube"):
        assert 1 <= a.stats[k] <= 65 and 1 <= b.stats[k] <= 65


def test_connect_rejects_mismatched_critical_list(ctx):
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    f = fields.random_field((10, 9, 8), seed=3)
    fd = to_dev(f)
    g = ctx.gradient(fd)
    ids, idx, val, vm, cnt = ctx.critical(fd, g)
    bad = ids.clone()
    bad[0] = bad[1]  # not strictly increasing
    with pytest.raises(msc.MscError) as e:
        ctx.connect(g, (10, 9, 8), bad, cnt)
    assert e.value.status == msc.MS_ERR_INTERNAL


def test_record_buffers_reused_across_sizes():
    """The critical records are scattered before the host reads their count
    whenever the context already holds record buffers; a call whose records
    do not fit them writes nothing there and scatters again once they have
    grown.  A fresh context sees: no buffers, then more records than they
    hold, fewer, far fewer, more again -- each result equal to the oracle's."""
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = msc.Context()
    try:
        for dims, seed in [((12, 10, 9), 1), ((40, 38, 30), 2), ((20, 22, 18), 3), ((3, 2, 2), 4), ((44, 40, 33), 5)]:
            check_complex(c, fields.random_field(dims, seed=seed))
    finally:
        c.close()
