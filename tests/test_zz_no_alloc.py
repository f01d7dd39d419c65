"""ms_critical_noalloc: the allocation-free variant of ms_critical.

It is called through the C ABI on a context whose allocator fails the test
if it is ever called, and must give the same counts and the same critical
list as ms_critical on two calls in a row, the second on a smaller field
(the fixed scratch keeps the first call's contents).  Fields too large for
the fixed scratch are refused before any device work."""
import numpy as np
import pytest

from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _no_alloc_context():
    from paper_2009_03707_amd import msc
    calls = []

    def alloc(user, nbytes, stream):
        calls.append(int(nbytes))
        return None

    def free(user, ptr, nbytes, stream):
        calls.append(-1)

    fns = (msc.ALLOC_FN(alloc), msc.FREE_FN(free))
    ctx = msc.Context(allocator=fns)
    return ctx, calls, fns


def _expected(f_dev):
    """Gradient and critical list from the allocating entry points."""
    from paper_2009_03707_amd import msc
    ctx = msc.Context()
    g = ctx.gradient(f_dev)
    ids, idx, val, vm, cnt = ctx.critical(f_dev, g)
    out = (g, ids.clone(), idx.clone(), val.clone(), vm.clone(), cnt)
    torch.cuda.synchronize()
    ctx.close()
    return out


def _run_noalloc(ctx, f_dev, g, n):
    dev = f_dev.device
    bufs = (torch.full((n,), -7, dtype=torch.int32, device=dev), torch.full((n,), 0xEE, dtype=torch.uint8, device=dev),
            torch.full((n,), -1.0, dtype=torch.float32, device=dev), torch.full((n,), -7, dtype=torch.int32, device=dev))
    cnt = ctx.critical_noalloc(f_dev, g, bufs)
    torch.cuda.synchronize()
    return cnt, bufs


def _same(cnt, bufs, want):
    g, ids, idx, val, vm, wcnt = want
    assert cnt == wcnt
    n = sum(wcnt)
    np.testing.assert_array_equal(bufs[0][:n].cpu().numpy(), ids.cpu().numpy())
    np.testing.assert_array_equal(bufs[1][:n].cpu().numpy(), idx.cpu().numpy())
    np.testing.assert_array_equal(bufs[2][:n].cpu().numpy().view(np.uint32), val.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(bufs[3][:n].cpu().numpy(), vm.cpu().numpy())


def test_noalloc_matches_critical_twice_then_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from gpu_util import to_dev
    ctx, calls, fns = _no_alloc_context()
    ctx.set_timing(True)
    big = to_dev(fields.blob_field((160, 150, 140), nblobs=40, seed=9))
    small = to_dev(fields.grf_field((37, 29, 23), seed=5))
    want_big, want_small = _expected(big), _expected(small)
    for f, want in ((big, want_big), (small, want_small)):
        n = sum(want[5])
        # counts only, then the list
        assert ctx.critical_noalloc(f, want[0], None) == want[5]
        cnt, bufs = _run_noalloc(ctx, f, want[0], n + 5)
        _same(cnt, bufs, want)
        # the 5 extra entries are untouched
        assert (bufs[0][n:].cpu().numpy() == -7).all()
    t = ctx.timing()
    assert calls == [] and t["allocations"] == 0 and t["workspace_bytes"] == 0
    ctx.close()


def test_noalloc_capacity_and_size_errors():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    ctx, calls, fns = _no_alloc_context()
    f = to_dev(fields.random_field((20, 18, 16), seed=2))
    want = _expected(f)
    n = sum(want[5])
    with pytest.raises(msc.MscError) as e:
        _run_noalloc(ctx, f, want[0], n - 1)
    assert e.value.status == msc.MS_ERR_CAPACITY
    # dims beyond the fixed scratch: refused on the host before any launch
    # (the tiny tensors are never read)
    lib, C = msc.lib(), msc.C
    cnt = (C.c_int64 * 4)()
    st = lib.ms_critical_noalloc(ctx._h, C.c_void_p(f.data_ptr()), C.c_void_p(want[0].data_ptr()),
                                 msc.Dims(1024, 1024, 300), None, cnt)
    assert st == msc.MS_ERR_TOO_LARGE
    assert b"fixed scratch" in lib.ms_last_error(ctx._h)
    assert calls == []
    ctx.close()
