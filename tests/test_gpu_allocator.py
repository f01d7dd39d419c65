"""The workspace allocator hooks of ms_ctx_create (include/msc.h).

A context whose allocator refuses its k-th request must fail that call with
MS_ERR_OOM, leak nothing (the context's workspace_bytes equals what the
allocator still has out), stay usable, and give on a retry the same result
and the same workspace as a context that never failed."""
import numpy as np
import pytest

from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


class CountingAllocator:
    """Allocates from torch's caching allocator, counts requests, refuses
    request number `fail_at` (1-based), and tracks every live block."""

    def __init__(self, fail_at=None):
        from paper_2009_03707_amd import msc
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.fns = (msc.ALLOC_FN(self._alloc), msc.FREE_FN(self._free))

    def _alloc(self, user, nbytes, stream):
        self.calls += 1
        if self.fail_at is not None and self.calls == self.fail_at:
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        self.live[p] = int(nbytes)
        return p

    def _free(self, user, ptr, nbytes, stream):
        assert self.live.pop(int(ptr)) == int(nbytes)
        torch.cuda.caching_allocator_delete(int(ptr))

    @property
    def live_bytes(self):
        return sum(self.live.values())


def _field():
    return fields.blob_field((40, 36, 32), nblobs=5, seed=3)


def _reference():
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    a = CountingAllocator()
    ctx = msc.Context(allocator=a.fns)
    ctx.set_timing(True)
    out = msc.complex_(to_dev(_field()), ctx)
    ws = ctx.timing()["workspace_bytes"]
    assert ws == a.live_bytes > 0
    ctx.close()
    assert a.live == {}
    return out, ws, a.calls


@pytest.fixture(scope="module")
def reference():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return _reference()


def test_hooks_carry_every_workspace_block(reference):
    out, ws, calls = reference
    assert calls > 10


@pytest.mark.parametrize("where", ["first", "early", "middle", "last"])
def test_oom_then_retry(reference, where):
    from gpu_util import same_complex, to_dev
    from paper_2009_03707_amd import msc
    want, ws_ref, calls = reference
    k = {"first": 1, "early": 3, "middle": calls // 2, "last": calls}[where]
    a = CountingAllocator(fail_at=k)
    ctx = msc.Context(allocator=a.fns)
    ctx.set_timing(True)
    f = to_dev(_field())
    with pytest.raises(msc.MscError) as e:
        msc.complex_(f, ctx)
    assert e.value.status == msc.MS_ERR_OOM
    assert "allocation" in str(e.value)
    assert ctx.timing()["workspace_bytes"] == a.live_bytes
    a.fail_at = None
    got = msc.complex_(f, ctx)
    same_complex(got, want)
    np.testing.assert_array_equal(got.min_label.cpu().numpy(), want.min_label.cpu().numpy())
    np.testing.assert_array_equal(got.max_label.cpu().numpy(), want.max_label.cpu().numpy())
    assert ctx.timing()["workspace_bytes"] == a.live_bytes == ws_ref
    ctx.close()
    assert a.live == {}


def test_one_hook_alone_is_rejected():
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    a = CountingAllocator()
    with pytest.raises(msc.MscError) as e:
        msc.Context(allocator=(a.fns[0], msc.FREE_FN()))
    assert e.value.status == msc.MS_ERR_INVALID_ARG


def test_hip_allocator_path(reference):
    """NULL hooks: the library's own hipMalloc path gives the same result."""
    from gpu_util import same_complex, to_dev
    from paper_2009_03707_amd import msc
    want = reference[0]
    ctx = msc.Context(allocator="hip")
    same_complex(msc.complex_(to_dev(_field()), ctx), want)
    ctx.close()
