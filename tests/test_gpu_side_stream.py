"""The saddle-extremum arcs (pointer jumping, M10, M32, their transposes,
the manifold labels) and, with the entry schedule, the transposes of B* and
D run on a second stream of the context, queued by a helper thread while
the calling thread queues the minor and the path counting; the context's
own stream waits for them where their results are needed.

* A context bound to a non-default torch stream gives, call after call, the
  same complexes (and manifold labels) as one on the default stream, under
  every path schedule.
* With timing on, the side work's own span is reported, and enabling
  timing again resets it."""
import numpy as np
import pytest

from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _field(seed):
    return fields.blob_field((48, 40, 36), nblobs=6, seed=seed)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("schedule", ["ready", "power", "entry"])
def test_user_stream_matches_default_stream(schedule):
    from gpu_util import same_complex, to_dev
    from paper_2009_03707_amd import msc
    _need_gpu()
    sched = {"ready": msc.MS_PATHS_READY, "power": msc.MS_PATHS_POWER, "entry": msc.MS_PATHS_ENTRY}[schedule]
    fs = [to_dev(_field(s)) for s in range(3)]
    ref = msc.Context()
    want = [msc.complex_(f, ref) for f in fs]
    ref.close()
    user = torch.cuda.Stream()
    with torch.cuda.stream(user):
        ctx = msc.Context()
        ctx.set_path_schedule(sched)
        for rep in range(2):
            for f, w in zip(fs, want):
                got = msc.complex_(f, ctx)
                same_complex(got, w)
                np.testing.assert_array_equal(got.min_label.cpu().numpy(), w.min_label.cpu().numpy())
                np.testing.assert_array_equal(got.max_label.cpu().numpy(), w.max_label.cpu().numpy())
        ctx.close()


def test_side_time_reported_and_reset():
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    _need_gpu()
    f = to_dev(_field(7))
    ctx = msc.Context()
    ctx.set_timing(True)
    msc.complex_(f, ctx)
    msc.complex_(f, ctx)
    t = ctx.timing()
    assert t["calls"] == 2
    assert t["side_ms"] > 0
    ctx.set_timing(True)
    assert ctx.timing()["side_ms"] == 0
    ctx.close()


class SideFailingAllocator:
    """Allocates from torch's caching allocator and tracks every live block;
    while `refuse_side` is set it refuses every request made for a stream
    other than `main` (the helper thread's side stream)."""

    def __init__(self, main_stream):
        from paper_2009_03707_amd import msc
        self.main = int(main_stream or 0)
        self.refuse_side = True
        self.refused = 0
        self.live = {}
        self.fns = (msc.ALLOC_FN(self._alloc), msc.FREE_FN(self._free))

    def _alloc(self, user, nbytes, stream):
        if self.refuse_side and int(stream or 0) != self.main:
            self.refused += 1
            return None
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0, int(stream or 0))
        self.live[p] = int(nbytes)
        return p

    def _free(self, user, ptr, nbytes, stream):
        assert self.live.pop(int(ptr)) == int(nbytes)
        torch.cuda.caching_allocator_delete(int(ptr))


@pytest.mark.parametrize("schedule", ["ready", "entry"])
def test_side_failure_is_reported_and_recovered(schedule):
    """An allocation refused on the helper thread fails the call with
    MS_ERR_OOM and its text, leaks nothing, and the same context then gives
    the same complex as a context that never failed."""
    from gpu_util import same_complex, to_dev
    from paper_2009_03707_amd import msc
    _need_gpu()
    sched = {"ready": msc.MS_PATHS_READY, "entry": msc.MS_PATHS_ENTRY}[schedule]
    f = to_dev(_field(11))
    ref = msc.Context()
    ref.set_path_schedule(sched)
    want = msc.complex_(f, ref)
    ref.close()
    a = SideFailingAllocator(torch.cuda.current_stream().cuda_stream)
    ctx = msc.Context(allocator=a.fns)
    ctx.set_path_schedule(sched)
    ctx.set_timing(True)
    with pytest.raises(msc.MscError) as e:
        msc.complex_(f, ctx)
    assert e.value.status == msc.MS_ERR_OOM
    assert "allocation" in str(e.value)
    assert a.refused >= 1
    assert ctx.timing()["workspace_bytes"] == sum(a.live.values())
    a.refuse_side = False
    got = msc.complex_(f, ctx)
    same_complex(got, want)
    np.testing.assert_array_equal(got.min_label.cpu().numpy(), want.min_label.cpu().numpy())
    np.testing.assert_array_equal(got.max_label.cpu().numpy(), want.max_label.cpu().numpy())
    ctx.close()
    assert a.live == {}


def test_release_between_calls():
    """ms_ctx_release frees the whole workspace, the helper thread's buffers
    included; the next calls reallocate it and give the same complex, and the
    workspace then equals what one call needs from scratch."""
    from gpu_util import same_complex, to_dev
    from paper_2009_03707_amd import msc
    _need_gpu()
    f = to_dev(_field(5))
    ctx = msc.Context()
    ctx.set_path_schedule(msc.MS_PATHS_ENTRY)
    ctx.set_timing(True)
    want = msc.complex_(f, ctx)
    ws = ctx.timing()["workspace_bytes"]
    assert ws > 0
    ctx.release()
    assert ctx.timing()["workspace_bytes"] == 0
    for _ in range(2):
        got = msc.complex_(f, ctx)
        same_complex(got, want)
        np.testing.assert_array_equal(got.min_label.cpu().numpy(), want.min_label.cpu().numpy())
    assert ctx.timing()["workspace_bytes"] == ws
    ctx.close()
