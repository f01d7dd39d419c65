"""The captured front of ms_complex_batch (MS_OPT_BATCH_GRAPH): the graph
holding the gradient, the critical counts, their scan and totals is
captured once per set of dims and replayed; every replay -- with new field
contents, and with the context's own eager work and synchronisations in
between -- gives results byte-identical to the eager launch."""
import pytest

from paper_2009_03707_amd import fields

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DIMS = [(21, 13, 17), (9, 8, 7), (30, 1, 12), (16, 16, 16)]


def _fields(seed):
    out = []
    for i, d in enumerate(DIMS):
        if i % 2:
            out.append(fields.grf_field(d, seed=seed + i))
        else:
            out.append(fields.random_field(d, seed=seed + i, levels=(seed + i) % 3))
    return out


def _dev(fs):
    from gpu_util import to_dev
    return [to_dev(f) for f in fs]


def test_replays_equal_eager():
    from gpu_util import same_complex
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = msc.Context()
    e = msc.Context()
    e.set_option(msc.MS_OPT_BATCH_GRAPH, 0)
    t0 = g.timing()
    for rep, seed in enumerate((1, 2, 3, 1, 4)):
        fs = _dev(_fields(seed))
        got = msc.complex_batch(fs, g)
        want = msc.complex_batch(fs, e)
        for a, b in zip(got, want):
            same_complex(a, b)
        # eager work on the graph's own context between replays
        same_complex(msc.complex_(fs[0], g), want[0])
        torch.cuda.synchronize()
    t = g.timing()
    assert t["graph_captures"] - t0["graph_captures"] == 1
    assert t["graph_replays"] - t0["graph_replays"] == 5
    assert e.timing()["graph_replays"] == 0
    # other dims: a new capture, still equal to eager
    fs = _dev([fields.grf_field((12, 11, 10), seed=7), fields.random_field((5, 6, 7), seed=8)])
    for a, b in zip(msc.complex_batch(fs, g), msc.complex_batch(fs, e)):
        same_complex(a, b)
    assert g.timing()["graph_captures"] - t0["graph_captures"] == 2
    g.close()
    e.close()


def test_nonfinite_member_reported_through_the_graph():
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = msc.Context()
    fs = _fields(5)
    msc.complex_batch(_dev(fs), g)  # capture
    bad = [f.copy() for f in fs]
    bad[2].reshape(-1)[7] = float("nan")
    with pytest.raises(msc.MscError) as ex:
        msc.complex_batch(_dev(bad), g)  # replay with a NaN in one field
    assert ex.value.status == msc.MS_ERR_NONFINITE
    msc.complex_batch(_dev(fs), g)  # and the flag is cleared again on the next replay
    g.close()
