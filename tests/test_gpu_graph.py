"""ms_graph_build from device results (ms_complex and one field of
ms_complex_batch): the host MS-complex graph equals the oracle's, and its
serial simplification equals the oracle's cancellation by cancellation."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import simplify as S
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


def _live(g):
    from paper_2009_03707_amd import msc
    out = {}
    for i in range(g.num_nodes()):
        nd = g.node(i)
        if nd["alive"]:
            nbr, mult = g.arcs(i, msc.MS_DOWN)
            out[i] = (nd["index"], {int(a): int(b) for a, b in zip(nbr, mult)})
    return out


def _check(g, f, thr):
    from paper_2009_03707_amd import msc
    og = S.from_complex(O.complex_(f, labels=False))
    assert g.num_nodes() == len(og.index)
    assert [g.node(i)["cell"] for i in range(g.num_nodes())] == og.cell
    for i in range(g.num_nodes()):
        nbr, mult = g.arcs(i, msc.MS_UP)
        assert {int(a): int(b) for a, b in zip(nbr, mult)} == og.up[i]
    assert _live(g) == S.live_graph(og)
    g.simplify(thr, msc.MS_SIMPLIFY_SERIAL, 1)
    S.simplify(og, thr)
    assert g.cancellations() == [(u, l, p) for u, l, p in og.log]
    assert _live(g) == S.live_graph(og)


@pytest.mark.parametrize("dims,seed,thr", [((16, 14, 12), 0, 0.1), ((30, 20, 10), 1, float("inf")),
                                           ((9, 1, 40), 2, 0.3)])
def test_graph_from_complex(ctx, dims, seed, thr):
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    f = fields.grf_field(dims, seed=seed)
    r = ctx.complex_raw(to_dev(f))
    g = msc.Graph.from_result(ctx, r, dims, nthreads=4)
    _check(g, f, thr)
    g.close()


def test_graph_from_batch_member(ctx):
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    fs = [fields.random_field((7, 6, 5), seed=3), fields.blob_field((20, 18, 16), nblobs=4, seed=2),
          fields.grf_field((12, 11, 10), seed=4)]
    rs = ctx.complex_batch_raw([to_dev(f) for f in fs])
    for f, r in zip(fs, rs):
        nz, ny, nx = f.shape
        g = msc.Graph.from_result(ctx, r, (nx, ny, nz), nthreads=2)
        _check(g, f, 0.2)
        g.close()
