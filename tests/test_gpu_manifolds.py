"""GPU parity of the ascending / descending 3-manifold labels (Section 3.4:
the pointer jumping that yields the saddle-extremum arcs also gives every
vertex its minimum and every cube its maximum; Section 3.5 keeps them in an
extra array).  The labels exported by ms_complex, ms_connect and
ms_complex_batch must equal the oracle's (pinned on the CPU in
tests/test_oracle_manifolds.py) word for word."""
import numpy as np
import pytest

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


def _field(kind, dims, seed):
    if kind == "rand":
        return fields.random_field(dims, seed=seed, levels=seed % 3)
    if kind == "sine":
        return fields.sine_field(dims)
    if kind == "grf":
        return fields.grf_field(dims, seed=seed)
    return fields.blob_field(dims, nblobs=6, seed=seed)


CASES = [("rand", (1, 1, 1), 0), ("rand", (7, 1, 1), 1), ("rand", (1, 9, 4), 2), ("rand", (13, 11, 9), 3),
         ("rand", (33, 17, 5), 4), ("sine", 32, 0), ("grf", (48, 44, 40), 2), ("blob", (64, 60, 52), 5)]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("kind,dims,seed", CASES)
def test_labels_equal_oracle(ctx, kind, dims, seed):
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    f = _field(kind, dims, seed)
    ref = O.complex_(f)
    got = msc.complex_(to_dev(f), ctx)
    np.testing.assert_array_equal(_u32(got.min_label).reshape(f.shape), ref.min_label)
    np.testing.assert_array_equal(_u32(got.max_label).reshape(f.shape), ref.max_label)


def test_labels_from_connect(ctx):
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    f = fields.grf_field((30, 25, 20), seed=4)
    fd = to_dev(f)
    g = ctx.gradient(fd)
    ids, idx, val, vm, cnt = ctx.critical(fd, g)
    arcs = ctx.connect(g, (30, 25, 20), ids, cnt)
    nv = f.size
    lo = msc._copy_dev(arcs.min_label, 4 * nv, torch.int32, nv, fd.device)
    hi = msc._copy_dev(arcs.max_label, 4 * nv, torch.int32, nv, fd.device)
    torch.cuda.synchronize()
    ref = O.complex_(f)
    np.testing.assert_array_equal(_u32(lo).reshape(f.shape), ref.min_label)
    np.testing.assert_array_equal(_u32(hi).reshape(f.shape), ref.max_label)


def test_batch_labels_are_per_field(ctx):
    """In a batch, ranks are the field's own (not batch-wide) and every field's
    labels equal the oracle's for that field alone."""
    from gpu_util import to_dev
    from paper_2009_03707_amd import msc
    fs = [fields.random_field((9, 8, 7), seed=11), fields.grf_field((21, 13, 17), seed=3),
          fields.random_field((1, 1, 1), seed=1), fields.blob_field((20, 19, 18), nblobs=4, seed=2),
          fields.random_field((5, 1, 12), seed=4, levels=2)]
    outs = msc.complex_batch([to_dev(f) for f in fs], ctx)
    for f, got in zip(fs, outs):
        ref = O.complex_(f)
        np.testing.assert_array_equal(_u32(got.min_label).reshape(f.shape), ref.min_label)
        np.testing.assert_array_equal(_u32(got.max_label).reshape(f.shape), ref.max_label)
