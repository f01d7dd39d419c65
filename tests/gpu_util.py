"""Helpers for the GPU parity tests: run the library through the C ABI and
bring results back as numpy arrays."""
import numpy as np
import torch

from paper_2009_03707_amd import msc


def to_dev(f: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def csr_np(m):
    return m.rowptr.cpu().numpy(), u32(m.col), u64(m.val)


def coo_to_csr(coo):
    """Oracle COO (sorted) -> (rowptr, col, val) numpy."""
    return coo.csr()


NAMES = ("m10", "m10t", "m21", "m21t", "m32", "m32t")


def same_complex(a, b):
    """Two msc.Complex results are byte-identical."""
    np.testing.assert_array_equal(u32(a.grad), u32(b.grad))
    assert a.count == b.count
    for x, y in ((a.crit_id, b.crit_id), (a.crit_vmax, b.crit_vmax)):
        np.testing.assert_array_equal(u32(x), u32(y))
    np.testing.assert_array_equal(a.crit_index.cpu().numpy(), b.crit_index.cpu().numpy())
    np.testing.assert_array_equal(a.crit_value.cpu().numpy().view(np.uint32), b.crit_value.cpu().numpy().view(np.uint32))
    for nm in NAMES:
        ma, mb = getattr(a, nm), getattr(b, nm)
        assert (ma.nrows, ma.ncols) == (mb.nrows, mb.ncols), nm
        for x, y in zip(csr_np(ma), csr_np(mb)):
            np.testing.assert_array_equal(x, y, err_msg=nm)
    assert a.n_saturated == b.n_saturated
