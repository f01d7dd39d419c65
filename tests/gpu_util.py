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
