"""The forest check of manifold labels (tests/forest.py), which the GPU
tests use where no oracle run fits, is itself checked on the CPU: it accepts
the oracle's labels (pinned in tests/test_oracle_manifolds.py) for every
split of the rows into chunks, and rejects labels with one planted mistake
(a label off by one, or an exit label where there is a maximum, or the
reverse), wherever the mistake is, given the roots it checks separately."""
import numpy as np
import pytest

from forest import EXIT64, check_forest, widen_exit
from oracle import oracle as O
from paper_2009_03707_amd import fields

FIELDS = [("blob", (40, 33, 27), 5), ("rand", (9, 8, 7), 0), ("grf", (30, 24, 20), 4), ("rand", (1, 1, 9), 2),
          ("rand", (13, 1, 6), 3)]


def _field(kind, dims, seed):
    if kind == "rand":
        return fields.random_field(dims, seed=seed, levels=seed % 3)
    if kind == "grf":
        return fields.grf_field(dims, seed=seed)
    return fields.blob_field(dims, nblobs=6, seed=seed)


def _case(kind, dims, seed):
    f = _field(kind, dims, seed)
    g = O.gradient(f)
    cr = O.critical(f, g)
    lo, hi = O.manifolds(f, g, cr)
    off = np.cumsum([0] + cr.count.tolist())
    ids = cr.id.astype(np.int64)
    return g, lo.astype(np.uint64), widen_exit(hi), ids[off[0]:off[1]] >> 3, ids[off[3]:off[4]] >> 3


def _check_all(g, lab, roots, cube, step):
    nz = lab.shape[0]
    for z0 in range(0, nz, step):
        check_forest(g, lab, roots, 7 if cube else 0, cube, z0, min(nz, z0 + step), EXIT64 if cube else None)


@pytest.mark.parametrize("kind,dims,seed", FIELDS)
def test_accepts_oracle_labels(kind, dims, seed):
    g, lo, hi, vmin, vmax = _case(kind, dims, seed)
    for step in (1, 3, lo.shape[0]):
        _check_all(g, lo, vmin, False, step)
        _check_all(g, hi, vmax, True, step)


@pytest.mark.parametrize("kind,dims,seed", FIELDS[:3])
def test_rejects_planted_mistakes(kind, dims, seed):
    g, lo, hi, vmin, vmax = _case(kind, dims, seed)
    rng = np.random.default_rng(seed)
    for lab, roots, cube in ((lo, vmin, False), (hi, vmax, True)):
        flat = lab.reshape(-1)
        rootset = set(roots.tolist())
        cand = [v for v in range(flat.size) if v not in rootset]  # root labels are checked apart
        for v in rng.choice(cand, size=min(25, len(cand)), replace=False):
            bad = lab.copy()
            b = bad.reshape(-1)
            b[v] = np.uint64(0) if b[v] == EXIT64 else (EXIT64 if cube and b[v] == 0 else b[v] + np.uint64(1))
            with pytest.raises(AssertionError):
                _check_all(g, bad, roots, cube, 4)
