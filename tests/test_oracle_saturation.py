"""Pins of the oracle's saturating path counts (CPU).

The paper notes that the number of gradient paths between two saddles grows
exponentially with the number of splits and merges (Sections 3.1 and 3.3;
its experiments report multiplicities near 1e10).  The contract counts paths
as unsigned 64-bit integers that saturate at 2^64 - 1, i.e. every count is
min(true count, 2^64 - 1).  A hand-built gradient (tests/diamonds.py) with k
split-merge diamonds in a row has exactly 2^k paths from its source 1-saddle
to each of its two end 2-saddles, which crosses 2^64 at k = 64.  The oracle
is pinned by:
  * the closed form 2^k (capped) for the chain's own entries;
  * explicit V-path enumeration (Section 2.2 definition) of the whole
    matrix for k <= 12;
  * exact arbitrary-precision path counts over the DAG for every entry and
    for the number of saturated entries, at k = 63, 64, 65, 70.
"""
import numpy as np
import pytest

import cellgeom as CG
import diamonds
from oracle import oracle as O

U64_MAX = (1 << 64) - 1


def _setup(k):
    grad, info = diamonds.build(k)
    nx, ny, nz = info["dims"]
    G = CG.Grid(np.zeros((nz, ny, nx), np.float32))
    crit = CG.critical_from_grad(G, grad)
    count = np.array([len(c) for c in crit], np.int64)
    ids = np.array([c for lst in crit for c in lst], np.uint32)
    cr = O.Critical(ids, np.zeros(len(ids), np.uint8), np.zeros(len(ids), np.float32),
                    np.zeros(len(ids), np.uint32), count)
    return grad, info, G, crit, cr


def _oracle_p_by_ids(grad, crit, cr):
    p = O.ss_paths(np.zeros(grad.shape, np.float32), grad, cr)
    s1, s2 = crit[1], crit[2]
    return {(s1[int(r)], s2[int(c)]): int(v) for r, c, v in zip(p.row, p.col, p.val)}


@pytest.mark.parametrize("k", [0, 1, 2, 5, 12, 70])
def test_diamond_gradient_is_valid(k):
    grad, info, G, crit, cr = _setup(k)
    CG.check_gradient_valid(G, grad, lower_star=False)
    assert info["source"] in crit[1]
    assert all(e in crit[2] for e in info["ends"])


@pytest.mark.parametrize("k", [0, 1, 2, 3, 6, 9, 12])
def test_diamond_counts_equal_vpath_enumeration(k):
    grad, info, G, crit, cr = _setup(k)
    got = _oracle_p_by_ids(grad, crit, cr)
    # explicit V-paths, walked down from every 2-saddle (Section 2.2)
    vp = CG.vpath_counts(G, grad, crit)[1]
    want = {(lo, hi): c for (hi, lo), c in vp.items()}
    assert got == want
    for e in info["ends"]:
        assert got[(info["source"], e)] == 2 ** k
    assert got[(info["source"], info["near"])] == 1
    assert {q for (s, q) in got if s == info["source"]} == set(info["ends"]) | {info["near"]}


@pytest.mark.parametrize("k", [63, 64, 65, 70])
def test_diamond_counts_saturate(k):
    grad, info, G, crit, cr = _setup(k)
    got = _oracle_p_by_ids(grad, crit, cr)
    for e in info["ends"]:
        assert got[(info["source"], e)] == min(2 ** k, U64_MAX)
    exact = CG.exact_path_counts(G, grad, crit[1])
    assert set(got) == set(exact)
    for key, c in exact.items():
        assert got[key] == min(c, U64_MAX), key
    n_sat = sum(1 for v in got.values() if v == U64_MAX)
    assert n_sat == sum(1 for c in exact.values() if c >= U64_MAX)
    if k >= 64:
        assert n_sat >= 2
    else:
        assert n_sat == 0
