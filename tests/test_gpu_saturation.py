"""GPU parity of saturating path counts (u64, capped at 2^64 - 1).

The hand-built gradient of tests/diamonds.py chains k split-merge diamonds
(Section 3.1 and Figure 6: gradient paths between saddles split and merge),
so its source 1-saddle reaches each of its two end 2-saddles by exactly 2^k
gradient paths, and every DAG-minor edge between consecutive branch edges
has multiplicity 2 (the saturating product's overflow branch is taken once
the count passes 2^63).  ms_connect runs on that gradient under every
path-count schedule and its M21 / M21^T, n_saturated, M10 and M32 must equal
the oracle's, which is pinned on the CPU against the closed form, explicit
V-path enumeration and exact big-integer counts
(tests/test_oracle_saturation.py)."""
import numpy as np
import pytest

import cellgeom as CG
import diamonds
from oracle import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U64_MAX = (1 << 64) - 1


@pytest.fixture(scope="module", params=["ready", "power", "entry"])
def ctx(request):
    from paper_2009_03707_amd import msc
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = msc.Context()
    c.set_path_schedule({"ready": msc.MS_PATHS_READY, "power": msc.MS_PATHS_POWER,
                         "entry": msc.MS_PATHS_ENTRY}[request.param])
    yield c
    c.close()


def _oracle(k):
    grad, info = diamonds.build(k)
    nx, ny, nz = info["dims"]
    G = CG.Grid(np.zeros((nz, ny, nx), np.float32))
    crit = CG.critical_from_grad(G, grad)
    count = np.array([len(c) for c in crit], np.int64)
    ids = np.array([c for lst in crit for c in lst], np.uint32)
    cr = O.Critical(ids, np.zeros(len(ids), np.uint8), np.zeros(len(ids), np.float32),
                    np.zeros(len(ids), np.uint32), count)
    f0 = np.zeros(grad.shape, np.float32)
    p = O.ss_paths(f0, grad, cr)
    m10, m32 = O.se_arcs(f0, grad, cr)
    return grad, info, crit, cr, p, m10, m32


@pytest.mark.parametrize("k", [0, 1, 5, 12, 62, 63, 64, 65, 70, 90])
def test_diamond_chain_counts_saturate(ctx, k):
    from gpu_util import csr_np
    from paper_2009_03707_amd import msc
    grad, info, crit, cr, p, m10, m32 = _oracle(k)
    dev = torch.device("cuda")
    g = torch.from_numpy(grad.view(np.int32).copy()).to(dev)
    ids = torch.from_numpy(cr.id.view(np.int32).copy()).to(dev)
    arcs = ctx.connect(g, info["dims"], ids, cr.count.tolist())
    got = {nm: msc.csr_to_torch(getattr(arcs, nm), dev) for nm in ("m21t", "m21", "m10", "m32")}
    n_sat = int(arcs.n_saturated)
    torch.cuda.synchronize()
    rp, col, val = p.csr()
    g_rp, g_col, g_val = csr_np(got["m21t"])
    np.testing.assert_array_equal(g_rp, rp)
    np.testing.assert_array_equal(g_col, col)
    np.testing.assert_array_equal(g_val, val)
    # closed form for the chain's own entries: min(2^k, 2^64 - 1)
    s1, s2 = crit[1], crit[2]
    row = s1.index(info["source"])
    mine = {s2[int(c)]: int(v) for c, v in zip(g_col[g_rp[row]:g_rp[row + 1]], g_val[g_rp[row]:g_rp[row + 1]])}
    for e in info["ends"]:
        assert mine[e] == min(2 ** k, U64_MAX)
    assert mine[info["near"]] == 1
    want_sat = int((val == np.uint64(U64_MAX)).sum())
    assert n_sat == want_sat
    assert (want_sat >= 2) == (k >= 64)
    # M21 is the transpose of P, entry for entry
    t_rp, t_col, t_val = csr_np(got["m21"])
    order = np.lexsort((p.row, p.col))
    np.testing.assert_array_equal(t_col, p.row[order])
    np.testing.assert_array_equal(t_val, p.val[order])
    for nm, coo in (("m10", m10), ("m32", m32)):
        for a, b in zip(csr_np(got[nm]), coo.csr()):
            np.testing.assert_array_equal(a, b, err_msg=nm)
