"""Pins of the oracle's ascending and descending 3-manifold labels (CPU).

Section 3.4: the traversal that yields the saddle-extremum arcs also yields,
for every vertex, the minimum its (0,1) gradient path reaches (the ascending
manifolds of the minima) and, for every cube, the maximum its (2,3) gradient
path reaches (the descending manifolds of the maxima).  The oracle's labels
are pinned by:
  * a closed form for the vertex labels: under the lower-star rule a vertex
    that has a lower face neighbour is paired with the edge to its lowest
    one, so the (0,1) paths are discrete steepest descent over the six face
    neighbours and the labels are its basins (computed here from f alone);
  * an independent walk of every cube's (2,3) path over the gradient;
  * agreement with the M10 rows and M32 columns, which the V-path
    enumeration pins elsewhere;
  * every extremum labels itself, and maxima labels never decrease the
    highest vertex along a path.
"""
import numpy as np
import pytest

import cellgeom as CG
from oracle import oracle as O
from paper_2009_03707_amd import fields

NO = O.NO_LABEL


def steepest_descent_basins(f):
    """Vertex -> minimum vertex id by steepest descent over the 6 face
    neighbours in the order (value, id), -0.0 == +0.0."""
    nz, ny, nx = f.shape
    n = f.size
    val = f.reshape(-1).astype(np.float64) + 0.0
    vid = np.arange(n)
    # rank of every vertex in the total order (value, id)
    order = np.lexsort((vid, val))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    x, y, z = vid % nx, (vid // nx) % ny, vid // (nx * ny)
    best = vid.copy()
    for axis, size, coord, stride in ((0, nx, x, 1), (1, ny, y, nx), (2, nz, z, nx * ny)):
        for s in (-1, 1):
            ok = (coord + s >= 0) & (coord + s < size)
            nb = np.where(ok, vid + s * stride, vid)
            lower = ok & (rank[nb] < rank[best])
            best = np.where(lower, nb, best)
    root = best.copy()
    while True:
        nxt = root[root]
        if np.array_equal(nxt, root):
            break
        root = nxt
    return root


def _cube_walk(G, grad, crit):
    """Cube (by lowest corner) -> maximum cell id, or None (no cube / exit)."""
    maxs = set(crit[3])
    out = {}
    nx, ny, nz = G.n
    for w in range(G.nv):
        x, y, z = G.vxyz(w)
        if x + 1 >= nx or y + 1 >= ny or z + 1 >= nz:
            out[w] = None
            continue
        c = 8 * w + 7
        for _ in range(G.nv + 1):
            if c in maxs:
                break
            q = CG.partner(G, grad, c)
            assert q is not None and G.dim(q) == 2
            others = [d for d in G.cofacets(q) if d != c]
            if not others:
                c = None
                break
            c = others[0]
        out[w] = c
    return out


CASES = [("rand", (4, 4, 4), 0, 0), ("rand", (5, 4, 3), 1, 3), ("rand", (6, 6, 4), 2, 0),
         ("rand", (2, 6, 5), 6, 5), ("rand", (4, 1, 6), 7, 2), ("rand", (7, 1, 1), 8, 0),
         ("rand", (1, 1, 1), 9, 0), ("sine", 12, 0, 0), ("grf", (11, 9, 8), 3, 0), ("blob", (13, 12, 10), 4, 0)]


def _field(kind, dims, seed, levels):
    if kind == "rand":
        return fields.random_field(dims, seed=seed, levels=levels)
    if kind == "sine":
        return fields.sine_field(dims)
    if kind == "grf":
        return fields.grf_field(dims, seed=seed)
    return fields.blob_field(dims, nblobs=15, seed=seed)


@pytest.mark.parametrize("kind,dims,seed,levels", CASES)
def test_manifold_labels(kind, dims, seed, levels):
    f = _field(kind, dims, seed, levels)
    G = CG.Grid(f)
    cx = O.complex_(f)
    lo, hi = cx.min_label.reshape(-1), cx.max_label.reshape(-1)
    crit = CG.critical_from_grad(G, cx.grad)
    mins = [c >> 3 for c in crit[0]]
    # vertex labels: steepest-descent basins (closed form from f)
    basin = steepest_descent_basins(f)
    rank_of_min = {v: r for r, v in enumerate(mins)}
    assert set(np.unique(basin).tolist()) == set(mins)
    assert lo.tolist() == [rank_of_min[int(b)] for b in basin]
    # each minimum labels itself
    for r, v in enumerate(mins):
        assert lo[v] == r
    # cube labels: independent walk of the (2,3) paths
    walk = _cube_walk(G, cx.grad, crit)
    rank_of_max = {c: r for r, c in enumerate(crit[3])}
    for w in range(G.nv):
        want = NO if walk[w] is None else rank_of_max[walk[w]]
        assert hi[w] == want, w
        if walk[w] is not None:
            # the highest vertex never decreases along a (2,3) path
            assert G.key(G.maxv(walk[w])) >= G.key(G.maxv(8 * w + 7))
    for r, c in enumerate(crit[3]):
        assert hi[c >> 3] == r
    # agreement with the saddle-extremum arcs
    m10 = {}
    for e in crit[1]:
        u, v = G.verts(e)
        row = {}
        for t in (u, v):
            row[int(lo[t])] = row.get(int(lo[t]), 0) + 1
        m10[e] = row
    got10 = {}
    for r, c, v in zip(cx.m10.row, cx.m10.col, cx.m10.val):
        got10.setdefault(crit[1][int(r)], {})[int(c)] = int(v)
    assert {e: m10[e] for e in crit[1]} == {e: got10.get(e, {}) for e in crit[1]}
    m32 = {}
    for q in crit[2]:
        col = {}
        for c in G.cofacets(q):
            lab = int(hi[c >> 3])
            if lab != NO:
                col[lab] = col.get(lab, 0) + 1
        m32[q] = col
    got32 = {}
    for r, c, v in zip(cx.m32.row, cx.m32.col, cx.m32.val):
        got32.setdefault(crit[2][int(c)], {})[int(r)] = int(v)
    assert {q: m32[q] for q in crit[2]} == {q: got32.get(q, {}) for q in crit[2]}


def test_manifolds_partition_cells():
    """Every vertex carries exactly one minimum label and every cube at most
    one maximum label (NO_LABEL only for paths that leave the box); the label
    sets cover all extrema."""
    f = fields.grf_field((10, 9, 7), seed=5)
    cx = O.complex_(f)
    c = cx.crit.count
    lo, hi = cx.min_label, cx.max_label
    assert lo.max() < c[0] and np.unique(lo).size == c[0]
    real = hi[:-1, :-1, :-1].reshape(-1)
    assert (hi[-1, :, :] == NO).all() and (hi[:, -1, :] == NO).all() and (hi[:, :, -1] == NO).all()
    assert set(np.unique(real[real != NO]).tolist()) == set(range(int(c[3])))
