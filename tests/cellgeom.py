"""Independent Python statements of the cubical-complex geometry and of the
checks that pin the oracle (brute force, invariants, homology).

This is test code.  It does not call the oracle's C code for anything it
checks: it decodes gradient words and critical lists on its own, from the
definitions in Section 2.2 of the paper (gradient pair, critical cell, index,
V-path) and from the conventions of the contract (cell ids, nibble encoding,
vertex order with id tie-break).
"""
from __future__ import annotations

import itertools

import numpy as np

CRIT = 8
NOCELL = 7


class Grid:
    def __init__(self, f: np.ndarray):
        self.f = np.ascontiguousarray(f, dtype=np.float32)
        nz, ny, nx = self.f.shape
        self.n = (nx, ny, nz)
        self.nv = nx * ny * nz
        self.flat = self.f.reshape(-1)

    # vertices --------------------------------------------------------------
    def vid(self, x, y, z):
        return x + self.n[0] * (y + self.n[1] * z)

    def vxyz(self, v):
        nx, ny, _ = self.n
        return v % nx, (v // nx) % ny, v // (nx * ny)

    def key(self, v):
        """Vertex order key: value (with -0.0 == +0.0), then id."""
        return (float(self.flat[v]) + 0.0, v)

    # cells -----------------------------------------------------------------
    def cell_id(self, r):
        X, Y, Z = r
        return 8 * self.vid(X >> 1, Y >> 1, Z >> 1) + (X & 1) + 2 * (Y & 1) + 4 * (Z & 1)

    def cell_ref(self, cid):
        x, y, z = self.vxyz(cid >> 3)
        k = cid & 7
        return (2 * x + (k & 1), 2 * y + ((k >> 1) & 1), 2 * z + ((k >> 2) & 1))

    def in_range(self, r):
        return all(0 <= r[a] <= 2 * self.n[a] - 2 for a in range(3))

    def dim(self, cid):
        return bin(cid & 7).count("1")

    def verts(self, cid):
        r = self.cell_ref(cid)
        rng = [(r[a] >> 1,) if r[a] % 2 == 0 else (r[a] >> 1, (r[a] >> 1) + 1) for a in range(3)]
        return [self.vid(x, y, z) for z in rng[2] for y in rng[1] for x in rng[0]]

    def maxv(self, cid):
        return max(self.verts(cid), key=self.key)

    def step(self, cid, axis, sign):
        r = list(self.cell_ref(cid))
        r[axis] += sign
        return self.cell_id(r) if self.in_range(r) else None

    def facets(self, cid):
        r = self.cell_ref(cid)
        out = []
        for a in range(3):
            if r[a] % 2 == 1:
                for s in (-1, 1):
                    out.append(self.step(cid, a, s))
        return out

    def cofacets(self, cid):
        r = self.cell_ref(cid)
        out = []
        for a in range(3):
            if r[a] % 2 == 0:
                for s in (-1, 1):
                    c = self.step(cid, a, s)
                    if c is not None:
                        out.append(c)
        return out

    def all_cells(self):
        nx, ny, nz = self.n
        for Z in range(2 * nz - 1):
            for Y in range(2 * ny - 1):
                for X in range(2 * nx - 1):
                    yield self.cell_id((X, Y, Z))


def nib(grad, cid):
    return (int(grad.reshape(-1)[cid >> 3]) >> (4 * (cid & 7))) & 15


def partner(G: Grid, grad, cid):
    """Partner cell id, or None when the cell is critical."""
    v = nib(grad, cid)
    if v >= CRIT:
        return None
    assert 1 <= v <= 6, (cid, v)
    axis, sign = (v - 1) // 2, (-1 if (v - 1) % 2 else 1)
    p = G.step(cid, axis, sign)
    assert p is not None
    return p


# ---- invariants of a discrete gradient ------------------------------------------

def check_gradient_valid(G: Grid, grad, lower_star: bool = True):
    """Every existing cell is critical or in exactly one pair with a facet or
    cofacet; pairs are symmetric; both cells of a pair share their highest
    vertex (lower-star property); a critical cell's encoded corner is its
    highest vertex; cells that do not exist are marked as such; and no
    (i, i+1) V-path closes a cycle.  With lower_star=False the two checks
    that involve field values are skipped (for hand-built gradients)."""
    g = grad.reshape(-1)
    existing = set(G.all_cells())
    for w in range(G.nv):
        for k in range(8):
            cid = 8 * w + k
            v = (int(g[w]) >> (4 * k)) & 15
            if cid not in existing:
                assert v == NOCELL, (cid, v)
                continue
            assert v != 0 and v != NOCELL, (cid, v)
            if v >= CRIT:
                if not lower_star:
                    continue
                x, y, z = G.vxyz(w)
                d = v - CRIT
                top = G.vid(x + (d & 1), y + ((d >> 1) & 1), z + ((d >> 2) & 1))
                assert top == G.maxv(cid), (cid, top)
            else:
                p = partner(G, grad, cid)
                assert partner(G, grad, p) == cid, (cid, p)
                if lower_star:
                    assert G.maxv(p) == G.maxv(cid), (cid, p)
    # acyclicity of V-paths in each dimension pair, by Kahn's algorithm
    for i in range(3):
        nodes = [c for c in existing if G.dim(c) == i]
        succ = {c: [] for c in nodes}
        for a in nodes:
            b = partner(G, grad, a)
            if b is None or G.dim(b) != i + 1:
                continue
            for a2 in G.facets(b):
                if a2 != a:
                    succ[a].append(a2)
        indeg = {c: 0 for c in nodes}
        for a in nodes:
            for b in succ[a]:
                indeg[b] += 1
        q = [c for c in nodes if indeg[c] == 0]
        seen = 0
        while q:
            a = q.pop()
            seen += 1
            for b in succ[a]:
                indeg[b] -= 1
                if indeg[b] == 0:
                    q.append(b)
        assert seen == len(nodes), f"cycle among ({i},{i + 1}) V-paths"


def critical_from_grad(G: Grid, grad):
    """Critical cell ids per index, each sorted by id (decoded here)."""
    out = [[], [], [], []]
    for cid in sorted(G.all_cells()):
        if nib(grad, cid) >= CRIT:
            out[G.dim(cid)].append(cid)
    return out


# ---- lower-link homology (brute force on the octahedral link) ----------------------

def lower_link_betti(G: Grid, v):
    """Reduced Betti numbers (b_-1, b_0, b_1, b_2) of the lower link of v.

    The link of a vertex in the cubical grid is (part of) an octahedron:
    link vertices are the edges at v, link edges the quads at v, link
    triangles the cubes at v.  A link cell is lower when every vertex of the
    corresponding grid cell other than v precedes v."""
    x, y, z = G.vxyz(v)
    kv = G.key(v)

    def lower(off):
        # all vertices of the cell spanned by offset `off` (other than v) are lower
        rng = [(0,) if o == 0 else (0, o) for o in off]
        for d in itertools.product(*rng):
            if d == (0, 0, 0):
                continue
            p = (x + d[0], y + d[1], z + d[2])
            if not all(0 <= p[a] < G.n[a] for a in range(3)):
                return False
            if not G.key(G.vid(*p)) < kv:
                return False
        return True

    axes = [(a, s) for a in range(3) for s in (-1, 1)]

    def off_of(items):
        o = [0, 0, 0]
        for a, s in items:
            o[a] = s
        return tuple(o)

    V = [av for av in axes if lower(off_of([av]))]
    E = [(p, q) for p, q in itertools.combinations(axes, 2)
         if p[0] != q[0] and lower(off_of([p, q]))]
    F = [t for t in itertools.combinations(axes, 3)
         if len({a for a, _ in t}) == 3 and lower(off_of(t))]
    if not V:
        return (1, 0, 0, 0)
    parent = {a: a for a in V}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for p, q in E:
        parent[find(p)] = find(q)
    b0 = len({find(a) for a in V})
    b2 = 1 if len(F) == 8 else 0
    chi = len(V) - len(E) + len(F)
    b1 = b0 - chi + b2
    return (0, b0 - 1, b1, b2)


# ---- V-path enumeration (brute force from the definition) ---------------------------

def vpath_counts(G: Grid, grad, crit):
    """Counts of maximal V-paths between critical cells of consecutive index,
    enumerated explicitly (no memoisation).  crit = per-index sorted id lists.
    Returns dicts keyed by (higher cell id, lower cell id)."""
    crit_set = [set(c) for c in crit]
    res = [dict(), dict(), dict()]  # index i+1 -> i, for i = 0, 1, 2

    def walk(i, alpha, src, acc):
        # alpha: an i-cell reached from a facet step; continue the V-path
        if alpha in crit_set[i]:
            acc[(src, alpha)] = acc.get((src, alpha), 0) + 1
            return
        beta = partner(G, grad, alpha)
        if beta is None or G.dim(beta) != i + 1:
            return  # paired downward: the path cannot continue
        for a2 in G.facets(beta):
            if a2 != alpha:
                walk(i, a2, src, acc)

    for i in range(3):
        for s in crit[i + 1]:
            for a in G.facets(s):
                walk(i, a, s, res[i])
    return res


# ---- exact path counts (arbitrary precision) -------------------------------------

def dag_out(G: Grid, grad, e):
    """Out-neighbours of edge e in the DAG of 1-2 gradient pairs (Section 3.1,
    Figure 6 (d)): for each cofacet quad Q other than the quad e is paired
    with, ("s2", Q) if Q is critical, ("e", e2) if Q is paired with edge e2;
    quads paired with cubes give nothing."""
    ve = partner(G, grad, e)
    out = []
    for q in G.cofacets(e):
        if q == ve:
            continue
        p = partner(G, grad, q)
        if p is None:
            out.append(("s2", q))
        elif G.dim(p) == 1:
            out.append(("e", p))
    return out


def exact_path_counts(G: Grid, grad, sources):
    """{(s1, s2): number of directed DAG paths} for the given 1-saddles, in
    Python integers (no bound), by memoised recursion over the DAG."""
    import sys
    sys.setrecursionlimit(max(10000, sys.getrecursionlimit()))
    memo = {}

    def counts(e):
        if e in memo:
            return memo[e]
        acc = {}
        for kind, t in dag_out(G, grad, e):
            if kind == "s2":
                acc[t] = acc.get(t, 0) + 1
            else:
                for q, c in counts(t).items():
                    acc[q] = acc.get(q, 0) + c
        memo[e] = acc
        return acc

    res = {}
    for s in sources:
        for q, c in counts(s).items():
            res[(s, q)] = c
    return res


# ---- GF(2) linear algebra ---------------------------------------------------------

def gf2_rank(m: np.ndarray) -> int:
    a = (np.asarray(m) % 2).astype(bool).copy()
    if a.size == 0:
        return 0
    rows, cols = a.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if a[i, c]:
                piv = i
                break
        if piv is None:
            continue
        if piv != r:
            a[[r, piv]] = a[[piv, r]]
        mask = a[:, c].copy()
        mask[r] = False
        a[mask] ^= a[r]
        r += 1
        if r == rows:
            break
    return r
