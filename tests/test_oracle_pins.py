"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties the oracle to something other than itself:
  * hand-derived worked examples (tests/golden/hand_*.json);
  * closed forms: constant/monotone fields, 1D textbook extrema, separable
    integer fields, the sine-field counts (tests/golden/sine32_counts.json);
  * invariants of a discrete gradient (Section 2.2): valid pairing, lower-star
    property, acyclic V-paths, Euler characteristic of the box;
  * brute force: per-vertex lower-link homology; explicit V-path enumeration
    for the saddle-extremum and saddle-saddle counts (Sections 3.1, 3.4);
  * Morse homology over Z2: the arc matrices are boundary maps whose
    composition vanishes and whose homology is that of a point.
"""
import json
import os

import numpy as np
import pytest

import cellgeom as CG
from oracle import oracle as O
from paper_2009_03707_amd import fields

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _coo_triples(c):
    return [(int(r), int(k), int(v)) for r, k, v in zip(c.row, c.col, c.val)]


# ---------------------------------------------------------------- worked examples

@pytest.mark.parametrize("name", ["hand_2x2x1", "hand_2x2x2"])
def test_hand_derived_examples(name):
    d = json.load(open(os.path.join(GOLD, name + ".json")))
    nx, ny, nz = d["dims"]
    f = np.array(d["f_by_vid"], np.float32).reshape(nz, ny, nx)
    cx = O.complex_(f)
    assert [int(x) for x in cx.grad.reshape(-1)] == [int(h, 16) for h in d["grad_by_vid"]]
    assert cx.crit.id.tolist() == d["critical_ids"]
    assert cx.crit.index.tolist() == d["critical_index"]
    assert _coo_triples(cx.m10) == [tuple(t) for t in d["m10"]]
    assert _coo_triples(cx.m32) == [tuple(t) for t in d["m32"]]
    assert _coo_triples(cx.p) == [tuple(t) for t in d["p"]]


# ---------------------------------------------------------------- closed forms

DIMS_SMALL = [(1, 1, 1), (5, 1, 1), (1, 4, 1), (1, 1, 6), (3, 4, 1), (3, 1, 4), (1, 3, 3), (3, 4, 5), (6, 5, 2)]


@pytest.mark.parametrize("dims", DIMS_SMALL)
@pytest.mark.parametrize("kind", ["const", "inc", "dec", "negzero"])
def test_constant_and_monotone_fields(dims, kind):
    nx, ny, nz = dims
    n = nx * ny * nz
    if kind == "const":
        f = np.full(n, 0.5, np.float32)
    elif kind == "inc":
        f = np.arange(n, dtype=np.float32)
    elif kind == "dec":
        f = -np.arange(n, dtype=np.float32)
    else:  # mixed signed zeros compare equal: id order decides
        f = np.where(np.arange(n) % 2 == 0, np.float32(0.0), np.float32(-0.0)).astype(np.float32)
    f = f.reshape(nz, ny, nx)
    cx = O.complex_(f)
    gmin = n - 1 if kind == "dec" else 0
    assert cx.crit.count.tolist() == [1, 0, 0, 0]
    assert cx.crit.id.tolist() == [8 * gmin]
    assert cx.crit.vmax.tolist() == [gmin]
    assert len(cx.m10.val) == len(cx.m32.val) == len(cx.p.val) == 0


def _textbook_1d(vals):
    """Local minima (an endpoint counts when its only neighbour is higher) and,
    for each interior strict maximum i, the nearest minimum on each side."""
    n = len(vals)
    mins = [i for i in range(n)
            if (i == 0 or vals[i - 1] > vals[i]) and (i == n - 1 or vals[i + 1] > vals[i])]
    arcs = []
    for i in range(1, n - 1):
        if vals[i - 1] < vals[i] > vals[i + 1]:
            lft = i - 1
            while lft > 0 and vals[lft - 1] < vals[lft]:
                lft -= 1
            rgt = i + 1
            while rgt < n - 1 and vals[rgt + 1] < vals[rgt]:
                rgt += 1
            hi_side = i - 1 if vals[i - 1] > vals[i + 1] else i + 1
            arcs.append((min(i, hi_side), lft, rgt))
    return mins, arcs


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("seed", range(6))
def test_1d_grids_match_textbook(axis, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    vals = rng.permutation(n).astype(np.float32)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    f = vals.reshape(shape)
    cx = O.complex_(f)
    mins, arcs = _textbook_1d(list(vals))
    stride = 8
    bit = 1 << axis
    assert cx.crit.count.tolist() == [len(mins), len(arcs), 0, 0]
    assert cx.crit.of_index(0).tolist() == [stride * i for i in mins]
    assert cx.crit.of_index(1).tolist() == [stride * lo + bit for lo, _, _ in arcs]
    rank = {m: r for r, m in enumerate(mins)}
    expect = []
    for r, (_, lft, rgt) in enumerate(arcs):
        a, b = sorted((rank[lft], rank[rgt]))
        expect += [(r, a, 1), (r, b, 1)]
    assert _coo_triples(cx.m10) == expect


def _count_poly_1d(seq):
    n = len(seq)
    m = sum(1 for i in range(n) if (i == 0 or seq[i - 1] > seq[i]) and (i == n - 1 or seq[i + 1] > seq[i]))
    M = sum(1 for i in range(1, n - 1) if seq[i - 1] < seq[i] > seq[i + 1])
    return m, M


def _distinct_neighbours_seq(rng, n):
    s = [int(rng.integers(0, 10))]
    while len(s) < n:
        v = int(rng.integers(0, 10))
        if v != s[-1]:
            s.append(v)
    return np.array(s, dtype=np.float64)


@pytest.mark.parametrize("dims", [(7, 5, 3), (12, 9, 6), (1, 8, 9), (2, 2, 13), (40, 30, 20)])
@pytest.mark.parametrize("seed", range(3))
def test_separable_integer_fields_count_polynomial(dims, seed):
    rng = np.random.default_rng(100 + seed)
    nx, ny, nz = dims
    a, b, c = (_distinct_neighbours_seq(rng, n) for n in (nx, ny, nz))
    f = (a[None, None, :] + b[None, :, None] + c[:, None, None]).astype(np.float32)
    g = O.gradient(f)
    cr = O.critical(f, g)
    poly = np.array([1])
    for seq in (a, b, c):
        m, M = _count_poly_1d(list(seq))
        poly = np.polymul(poly, np.array([M, m]))  # highest degree first
    coeffs = list(poly[::-1]) + [0] * 4
    assert cr.count.tolist() == [int(x) for x in coeffs[:4]]


def test_sine_field_counts():
    gold = json.load(open(os.path.join(GOLD, "sine32_counts.json")))
    f = fields.sine_field(32, seed=0)
    t = np.linspace(0.0, 2 * np.pi, 32)
    poly = np.array([1])
    for k in (3, 5, 7):
        m, M = _count_poly_1d(list(np.sin(k * t)))
        poly = np.polymul(poly, np.array([M, m]))
    expect = [int(x) for x in poly[::-1]]
    assert expect == gold["counts"]
    g = O.gradient(f)
    cr = O.critical(f, g)
    assert cr.count.tolist() == gold["counts"]


# ---------------------------------------------------------------- brute force and invariants

RANDOM_CASES = [((4, 4, 4), 0, 0), ((5, 4, 3), 1, 3), ((6, 6, 4), 2, 0), ((3, 5, 5), 3, 4),
                ((5, 5, 5), 4, 2), ((6, 3, 4), 5, 0), ((2, 6, 5), 6, 5), ((4, 1, 6), 7, 2),
                ((6, 6, 4), 8, 6), ((5, 5, 4), 9, 0)]


@pytest.mark.parametrize("dims,seed,levels", RANDOM_CASES)
def test_random_small_fields_brute_force(dims, seed, levels):
    f = fields.random_field(dims, seed=seed, levels=levels)
    G = CG.Grid(f)
    cx = O.complex_(f)
    # gradient invariants
    CG.check_gradient_valid(G, cx.grad)
    crit = CG.critical_from_grad(G, cx.grad)
    assert cx.crit.id.tolist() == sum(crit, [])
    assert cx.crit.count.tolist() == [len(c) for c in crit]
    assert int(cx.crit.count @ np.array([1, -1, 1, -1])) == 1
    for cid, vm, val in zip(cx.crit.id, cx.crit.vmax, cx.crit.value):
        assert int(vm) == G.maxv(int(cid))
        assert np.float32(val).tobytes() == f.reshape(-1)[int(vm)].tobytes()
    # per-vertex perfection: critical cells in L(x) = reduced homology of the lower link
    per = np.zeros((G.nv, 4), int)
    for cid, vm in zip(cx.crit.id, cx.crit.vmax):
        per[int(vm), G.dim(int(cid))] += 1
    for v in range(G.nv):
        assert tuple(per[v]) == CG.lower_link_betti(G, v), v
    # V-path enumeration vs the oracle's arc matrices
    vp = CG.vpath_counts(G, cx.grad, crit)
    r10 = {(crit[1][r], crit[0][c]): int(v) for r, c, v in _coo_triples(cx.m10)}
    assert r10 == vp[0]
    r32 = {(crit[3][r], crit[2][c]): int(v) for r, c, v in _coo_triples(cx.m32)}
    assert r32 == vp[2]
    rP = {(crit[2][c], crit[1][r]): int(v) for r, c, v in _coo_triples(cx.p)}
    assert rP == vp[1]


def _morse_z2_checks(cx):
    c = cx.crit.count
    d1 = cx.m10.dense().T % 2          # C1 -> C0
    d2 = cx.p.dense() % 2              # C2 -> C1
    d3 = cx.m32.dense().T % 2          # C3 -> C2
    assert not ((d1.astype(np.int64) @ d2.astype(np.int64)) % 2).any()
    assert not ((d2.astype(np.int64) @ d3.astype(np.int64)) % 2).any()
    r1, r2, r3 = CG.gf2_rank(d1), CG.gf2_rank(d2), CG.gf2_rank(d3)
    betti = (c[0] - r1, c[1] - r1 - r2, c[2] - r2 - r3, c[3] - r3)
    assert tuple(int(b) for b in betti) == (1, 0, 0, 0)


@pytest.mark.parametrize("dims,seed,levels", RANDOM_CASES)
def test_morse_homology_z2_small(dims, seed, levels):
    cx = O.complex_(fields.random_field(dims, seed=seed, levels=levels))
    _morse_z2_checks(cx)


@pytest.mark.parametrize("make", ["sine16", "grf12", "blob14", "rand9"])
def test_morse_homology_z2_medium(make):
    if make == "sine16":
        f = fields.sine_field(16)
    elif make == "grf12":
        f = fields.grf_field((12, 11, 10), seed=3)
    elif make == "blob14":
        f = fields.blob_field((14, 13, 12), nblobs=20, seed=4)
    else:
        f = fields.random_field((9, 8, 7), seed=11, levels=4)
    cx = O.complex_(f)
    assert int(cx.crit.count @ np.array([1, -1, 1, -1])) == 1
    _morse_z2_checks(cx)
    # M10 rows sum to 2 (each 1-saddle has two descending paths); each
    # 2-saddle has at most two cofacet cubes
    if len(cx.m10.val):
        assert (np.bincount(cx.m10.row, weights=cx.m10.val.astype(float), minlength=cx.m10.shape[0]) == 2).all()
    if len(cx.m32.val):
        assert (np.bincount(cx.m32.col, weights=cx.m32.val.astype(float), minlength=cx.m32.shape[1]) <= 2).all()


def test_direct_saddle_adjacency():
    """A 1-saddle that is a facet of a 2-saddle has a direct path to it
    (caption of Figure 6: the two-node component of the DAG)."""
    found = 0
    for seed in range(6):
        f = fields.random_field((6, 6, 6), seed=seed)
        G = CG.Grid(f)
        cx = O.complex_(f)
        s1 = cx.crit.of_index(1).tolist()
        s2 = cx.crit.of_index(2).tolist()
        rank2 = {q: i for i, q in enumerate(s2)}
        P = {(r, c): v for r, c, v in _coo_triples(cx.p)}
        for r, e in enumerate(s1):
            for q in G.cofacets(e):
                if q in rank2:
                    found += 1
                    assert P.get((r, rank2[q]), 0) >= 1
    assert found > 0


def test_full_gradient_passes_invariants_on_sine_and_grf():
    for f in (fields.sine_field(12), fields.grf_field((10, 9, 8), seed=1)):
        G = CG.Grid(f)
        g = O.gradient(f)
        CG.check_gradient_valid(G, g)
        per = np.zeros((G.nv, 4), int)
        cr = O.critical(f, g)
        for cid, vm in zip(cr.id, cr.vmax):
            per[int(vm), G.dim(int(cid))] += 1
        for v in range(G.nv):
            assert tuple(per[v]) == CG.lower_link_betti(G, v)


# ---------------------------------------------------------------- lazy accessors

def test_lazy_accessors_agree_with_full_results():
    f = fields.blob_field((11, 10, 9), nblobs=8, seed=2)
    cx = O.complex_(f)
    flat = cx.grad.reshape(-1)
    for v in range(0, flat.size, 7):
        assert O.word_lazy(f, v) == int(flat[v])
    s1 = cx.crit.of_index(1)
    mins = cx.crit.of_index(0)
    for r in range(0, len(s1), 3):
        got = sorted(O.m10_row_lazy(f, int(s1[r])).tolist())
        row = [(c, v) for rr, c, v in _coo_triples(cx.m10) if rr == r]
        exp = sorted(sum([[int(mins[c]) // 8] * v for c, v in row], []))
        assert got == exp
    s2 = cx.crit.of_index(2)
    rows = O.ss_rows_lazy(f, s1.astype(np.int64))
    lazy = {(int(r), int(c)): int(v) for r, c, v in zip(rows.row, rows.col, rows.val)}
    full = {(int(s1[r]), int(s2[c])): v for r, c, v in _coo_triples(cx.p)}
    assert lazy == full


def test_nonfinite_input_is_rejected():
    f = fields.random_field((3, 3, 3), seed=0)
    for bad in (np.nan, np.inf, -np.inf):
        g = f.copy()
        g[1, 1, 1] = bad
        with pytest.raises(O.OracleError) as e:
            O.gradient(g)
        assert e.value.code == O.ORC_ERR_NONFINITE
