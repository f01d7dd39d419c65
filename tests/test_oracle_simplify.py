"""Pins of the oracle's MS-complex graph and serial simplification (CPU).

* 1D closed form: on a path graph the persistence-ordered cancellation of
  saddle-minimum arcs realises the elder rule of 0-dimensional persistence
  (every merge vertex kills the younger of the two components it joins),
  computed here independently by union-find over the vertices in the order
  (value, id) -- the textbook algorithm, no MS complex involved.
* A hand-worked 1D example (tests/golden/simplify_1d_hand.json).
* Invariants on 3D fields: cancelling an index-adjacent pair keeps the Euler
  characteristic (= 1 on a box); the simplified complex is still a chain
  complex with the homology of a box over Z_2 (Morse homology: boundary
  matrices are the multiplicities mod 2, d1 d2 = d2 d3 = 0 and Betti numbers
  (1, 0, 0, 0)); no cancellable arc below the threshold is left; every
  logged cancellation was of a multiplicity-1 arc below the threshold.
* The graph itself is the oracle's arc matrices stored at both ends.
"""
import json
import os

import numpy as np
import pytest

import cellgeom as CG
from oracle import oracle as O
from oracle import simplify as S
from paper_2009_03707_amd import fields

HERE = os.path.dirname(os.path.abspath(__file__))


def elder_pairs(f1d):
    """0-dim persistence pairs (merge vertex, dying minimum) of a 1D
    sublevel-set filtration, vertex order (value, id)."""
    n = len(f1d)
    order = sorted(range(n), key=lambda v: (float(f1d[v]) + 0.0, v))
    parent = {}
    birth = {}

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    key = {v: (float(f1d[v]) + 0.0, v) for v in range(n)}
    pairs = set()
    for v in order:
        parent[v] = v
        birth[v] = v
        roots = {find(u) for u in (v - 1, v + 1) if 0 <= u < n and u in parent and u != v}
        roots = sorted(roots, key=lambda r: key[birth[r]])
        if not roots:
            continue
        # join v to the oldest component; a second component dies at v
        old = roots[0]
        parent[v] = old
        for r in roots[1:]:
            pairs.add((v, birth[r]))
            parent[r] = old
    return pairs


@pytest.mark.parametrize("n,seed", [(5, 0), (9, 1), (17, 2), (40, 3), (101, 4), (300, 5)])
def test_1d_cancellations_are_the_elder_pairs(n, seed):
    f = np.random.default_rng(seed).permutation(n).astype(np.float32).reshape(1, 1, n)
    cx = O.complex_(f)
    g = S.simplify(S.from_complex(cx), float("inf"))
    got = set()
    for u, l, p in g.log:
        assert g.index[u] == 1 and g.index[l] == 0
        # the critical edge's highest vertex is the merge vertex; the minimum's cell is 8 * vertex
        got.add((int(cx.crit.vmax[u]), g.cell[l] >> 3))
    assert got == elder_pairs(f.reshape(-1))
    # one minimum survives: the global one
    live = [i for i in range(len(g.index)) if g.alive[i]]
    assert len(live) == 1 and g.cell[live[0]] >> 3 == int(np.argmin(f.reshape(-1)))


def test_1d_hand_example():
    """Worked by hand from the cancellation rule (golden file)."""
    gold = json.load(open(os.path.join(HERE, "golden", "simplify_1d_hand.json")))
    f = np.array(gold["f"], np.float32).reshape(1, 1, -1)
    cx = O.complex_(f)
    g = S.from_complex(cx)
    assert g.cell == gold["cells"]
    assert {str(u): {str(l): m for l, m in d.items()} for u, d in enumerate(g.down) if d} == gold["arcs"]
    S.simplify(g, float("inf"))
    assert [[u, l, p] for u, l, p in g.log] == gold["log"]


def _betti_z2(g):
    live = [i for i in range(len(g.index)) if g.alive[i]]
    by = {k: [i for i in live if g.index[i] == k] for k in range(4)}
    pos = {k: {n: j for j, n in enumerate(by[k])} for k in range(4)}
    d = {}
    for k in (1, 2, 3):
        m = np.zeros((len(by[k - 1]), len(by[k])), np.uint8)
        for u in by[k]:
            for l, mult in g.live_arcs(u, "down").items():
                m[pos[k - 1][l], pos[k][u]] = mult & 1
        d[k] = m
    for k in (1, 2):
        prod = (d[k].astype(np.int64) @ d[k + 1].astype(np.int64)) % 2 if d[k].size and d[k + 1].size else None
        if prod is not None:
            assert not prod.any(), f"d{k} d{k + 1} != 0 mod 2"
    r = {k: CG.gf2_rank(d[k]) if d[k].size else 0 for k in (1, 2, 3)}
    n = [len(by[k]) for k in range(4)]
    return (n[0] - r[1], n[1] - r[1] - r[2], n[2] - r[2] - r[3], n[3] - r[3])


CASES = [((6, 5, 4), 0, 0), ((7, 7, 3), 1, 3), ((9, 6, 5), 2, 0), ((12, 1, 9), 3, 0), ("sine16", 0, 0),
         ("grf", 5, 0)]


def _f(dims, seed, levels):
    if dims == "sine16":
        return fields.sine_field(16)
    if dims == "grf":
        return fields.grf_field((14, 12, 10), seed=seed)
    return fields.random_field(dims, seed=seed, levels=levels)


@pytest.mark.parametrize("dims,seed,levels", CASES)
@pytest.mark.parametrize("thr", [0.05, 0.3, float("inf")])
def test_invariants_after_simplification(dims, seed, levels, thr):
    f = _f(dims, seed, levels)
    cx = O.complex_(f)
    g = S.from_complex(cx)
    # the graph stores every arc at both ends, as the oracle's matrices give it
    for u, d in enumerate(g.down):
        for l, m in d.items():
            assert g.up[l][u] == m and g.index[u] == g.index[l] + 1
    replay = S.from_complex(cx)
    S.simplify(g, thr)
    n = [sum(1 for i in range(len(g.index)) if g.alive[i] and g.index[i] == k) for k in range(4)]
    assert n[0] - n[1] + n[2] - n[3] == 1
    assert _betti_z2(g) == (1, 0, 0, 0)
    for u in range(len(g.index)):
        for l, m in g.live_arcs(u, "down").items():
            assert not (m == 1 and g.pers(u, l) < thr), "a cancellable arc is left"
    # every logged step was valid when it was made, and the steps rebuild g
    for u, l, p in g.log:
        assert S.valid(replay, u, l, thr) and p == replay.pers(u, l)
        S.cancel(replay, u, l)
    assert S.live_graph(replay) == S.live_graph(g)
    # the first cancellation is the least valid arc of the unsimplified graph
    if g.log:
        g0 = S.from_complex(cx)
        first = min((g0.pers(u, l), u, l) for u, d in enumerate(g0.down) for l in d if S.valid(g0, u, l, thr))
        assert (g.log[0][2], g.log[0][0], g.log[0][1]) == first


def test_strangled_pairs_are_kept():
    """A 1-saddle whose two descending paths reach the same minimum
    (multiplicity 2) is never cancelled with it."""
    f = fields.random_field((8, 8, 6), seed=11, levels=3)
    cx = O.complex_(f)
    g = S.from_complex(cx)
    doubles = {(u, l) for u in range(len(g.index)) for l, m in g.down[u].items() if m == 2 and g.index[u] == 1}
    assert doubles, "the field should have a 1-saddle with both paths to one minimum"
    S.simplify(g, float("inf"))
    assert not {(u, l) for u, l, _ in g.log} & doubles
