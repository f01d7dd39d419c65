"""A hand-built discrete gradient whose saddle-saddle path counts double k
times: a chain of k split-merge diamonds along a 2x2-vertex tube.

Test input only (used by the oracle pins and by the GPU parity tests alike);
it holds none of the method's arithmetic.  The cells and pairs are written
out here from the definitions of Section 2.2 (gradient pair, critical cell);
the splits and merges are the ones Section 3.1 and Figure 6 describe for
1-2 gradient paths.

Geometry (refined coordinates, X along the tube, Y and Z in {0, 1, 2}): the
tube has four faces F = Z0, Y0, Z2, Y2 (walked round in that order, so
consecutive faces share a corner line).  On face F, a "face edge" at even X
is the edge across the face at that X, a "face quad" at odd X is the quad of
the face between X-1 and X+1; the "cross quad" at even X is the yz quad
inside the tube; corner x-edges sit where two faces meet.

Diamond i (faces Fi = F[i % 4], Fn = F[(i + 1) % 4], at X = X0 + 2i) starts
at the branch edge b_i, the face edge of Fi at X:
  - the face quad of Fi at X+1 (R) is paired with the corner x-edge of
    Fi and Fn at X+1 (e1);
  - the cross quad at X (U) is paired with the face edge of Fn at X (e2);
  - the face quad of Fn at X+1 (M), which has both e1 and e2 as facets, is
    paired with the face edge of Fn at X+2, which is the next branch edge;
  - the other face quad of e2 (Fn at X-1) is paired with the cube at X-1, so
    that e1 and e2 each have exactly one way on (the DAG-minor edge from b_i
    to b_(i+1) then has multiplicity 2).
b_0 is critical (a 1-saddle); every cell not named above is critical.  The
last branch edge b_k has two critical cofacet quads (its "R" and "U"
positions): from b_0 each is reached by exactly 2^k gradient paths, and b_0
also reaches the critical face quad of F0 at X0-1 by one path.
"""
from __future__ import annotations

import numpy as np

FACES = ("Z0", "Y0", "Z2", "Y2")
X0 = 2


def _face_edge(face, X):
    return {"Z0": (X, 1, 0), "Y0": (X, 0, 1), "Z2": (X, 1, 2), "Y2": (X, 2, 1)}[face]


def _face_quad(face, X):
    return {"Z0": (X, 1, 0), "Y0": (X, 0, 1), "Z2": (X, 1, 2), "Y2": (X, 2, 1)}[face]


def _corner(fa, fb, X):
    y = {"Y0": 0, "Y2": 2}
    z = {"Z0": 0, "Z2": 2}
    fy = fa if fa in y else fb
    fz = fa if fa in z else fb
    return (X, y[fy], z[fz])


def dims_for(k: int):
    """(nx, ny, nz) vertex counts of the tube that holds k diamonds."""
    return (k + 3, 2, 2)


def _cell_id(n, r):
    X, Y, Z = r
    w = (X >> 1) + n[0] * ((Y >> 1) + n[1] * (Z >> 1))
    return 8 * w + (X & 1) + 2 * (Y & 1) + 4 * (Z & 1)


def build(k: int):
    """Returns (grad uint32 (nz, ny, nx), info) for a chain of k >= 0 diamonds.

    info: dict with the cell ids of the source 1-saddle b0 ("source"), the two
    end 2-saddles ("ends"), the 2-saddle next to the source ("near"), and the
    pairs as a list of refined-coordinate tuples ("pairs")."""
    n = dims_for(k)
    pairs = []
    for i in range(k):
        X = X0 + 2 * i
        fi, fn = FACES[i % 4], FACES[(i + 1) % 4]
        R = _face_quad(fi, X + 1)
        e1 = _corner(fi, fn, X + 1)
        U = (X, 1, 1)
        e2 = _face_edge(fn, X)
        M = _face_quad(fn, X + 1)
        b_next = _face_edge(fn, X + 2)
        D = _face_quad(fn, X - 1)
        cube = (X - 1, 1, 1)
        pairs += [(R, e1), (U, e2), (M, b_next), (D, cube)]
    # every cell starts critical (nibble 8) or absent (7)
    nx, ny, nz = n
    word = np.zeros((nz, ny, nx), np.uint32)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                w = 0
                for kk in range(8):
                    a, b, c = kk & 1, (kk >> 1) & 1, (kk >> 2) & 1
                    exists = (not a or x + 1 < nx) and (not b or y + 1 < ny) and (not c or z + 1 < nz)
                    w |= (8 if exists else 7) << (4 * kk)
                word[z, y, x] = w
    flat = word.reshape(-1)
    used = set()

    def put(r, p):
        cid = _cell_id(n, r)
        assert cid not in used, ("cell paired twice", r)
        used.add(cid)
        d = [p[a] - r[a] for a in range(3)]
        assert sorted(abs(t) for t in d) == [0, 0, 1], (r, p)
        axis = next(a for a in range(3) if d[a])
        nib = 1 + 2 * axis + (0 if d[axis] > 0 else 1)
        wv, kk = cid >> 3, cid & 7
        flat[wv] = (int(flat[wv]) & ~(15 << (4 * kk))) | (nib << (4 * kk))

    for a, b in pairs:
        for r in (a, b):
            assert all(0 <= r[t] <= 2 * n[t] - 2 for t in range(3)), ("outside the tube", r)
        put(a, b)
        put(b, a)
    Xk = X0 + 2 * k
    fk = FACES[k % 4]
    info = {
        "source": _cell_id(n, _face_edge(FACES[0], X0)),
        "ends": sorted([_cell_id(n, _face_quad(fk, Xk + 1)), _cell_id(n, (Xk, 1, 1))]),
        "near": _cell_id(n, _face_quad(FACES[0], X0 - 1)),
        "pairs": pairs,
        "dims": n,
    }
    return word, info
