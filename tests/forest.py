"""Checks of manifold labels that hold at any size (Section 3.4): the
labels of vertices (minima) and cubes (maxima) form the forest the gradient
words define.  A minimum or maximum labels itself with its rank; every other
vertex or cube carries the label of its successor along the (0,1) or (2,3)
path, or the exit label where a (2,3) path leaves the grid.  With the roots
given, this fixes every label, so it checks labels where no oracle run fits
(used by the GPU tests of out-of-core fields, and itself tested on the
oracle's labels in tests/test_forest_check.py)."""
import numpy as np

EXIT64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def widen_exit(lab):
    """32-bit labels widened to 64 bits, the exit label to all ones."""
    out = lab.astype(np.uint64)
    out[lab == 0xFFFFFFFF] = EXIT64
    return out


def check_forest(grad, lab, roots, nibble, cube, z0, z1, exit_label=None):
    """Labels of rows [z0, z1) of `lab` (nz, ny, nx) against their
    successors' along the (0,1) paths (nibble 0, vertices) or (2,3) paths
    (nibble 7, cubes; a neighbouring cube must exist, so a step leaves room
    for two vertices); roots are the extrema's vertices (flat ids)."""
    nz, ny, nx = lab.shape
    room = 2 if cube else 1
    code = ((grad[z0:z1] >> np.uint32(4 * nibble)) & np.uint32(15)).astype(np.uint8)
    got = lab[z0:z1]
    assert not (code == 0).any()
    if cube:
        assert (got[code == 7] == exit_label).all()
    else:
        assert not (code == 7).any()
    for axis in range(3):
        n, d = (nx, ny, nz)[axis], 2 - axis  # numpy dimension of the axis
        for neg in (False, True):
            c = 2 * axis + 1 + int(neg)
            lo, hi = (1, n) if neg else (0, n - room)  # cells whose successor exists
            sh = -1 if neg else 1
            if axis == 2:
                a, b = max(z0, lo), min(z1, hi)
                if a < b:
                    assert ((code[a - z0:b - z0] != c) | (lab[a:b] == lab[a + sh:b + sh])).all(), (axis, neg)
                out = [z for z in range(z0, z1) if not lo <= z < hi]
                sel = [z - z0 for z in out]
                cs, gs = code[sel], got[sel]
            else:
                if lo < hi:
                    src = [slice(None)] * 3
                    dst = [slice(None)] * 3
                    src[d], dst[d] = slice(lo, hi), slice(lo + sh, hi + sh)
                    assert ((code[tuple(src)] != c) | (got[tuple(src)] == got[tuple(dst)])).all(), (axis, neg)
                idx = [i for i in range(n) if not lo <= i < hi]
                cs, gs = np.take(code, idx, axis=d), np.take(got, idx, axis=d)
            if cube:  # the path leaves the grid
                assert (gs[cs == c] == exit_label).all()
            else:
                assert not (cs == c).any()
    assert (code >= 8).sum() == ((roots >= z0 * nx * ny) & (roots < z1 * nx * ny)).sum()
