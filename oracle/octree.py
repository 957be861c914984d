"""FP64 reference for the sparse network-depth octree (test infrastructure
only).

What is computed (Sec. 3.2, Eq. 5-7; Sec. 4.1 for the intersection test):

* Levels l = 0..D; a node at level l is a cell of side 2^(1-l) of the
  [-1, 1]^3 cube, integer coordinates (i, j, k) in [0, 2^l)^3, centre
  -1 + (i + 1/2) 2^(1-l) per axis. Children of (i, j, k) are
  (2i + a, 2j + b, 2k + c), a, b, c in {0, 1}.
* A node intersects the shape when the distance from its centre to the
  shape is at most half its diagonal, sqrt(3) 2^(-l) (Sec. 4.1). The shape
  is the one the network represents (Sec. 3.2: subdivision follows "the
  target shape represented by the implicit neural representation"), whose
  distance at the centre is read as |y_L(centre)|.
* Subdivision is top-down from the root: a node is subdivided (internal)
  when it intersects and l < D; its eight children are then nodes of level
  l + 1. Every other node reached this way is a leaf.
* A leaf at level D that intersects is near-surface: it stores the maximum
  over its s^3 sub-cell-centre samples of the required depth of Eq. 5
  (Eq. 6). Every other leaf is far: depth 0 and the signed distance at its
  centre, y_L(centre) (Eq. 7).
* A point is answered by the leaf whose cell contains it; cells are
  half-open and a point's cell at every level follows from its cell at
  level D by dropping low bits (the exact cell rule of oracle.tmlp).

Pins (tests/oracle_pins.py): a pure-Python recursive builder with the
scalar twin on a tiny model; constant-output models with closed-form trees
(root leaf; every level-D cell near with depth 1); structural invariants
(leaves tile the cube, each leaf's parent is internal and intersects,
internal nodes intersect, near leaves only at level D); lookups land in
the leaf that contains the point.
"""

import numpy as np

from .depthmap import required_depth, sample_points
from .tmlp import forward_all_tails, voxel_index

SQRT3 = float(np.sqrt(3.0))


def centres(level, ijk):
    return (np.asarray(ijk, dtype=np.float64) + 0.5) * (2.0 / (1 << level)) - 1.0


def y_last(model, pts):
    pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
    if pts.shape[0] == 0:
        return np.zeros(0)
    return forward_all_tails(model, pts)[:, -1]


def build(model, D, s, r):
    """The octree: {"D", "internal": [set of (i,j,k) per level 0..D-1],
    "leaves": {(l, i, j, k): (depth, value)}}."""
    internal = [set() for _ in range(D)]
    leaves = {}
    y0 = y_last(model, centres(0, [[0, 0, 0]]))[0]
    if abs(y0) <= SQRT3 and D > 0:
        internal[0].add((0, 0, 0))
    else:
        leaves[(0, 0, 0, 0)] = (0, float(y0))
    for l in range(1, D + 1):
        parents = sorted(internal[l - 1])
        if not parents:
            break
        kids = np.array([(2 * i + a, 2 * j + b, 2 * k + c) for (i, j, k) in parents
                         for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.int64)
        y = y_last(model, centres(l, kids))
        hit = np.abs(y) <= SQRT3 * 2.0 ** (-l)
        near = []
        for kid, yy, h in zip(map(tuple, kids), y, hit):
            if h and l < D:
                internal[l].add(kid)
            elif h:
                near.append(kid)
            else:
                leaves[(l,) + kid] = (0, float(yy))
        if near:
            R = 1 << l
            vox = np.array([(i * R + j) * R + k for (i, j, k) in near], dtype=np.int64)
            yall = forward_all_tails(model, sample_points(R, vox, s))
            d = required_depth(yall, r).reshape(len(near), s ** 3).max(axis=1)
            for kid, dd in zip(near, d):
                leaves[(l,) + kid] = (int(dd), 0.0)
    return {"D": D, "internal": internal, "leaves": leaves}


def lookup(tree, xyz):
    """(depth, value, level) of the leaf holding each point."""
    D = tree["D"]
    finest = voxel_index(xyz, 1 << D)                    # [n, 3] cells at level D
    n = finest.shape[0]
    depth = np.zeros(n, dtype=np.int64)
    value = np.zeros(n, dtype=np.float64)
    level = np.zeros(n, dtype=np.int64)
    for q in range(n):
        for l in range(0, D + 1):
            ijk = tuple(int(v) >> (D - l) for v in finest[q])
            key = (l,) + ijk
            if key in tree["leaves"]:
                depth[q], value[q] = tree["leaves"][key]
                level[q] = l
                break
            if l == D or ijk not in tree["internal"][l]:
                raise AssertionError("descent left the tree")
    return depth, value, level
