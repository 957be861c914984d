"""FP64 reference for map-free dynamic early exit (test infrastructure only).

What is computed (Sec. 4.4, the ablation on the necessity of the octree):
without a network-depth map, a point stops after the first layer whose
predicted residual is below the error threshold r in magnitude, and
otherwise runs to the last layer. The residual of layer i is its tail
output t_i (y_i = y_{i-1} + t_i, Eq. 2). Reading: the test starts at layer
2 -- t_1 is the base prediction, not a residual -- so

    d(x) = min { i >= 2 : |t_i(x)| < r },  or L if there is none,

then the level-of-detail clamp d <- min(d, max_depth) when max_depth > 0,
and the output is y_d (Eq. 2).

Pins (tests/oracle_pins.py): exit_from_tails against a pure-Python
loop over the definition on lattice values (exact ties at r, zeros,
negative tails); hand cases; monotone in r; tails computed per layer equal
the differences of the accumulated outputs; a model whose tails beyond
layer k vanish exits at layer k + 1 for tiny r; the scalar twin on a tiny
model.
"""

import numpy as np

from . import tmlp
from .tmlp import _tail, forward


def tails(model, xyz):
    """Every tail output t_1..t_L, float64 [n, L]."""
    h = np.asarray(xyz, dtype=np.float64)
    out = np.zeros((h.shape[0], model["L"]), dtype=np.float64)
    for j in range(1, model["L"] + 1):
        z = h @ model["W_"][j - 1].T + model["b_"][j - 1]
        h = tmlp.activation(model, j, z)
        out[:, j - 1] = _tail(model["tails"][j - 1], h)
    return out


def exit_from_tails(t, r, max_depth=0):
    """Exit depth per row of t = [n, L] tail outputs."""
    t = np.asarray(t, dtype=np.float64)
    n, L = t.shape
    small = np.abs(t) < r
    small[:, 0] = False                      # layer 1 is never tested
    small[:, L - 1] = True                   # without an earlier exit: L
    d = np.argmax(small, axis=1) + 1
    if max_depth > 0:
        d = np.minimum(d, max_depth)
    return d.astype(np.int64)


def dynamic_forward(model, xyz, r, max_depth=0):
    """(y_d, d) with d the dynamic exit depth of each point."""
    d = exit_from_tails(tails(model, xyz), r, max_depth)
    return forward(model, xyz, d), d
