"""Plant plausible mistakes in the oracle (CPU) and check a pin catches each.

Each mutant replaces one oracle function with a subtly wrong copy; the test
passes only if at least one of the checks in ``oracle_pins`` then fails.
"""

import numpy as np
import pytest

import oracle.depthmap as D
import oracle.dynamic as DY
import oracle.octree as OT
import oracle.tmlp as T
import oracle_pins as P


def _swapped_biases(t, h):
    if t[0] == "linear":
        return h @ t[1] + t[2]
    _, a0, c0, a1, c1 = t
    return (h @ a0 + c1) * (h @ a1 + c0)


def _additive_tail(t, h):
    if t[0] == "linear":
        return h @ t[1] + t[2]
    _, a0, c0, a1, c1 = t
    return (h @ a0 + c0) + (h @ a1 + c1)


def _forward_last_tail_only(model, xyz, d, far=None):
    x = np.asarray(xyz, dtype=np.float64)
    d = np.asarray(d, dtype=np.int64)
    y = _ORIG_FORWARD(model, xyz, np.where(d == 0, 0, 1), far) * (d == 0)
    for k in np.unique(d):
        if k == 0:
            continue
        rows = np.nonzero(d == k)[0]
        h = x[rows]
        for j in range(1, k + 1):
            h = np.sin(model["omega"][j - 1] * (h @ model["W_"][j - 1].T + model["b_"][j - 1]))
        y[rows] = T._tail(model["tails"][k - 1], h)
    return y


def _forward_off_by_one(model, xyz, d, far=None):
    return _ORIG_FORWARD(model, xyz, np.minimum(np.asarray(d) + 1, model["L"]), far)


def _forward_bias_outside_omega(model, xyz, d, far=None):
    x = np.asarray(xyz, dtype=np.float64)
    d = np.asarray(d, dtype=np.int64)
    y = _ORIG_FORWARD(model, xyz, np.where(d == 0, 0, 1), far) * (d == 0)
    rows = np.nonzero(d >= 1)[0]
    h = x[rows]
    for j in range(1, model["L"] + 1):
        if rows.size == 0:
            break
        h = np.sin(model["omega"][j - 1] * (h @ model["W_"][j - 1].T) + model["b_"][j - 1])
        y[rows] += T._tail(model["tails"][j - 1], h)
        keep = d[rows] > j
        rows, h = rows[keep], h[keep]
    return y


def _forward_transposed(model, xyz, d, far=None):
    m = dict(model)
    m["W_"] = [model["W_"][0]] + [w.T.copy() for w in model["W_"][1:]]
    return _ORIG_FORWARD(m, xyz, d, far)


def _cell_via_shift(xyz, R):
    x = np.asarray(xyz, dtype=np.float64)
    s = R // 2
    with np.errstate(invalid="ignore"):
        v = np.floor((x + 1.0) * s)
    v = np.where(np.isnan(v), 0, v)
    return np.clip(v, 0, R - 1).astype(np.int64)


def _cell_round(xyz, R):
    x = np.asarray(xyz, dtype=np.float64)
    s = R // 2
    with np.errstate(invalid="ignore"):
        v = np.round(x * s)
    v = np.where(np.isnan(v), -s, v)
    return (np.clip(v, -s, s - 1) + s).astype(np.int64)


def _tail_grad_swapped(t, h):
    if t[0] == "linear":
        return np.broadcast_to(t[1], h.shape)
    _, a0, c0, a1, c1 = t
    return (h @ a0 + c0)[:, None] * a0[None, :] + (h @ a1 + c1)[:, None] * a1[None, :]


def _gradient_no_intermediate_tails(model, xyz, d):
    m = dict(model)
    orig = T._tail_grad
    calls = {"n": 0}

    def only_first(t, h):
        calls["n"] += 1
        return orig(t, h) if calls["n"] == 1 else np.zeros_like(h)
    T._tail_grad = only_first
    try:
        out = []
        x = np.asarray(xyz, dtype=np.float64)
        d = np.asarray(d)
        g = np.zeros_like(x)
        for i in range(x.shape[0]):
            calls["n"] = 0
            g[i] = _ORIG_GRADIENT(m, x[i:i + 1], d[i:i + 1])[0]
        return g
    finally:
        T._tail_grad = orig


_ORIG_FORWARD = T.forward
_ORIG_GRADIENT = T.gradient
_ORIG_ACT = T.activation
_ORIG_SLOPE = T.activation_slope


def _finer_no_abs_term(model, j, z):
    if model["activation"] == "finer":
        return np.sin(model["omega"][j - 1] * z)            # |z| dropped: plain SIREN
    return _ORIG_ACT(model, j, z)


def _finer_signed(model, j, z):
    if model["activation"] == "finer":
        return np.sin(model["omega"][j - 1] * (z + 1.0) * z)  # abs dropped
    return _ORIG_ACT(model, j, z)


def _finer_slope_without_two(model, j, z):
    if model["activation"] == "finer":
        om = model["omega"][j - 1]
        return om * (np.abs(z) + 1.0) * np.cos(om * (np.abs(z) + 1.0) * z)
    return _ORIG_SLOPE(model, j, z)


# -- depth-map construction mutants --------------------------------------------

def _depth_inclusive(y_all, r):
    y = np.asarray(y_all, dtype=np.float64)
    ok = (np.abs(y[:, -1:] - y) <= r) & (np.sign(y) == np.sign(y[:, -1:]))
    return np.argmax(ok, axis=1) + 1


def _depth_no_sign(y_all, r):
    y = np.asarray(y_all, dtype=np.float64)
    return np.argmax(np.abs(y[:, -1:] - y) < r, axis=1) + 1


def _depth_zero_based(y_all, r):
    return _ORIG_REQUIRED(y_all, r) - 1


def _depth_against_previous(y_all, r):
    y = np.asarray(y_all, dtype=np.float64)
    ref = y[:, -2:-1]
    ok = (np.abs(ref - y) < r) & (np.sign(y) == np.sign(ref))
    ok[:, -1] = True
    return np.argmax(ok, axis=1) + 1


def _samples_at_corners(R, voxels, s):
    return _ORIG_SAMPLES(R, voxels, s) - (1.0 / (R * s))


def _min_pooling(model, R, voxels, s, r):
    v = np.asarray(voxels, dtype=np.int64)
    if v.size == 0:
        return np.zeros(0, dtype=np.int64)
    y = T.forward_all_tails(model, D.sample_points(R, v, s))
    return D.required_depth(y, r).reshape(v.size, s ** 3).min(axis=1)


def _far_keeps_depth(model, R, near, center_sdf, s, r):
    depth, far = _ORIG_CONSTRUCT(model, R, np.ones_like(np.asarray(near)), center_sdf, s, r)
    near = np.asarray(near).reshape(-1).astype(bool)
    return depth, np.where(near, 0.0, np.asarray(center_sdf, dtype=np.float64))


def _dyn_from_layer_one(t, r, max_depth=0):
    t = np.asarray(t, dtype=np.float64)
    small = np.abs(t) < r
    small[:, -1] = True
    d = np.argmax(small, axis=1) + 1
    return np.minimum(d, max_depth) if max_depth > 0 else d


def _dyn_inclusive(t, r, max_depth=0):
    t = np.asarray(t, dtype=np.float64)
    small = np.abs(t) <= r
    small[:, 0] = False
    small[:, -1] = True
    d = np.argmax(small, axis=1) + 1
    return np.minimum(d, max_depth) if max_depth > 0 else d


def _dyn_on_outputs(model, xyz):
    return T.forward_all_tails(model, xyz)          # y_i in place of t_i


def _dyn_signed(t, r, max_depth=0):
    return _signed_exit(t, r, max_depth)


def _signed_exit(t, r, max_depth):
    t = np.asarray(t, dtype=np.float64)
    small = t < r                                   # sign kept: negative tails exit at once
    small[:, 0] = False
    small[:, -1] = True
    d = np.argmax(small, axis=1) + 1
    return np.minimum(d, max_depth) if max_depth > 0 else d


def _dyn_no_clamp(t, r, max_depth=0):
    return _ORIG_EXIT(t, r, 0)


def _octree_variant(strict=False, half_side=False, corner=False, min_pool=False, extra_level=False):
    """A copy of the octree builder with one plausible mistake."""
    def build(model, Dmax, s, r):
        internal = [set() for _ in range(Dmax + (1 if extra_level else 0))]
        leaves = {}
        def h(l):
            return (2.0 ** (-l)) if half_side else OT.SQRT3 * 2.0 ** (-l)
        def test(y, l):
            return abs(y) < h(l) if strict else abs(y) <= h(l)
        y0 = OT.y_last(model, OT.centres(0, [[0, 0, 0]]))[0]
        if test(y0, 0) and Dmax > 0:
            internal[0].add((0, 0, 0))
        else:
            leaves[(0, 0, 0, 0)] = (0, float(y0))
        top = Dmax + (1 if extra_level else 0)
        for l in range(1, top + 1):
            parents = sorted(internal[l - 1])
            if not parents:
                break
            kids = np.array([(2 * i + a, 2 * j + b, 2 * k + c) for (i, j, k) in parents
                             for a in (0, 1) for b in (0, 1) for c in (0, 1)], dtype=np.int64)
            pts = OT.centres(l, kids) - (1.0 / (1 << l) if corner else 0.0)
            y = OT.y_last(model, pts)
            near = []
            for kid, yy in zip(map(tuple, kids), y):
                hit = test(yy, l)
                if hit and l < top:
                    internal[l].add(kid)
                elif hit:
                    near.append(kid)
                else:
                    leaves[(l,) + kid] = (0, float(yy))
            if near:
                R = 1 << l
                vox = np.array([(i * R + j) * R + k for (i, j, k) in near], dtype=np.int64)
                yall = T.forward_all_tails(model, D_sample(R, vox, s))
                d = _REQUIRED(yall, r).reshape(len(near), s ** 3)
                d = d.min(axis=1) if min_pool else d.max(axis=1)
                for kid, dd in zip(near, d):
                    leaves[(l,) + kid] = (int(dd), 0.0)
        return {"D": top, "internal": internal, "leaves": leaves}
    return build


def D_sample(R, vox, s):
    return _SAMPLES(R, vox, s)


_REQUIRED = D.required_depth
_SAMPLES = D.sample_points


def _lookup_xz_swapped(tree, xyz):
    x = np.asarray(xyz, dtype=np.float64)[:, ::-1].copy()
    return _ORIG_LOOKUP(tree, x)


_ORIG_LOOKUP = OT.lookup
_ORIG_EXIT = DY.exit_from_tails
_ORIG_REQUIRED = D.required_depth
_ORIG_SAMPLES = D.sample_points
_ORIG_CONSTRUCT = D.construct

MUTANTS = {
    "tail biases swapped": ("_tail", _swapped_biases),
    "tail factors added": ("_tail", _additive_tail),
    "output is last tail only": ("forward", _forward_last_tail_only),
    "one layer too many": ("forward", _forward_off_by_one),
    "bias outside omega": ("forward", _forward_bias_outside_omega),
    "hidden weights transposed": ("forward", _forward_transposed),
    "cell via (x+1)*s": ("voxel_index", _cell_via_shift),
    "cell by rounding": ("voxel_index", _cell_round),
    "tail gradient factors swapped": ("_tail_grad", _tail_grad_swapped),
    "gradient drops intermediate tails": ("gradient", _gradient_no_intermediate_tails),
    "depth threshold inclusive": (D, "required_depth", _depth_inclusive),
    "depth ignores the sign test": (D, "required_depth", _depth_no_sign),
    "depth zero-based": (D, "required_depth", _depth_zero_based),
    "depth against y_(L-1)": (D, "required_depth", _depth_against_previous),
    "samples at sub-cell corners": (D, "sample_points", _samples_at_corners),
    "min-pooling over a voxel": (D, "voxel_depths", _min_pooling),
    "far voxels keep a depth": (D, "construct", _far_keeps_depth),
    "dynamic test from layer 1": (DY, "exit_from_tails", _dyn_from_layer_one),
    "dynamic threshold inclusive": (DY, "exit_from_tails", _dyn_inclusive),
    "dynamic test on outputs": (DY, "tails", _dyn_on_outputs),
    "dynamic residual sign kept": (DY, "exit_from_tails", _dyn_signed),
    "dynamic ignores max_depth": (DY, "exit_from_tails", _dyn_no_clamp),
    "octree strict intersection test": (OT, "build", _octree_variant(strict=True)),
    "octree half side for half diagonal": (OT, "build", _octree_variant(half_side=True)),
    "octree far value at the corner": (OT, "build", _octree_variant(corner=True)),
    "octree min-pooling near leaves": (OT, "build", _octree_variant(min_pool=True)),
    "octree subdivides past D": (OT, "build", _octree_variant(extra_level=True)),
    "octree lookup axes swapped": (OT, "lookup", _lookup_xz_swapped),
    "finer activation drops |z|": ("activation", _finer_no_abs_term),
    "finer activation without abs": ("activation", _finer_signed),
    "finer slope without the factor 2": ("activation_slope", _finer_slope_without_two),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_some_pin_catches(name, monkeypatch):
    entry = MUTANTS[name]
    mod, attr, fn = entry if len(entry) == 3 else (T, *entry)
    monkeypatch.setattr(mod, attr, fn)
    caught = []
    for check in P.ALL_CHECKS:
        try:
            check()
        except AssertionError as e:
            caught.append(str(e))
    assert caught, f"no pin caught mutant: {name}"
