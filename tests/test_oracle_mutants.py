"""Plant plausible mistakes in the oracle (CPU) and check a pin catches each.

Each mutant replaces one oracle function with a subtly wrong copy; the test
passes only if at least one of the checks in ``oracle_pins`` then fails.
"""

import numpy as np
import pytest

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
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_some_pin_catches(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(T, attr, fn)
    caught = []
    for check in P.ALL_CHECKS:
        try:
            check()
        except AssertionError as e:
            caught.append(str(e))
    assert caught, f"no pin caught mutant: {name}"
