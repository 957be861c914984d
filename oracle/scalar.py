"""Pure-Python scalar twin of the oracle's forward pass (test infrastructure).

One point at a time, with math.sin and correctly-rounded math.fsum dot
products, no numpy: a brute-force counterpart for tiny networks that shares
no array code with ``oracle.tmlp``. Eq. 2 (layers, tails, accumulation) and
Eq. 3 (multiplicative tail); the activation is SIREN's sin(omega z) or
FINER's sin(omega (|z| + 1) z).
"""

import math


def _dot(w, h):
    return math.fsum(float(a) * float(b) for a, b in zip(w, h))


def tail_value(tail, h):
    if tail[0] == "linear":
        return _dot(tail[1], h) + float(tail[2])
    _, a0, c0, a1, c1 = tail
    return (_dot(a0, h) + float(c0)) * (_dot(a1, h) + float(c1))


def _sigma(kind, om, v):
    if kind == "finer":
        return math.sin(om * (abs(v) + 1.0) * v)
    return math.sin(om * v)


def forward_point(model, x, d):
    """y_d at one point ``x`` (3 floats) for exit depth d >= 1."""
    h = [float(v) for v in x]
    terms = []
    for j in range(1, d + 1):
        Wj = model["W_"][j - 1]
        bj = model["b_"][j - 1]
        om = model["omega"][j - 1]
        h = [_sigma(model["activation"], om, _dot(Wj[u], h) + float(bj[u]))
             for u in range(len(bj))]
        terms.append(tail_value(model["tails"][j - 1], h))
    return math.fsum(terms)
