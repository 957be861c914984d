"""Seeded T-MLP parameter sets with the SIREN initialisation.

The paper uses SIREN as its backbone but does not restate its initialisation
(Sec. 4.1 cites it). The scheme used here is the one the SIREN paper
publishes: first layer W_1 ~ U(-1/fan_in, 1/fan_in), hidden layers
W_j ~ U(-sqrt(6/fan_in)/omega, sqrt(6/fan_in)/omega), biases
~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)), omega = 30.

FINER backbone (``activation="finer"``, sin(omega (|z| + 1) z)): the same
weight draws; FINER widens the range of the first layer's bias so that |z|,
and with it the local frequency, varies across the input; here b_1 ~ U(-1, 1)
(the bound is this generator's choice).

Tail scales. A trained SAND model has a first tail that carries the signed
distance and later tails that carry small residuals which shrink with depth
(Sec. 4.3, Table 2). Random tails cannot reproduce training, so two synthetic
conventions are offered:

* ``TailScale.PLAIN``: every tail factor drawn U(-1/sqrt(W), 1/sqrt(W)).
* ``TailScale.RESIDUAL``: tail 1 as above; for tail i >= 2 each factor of the
  multiplicative head is drawn U(-s_i, s_i) with s_i = sqrt(sigma_i)/sqrt(W/6),
  so each factor has standard deviation about sqrt(sigma_i) and their product
  about sigma_i = 1.6e-2 * 0.5**(i-2). Tail biases are zero.
"""

import enum

import numpy as np

from .blob import TAIL_LINEAR, TAIL_MULT


class TailScale(enum.Enum):
    PLAIN = "plain"
    RESIDUAL = "residual"


def residual_sigma(i):
    """Target standard deviation of tail i (1-based, i >= 2) under RESIDUAL."""
    return 1.6e-2 * 0.5 ** (i - 2)


def siren_tmlp(seed, L, W, omega=30.0, tails="mult", scale=TailScale.RESIDUAL,
               activation="sine"):
    """Draw a T-MLP parameter dict (the ``write_blob`` input).

    ``tails``: ``"linear"`` (every tail linear) or ``"mult"`` (tail 1 linear,
    tails 2..L multiplicative, as in Eq. 3).
    Draw order (PCG64): W_1, b_1, then W_j, b_j for j = 2..L, then tails in
    layer order, each tail drawing its weight vector(s) before its bias(es).
    """
    if tails not in ("linear", "mult"):
        raise ValueError("tails must be 'linear' or 'mult'")
    scale = TailScale(scale)
    rng = np.random.Generator(np.random.PCG64(seed))
    weights, biases = [], []
    if activation not in ("sine", "finer"):
        raise ValueError("activation must be 'sine' or 'finer'")
    b1 = 1.0 if activation == "finer" else 1.0 / np.sqrt(3.0)
    weights.append(rng.uniform(-1.0 / 3.0, 1.0 / 3.0, size=(W, 3)))
    biases.append(rng.uniform(-b1, b1, size=W))
    lim = np.sqrt(6.0 / W) / omega
    for _ in range(1, L):
        weights.append(rng.uniform(-lim, lim, size=(W, W)))
        biases.append(rng.uniform(-1.0 / np.sqrt(W), 1.0 / np.sqrt(W), size=W))
    out_tails = []
    plain = 1.0 / np.sqrt(W)
    for i in range(1, L + 1):
        kind = TAIL_LINEAR if (tails == "linear" or i == 1) else TAIL_MULT
        if scale is TailScale.RESIDUAL and i >= 2:
            s = np.sqrt(residual_sigma(i)) / np.sqrt(W / 6.0)
            bias_lim = 0.0
        else:
            s = plain
            bias_lim = plain
        if kind == TAIL_LINEAR:
            a = rng.uniform(-s, s, size=W)
            c = rng.uniform(-bias_lim, bias_lim) if bias_lim > 0 else 0.0
            out_tails.append({"kind": TAIL_LINEAR, "a": a, "c": c})
        else:
            a0 = rng.uniform(-s, s, size=W)
            c0 = rng.uniform(-bias_lim, bias_lim) if bias_lim > 0 else 0.0
            a1 = rng.uniform(-s, s, size=W)
            c1 = rng.uniform(-bias_lim, bias_lim) if bias_lim > 0 else 0.0
            out_tails.append({"kind": TAIL_MULT, "a0": a0, "c0": c0,
                              "a1": a1, "c1": c1})
    f32 = lambda a: np.asarray(a, dtype=np.float32)
    return {
        "activation": activation,
        "omega_first": float(omega),
        "omega_hidden": float(omega),
        "weights": [f32(w) for w in weights],
        "biases": [f32(b) for b in biases],
        "tails": [{k: (f32(v) if isinstance(v, np.ndarray) else
                       (float(np.float32(v)) if k != "kind" else v))
                   for k, v in t.items()} for t in out_tails],
    }
