"""Model blob writer: the on-disk / in-memory format that ``sand_load_model``
accepts.

Layout (little-endian, version 1):

    offset  size  field
    0       8     magic  b"SANDTMLP"
    8       4     u32 version (= 1)
    12      4     u32 L, number of sine hidden layers (1..16)
    16      4     u32 W, hidden width (1..1024)
    20      4     u32 input dimension (= 3)
    24      4     f32 omega_first   (frequency of hidden layer 1)
    28      4     f32 omega_hidden  (frequency of hidden layers 2..L)
    32      16    u8 tail kind per layer i = 1..L (0 = linear, 1 = multiplicative),
                  unused entries 0
    48      1     u8 activation: 0 = SIREN sine sin(omega z),
                  1 = FINER variable-periodic sine sin(omega (|z| + 1) z)
    49      15    reserved, zero
    64      ...   f32 parameters, in this order:
                  W_1 [W x 3] row-major, b_1 [W],
                  for j = 2..L: W_j [W x W] row-major (out x in), b_j [W],
                  for i = 1..L: linear tail:          a [W], c
                                multiplicative tail:  a0 [W], c0, a1 [W], c1

Hidden layer j computes h_j = sigma(omega_j, W_j h_{j-1} + b_j) with the
activation named in the header (SIREN or FINER, the two backbones of Sec. 4.1); tail i is the linear head a.h + c or the product of two linear heads
(a0.h + c0)(a1.h + c1) (Sec. 3.1, Eq. 2 and Eq. 3).
"""

import struct

import numpy as np

MAGIC = b"SANDTMLP"
VERSION = 1
HEADER_BYTES = 64
MAX_LAYERS = 16
TAIL_LINEAR = 0
TAIL_MULT = 1
ACTIVATIONS = {"sine": 0, "finer": 1}


def blob_nbytes(L, W, tail_kinds):
    """Exact byte size of a version-1 blob with these dimensions."""
    n = W * 3 + W + (L - 1) * (W * W + W)
    for k in tail_kinds:
        n += (W + 1) * (2 if k == TAIL_MULT else 1)
    return HEADER_BYTES + 4 * n


def write_blob(model):
    """Serialise a parameter dict into blob bytes.

    ``model`` keys: ``omega_first``, ``omega_hidden`` (floats), ``weights``
    (list of L arrays: [W,3] then [W,W]), ``biases`` (list of L [W] arrays),
    ``tails`` (list of L dicts: ``{"kind": 0, "a", "c"}`` or
    ``{"kind": 1, "a0", "c0", "a1", "c1"}``), optionally ``activation``
    (``"sine"``, the default, or ``"finer"``). Arrays are cast to float32.
    """
    weights = model["weights"]
    biases = model["biases"]
    tails = model["tails"]
    L = len(weights)
    if not (1 <= L <= MAX_LAYERS):
        raise ValueError("number of layers must be in 1..16")
    W = int(np.asarray(weights[0]).shape[0])
    kinds = [int(t["kind"]) for t in tails]
    if len(biases) != L or len(tails) != L:
        raise ValueError("weights, biases and tails must have one entry per layer")
    head = bytearray(HEADER_BYTES)
    struct.pack_into("<8sIIIIff", head, 0, MAGIC, VERSION, L, W, 3,
                     float(model["omega_first"]), float(model["omega_hidden"]))
    for i, k in enumerate(kinds):
        head[32 + i] = k
    head[48] = ACTIVATIONS[model.get("activation", "sine")]
    parts = [bytes(head)]

    def f32(a, shape):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        if a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return a.astype("<f4").tobytes()

    parts.append(f32(weights[0], (W, 3)))
    parts.append(f32(biases[0], (W,)))
    for j in range(1, L):
        parts.append(f32(weights[j], (W, W)))
        parts.append(f32(biases[j], (W,)))
    for t in tails:
        if t["kind"] == TAIL_LINEAR:
            parts.append(f32(t["a"], (W,)))
            parts.append(f32([t["c"]], (1,)))
        elif t["kind"] == TAIL_MULT:
            parts.append(f32(t["a0"], (W,)))
            parts.append(f32([t["c0"]], (1,)))
            parts.append(f32(t["a1"], (W,)))
            parts.append(f32([t["c1"]], (1,)))
        else:
            raise ValueError("tail kind must be 0 (linear) or 1 (multiplicative)")
    out = b"".join(parts)
    assert len(out) == blob_nbytes(L, W, kinds)
    return out
