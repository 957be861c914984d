"""Model-blob parser for the oracle (test infrastructure only).

Reads the version-1 little-endian blob: a 64-byte header (magic b"SANDTMLP",
u32 version, u32 L, u32 W, u32 input dim = 3, f32 omega of layer 1, f32 omega
of layers 2..L, u8 tail kind per layer, u8 activation (0 = SIREN sine,
1 = FINER variable-periodic sine), 15 reserved bytes) followed by the
float32 parameters W_1, b_1, (W_j, b_j) for j = 2..L, then each tail in layer
order: linear (a, c) or multiplicative (a0, c0, a1, c1). Eq. 2 defines the
layers and tails; Eq. 3 the multiplicative tail.

All parameters are widened to float64 exactly.
"""

import struct

import numpy as np


def parse_blob(data):
    data = bytes(data)
    if len(data) < 64 or data[:8] != b"SANDTMLP":
        raise ValueError("not a SAND model blob")
    version, L, W, din = struct.unpack_from("<IIII", data, 8)
    om1, omh = struct.unpack_from("<ff", data, 24)
    if version != 1 or din != 3 or not (1 <= L <= 16) or W < 1:
        raise ValueError("unsupported blob header")
    kinds = list(data[32:32 + L])
    if any(k not in (0, 1) for k in kinds):
        raise ValueError("bad tail kind")
    if data[48] not in (0, 1):
        raise ValueError("bad activation")
    activation = ("sine", "finer")[data[48]]
    vals = np.frombuffer(data, dtype="<f4", offset=64).astype(np.float64)
    pos = 0

    def take(n):
        nonlocal pos
        out = vals[pos:pos + n]
        if out.size != n:
            raise ValueError("blob truncated")
        pos += n
        return out

    Ws, bs = [take(W * 3).reshape(W, 3)], [take(W)]
    for _ in range(1, L):
        Ws.append(take(W * W).reshape(W, W))
        bs.append(take(W))
    tails = []
    for k in kinds:
        if k == 0:
            a = take(W)
            c = take(1)[0]
            tails.append(("linear", a, c))
        else:
            a0 = take(W)
            c0 = take(1)[0]
            a1 = take(W)
            c1 = take(1)[0]
            tails.append(("mult", a0, c0, a1, c1))
    if pos != vals.size:
        raise ValueError("blob has trailing bytes")
    omegas = [float(np.float32(om1))] + [float(np.float32(omh))] * (L - 1)
    return {"L": L, "W": W, "omega": omegas, "W_": Ws, "b_": bs, "tails": tails,
            "activation": activation}
