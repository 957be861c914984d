"""Write the stored expected values under tests/golden/.

Calls only ``oracle`` and ``synth``: every stored number is the FP64 oracle's
output on seeded synthetic inputs. Run from the repository root:
    python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def small_case():
    """4x64 linear-tail T-MLP (seed 1), 32^3 sphere band map, 64 grid points."""
    model_seed, G, k = 1, 64, 64
    blob = synth.write_blob(synth.siren_tmlp(model_seed, 4, 64, tails="linear",
                                             scale="plain"))
    model = oracle.parse_blob(blob)
    dmap = synth.band_map_c1(32)
    idx = synth.sample_indices(G ** 3, k, seed=5)
    x = synth.grid_points_at(G, idx)
    d = oracle.lookup_depth(x, dmap, 4)
    y = oracle.forward(model, x, d)
    g = oracle.gradient(model, x, d)
    return {
        "what": "4x64 linear-tail SIREN T-MLP, seed 1, plain tails; 32^3 sphere "
                "band map; 64 cells of the 64^3 grid (index seed 5)",
        "model_seed": model_seed, "grid": G, "index": idx.tolist(),
        "depth": d.tolist(), "y": [float(v).hex() for v in y],
        "grad": [[float(v).hex() for v in row] for row in g],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "c1_oracle_sample.json"), "w") as f:
        json.dump(small_case(), f, indent=1)
    print("wrote", os.path.join(HERE, "c1_oracle_sample.json"))
