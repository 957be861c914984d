"""Seeded workloads shared by the GPU tests (inputs only; no method arithmetic).

Every case is built by ``synth`` from fixed seeds; expected values come from
``oracle`` at test time.
"""

import functools

import numpy as np

import synth

# Tolerances on |SDF - oracle| (absolute, domain [-1, 1]^3).
TOL = {"fp32": 1e-5, "bf16": 2e-3, "fp16": 2e-3}


@functools.lru_cache(maxsize=None)
def c1_case():
    """4x64 linear-tail SIREN T-MLP, 32^3 sphere band map, 64^3 cell centres."""
    blob = synth.write_blob(synth.siren_tmlp(1, 4, 64, tails="linear", scale="plain"))
    return blob, synth.band_map_c1(32), synth.grid_points(64)


@functools.lru_cache(maxsize=None)
def c2_map(seed=2000, R=128, L=8):
    return synth.band_map_c2(synth.random_primitives(seed), R=R, L=L)


@functools.lru_cache(maxsize=None)
def c2_blob(W=256, seed=1000, scale="residual"):
    return synth.write_blob(synth.siren_tmlp(seed, 8, W, tails="mult", scale=scale))


def c2_points(n, seed=7, G=512):
    """n cells of the G^3 grid: half a contiguous run, half uniform samples."""
    half = n // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    start = int(rng.integers(0, G ** 3 - half))
    run = np.arange(start, start + half, dtype=np.int64)
    uni = synth.sample_indices(G ** 3, n - half, seed + 1)
    return synth.grid_points_at(G, np.concatenate([run, uni]))


def edge_points(R, n_random=2000, seed=3):
    """Points on, just beside and beyond cell faces, the cube's corners and
    edges, far outside the cube, and NaN coordinates."""
    faces = []
    for i in range(R + 1):
        f = np.float32(-1.0 + 2.0 * i / R)
        faces += [f, np.nextafter(f, np.float32(2)), np.nextafter(f, np.float32(-2))]
    faces = np.array(faces + [1.0, -1.0, 0.0, -0.0, 1.0000001, -1.0000001, 3.0, -7.5],
                     dtype=np.float32)
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = rng.choice(faces, size=(n_random, 3)).astype(np.float32)
    mix = rng.uniform(-1, 1, size=(n_random, 3)).astype(np.float32)
    keep = rng.integers(0, 3, size=(n_random, 3)) == 0
    pts[keep] = mix[keep]
    nan = np.array([[np.nan, 0.1, 0.2], [0.3, np.nan, -0.4], [0.5, 0.5, np.nan],
                    [np.nan, np.nan, np.nan]], dtype=np.float32)
    return np.concatenate([pts, nan])


@functools.lru_cache(maxsize=None)
def finer_blob(W=256, seed=1000, L=8, tails="mult", scale="residual"):
    """The 8x256 case on the FINER backbone (SAND-FINER): the same draws
    except the first layer's wider bias range."""
    return synth.write_blob(synth.siren_tmlp(seed, L, W, tails=tails, scale=scale,
                                             activation="finer"))
