"""Synthetic dense network-depth maps.

The paper builds its map from a trained T-MLP (Sec. 3.2, Eq. 5-7); without
trained weights the maps here are drawn from an analytic surface instead,
with deeper exits nearer the surface and where the surface bends more. The
map is a uint8 array [R, R, R] in C order (x slowest, z fastest) over the
cube [-1, 1]^3; cell i along an axis covers [-1 + 2i/R, -1 + 2(i+1)/R).
Value 0 marks a far-field cell whose signed distance is stored separately
(Eq. 7); values 1..L are exit depths.
"""

import numpy as np


def voxel_centres(R):
    """Coordinates of the R cell centres along one axis: -1 + (2i+1)/R."""
    return (2.0 * np.arange(R) + 1.0) / R - 1.0


def _centre_grid(R):
    c = voxel_centres(R)
    return np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1)


def band_map_c1(R=32, radius=0.5):
    """Depth 1..4 by distance band to a sphere of the given radius.

    |sdf| < 0.05 -> 4, < 0.15 -> 3, < 0.4 -> 2, else 1, at each cell centre.
    """
    p = _centre_grid(R)
    d = np.abs(np.linalg.norm(p, axis=-1) - radius)
    m = np.ones(d.shape, dtype=np.uint8)
    m[d < 0.4] = 2
    m[d < 0.15] = 3
    m[d < 0.05] = 4
    return m


BANDS_C2 = (0.4, 0.2, 0.1, 0.05, 0.03, 0.02)


def band_map_c2(prims, R=128, L=8):
    """Depth 1..L by distance band plus a curvature bump.

    d = 1 + #{tau in BANDS_C2 : |sdf(c)| < tau} + [|sdf(c)| <= sqrt(3)/R]
    (the last test is the cell-intersects-surface test, centre distance at
    most half the cell diagonal), then +1 where the magnitude of the
    7-point discrete Laplacian of the sdf (spacing 2/R, edge-replicated
    padding) exceeds its 90th percentile over all cells; clamped to L.
    """
    s = prims.sdf(_centre_grid(R))
    a = np.abs(s)
    d = np.ones(s.shape, dtype=np.int32)
    for tau in BANDS_C2:
        d += (a < tau)
    d += (a <= np.sqrt(3.0) / R)
    h = 2.0 / R
    pad = np.pad(s, 1, mode="edge")
    lap = (pad[2:, 1:-1, 1:-1] + pad[:-2, 1:-1, 1:-1] + pad[1:-1, 2:, 1:-1]
           + pad[1:-1, :-2, 1:-1] + pad[1:-1, 1:-1, 2:] + pad[1:-1, 1:-1, :-2]
           - 6.0 * s) / (h * h)
    kappa = np.abs(lap)
    d += (kappa > np.percentile(kappa, 90))
    return np.minimum(d, L).astype(np.uint8)


def far_value_grid(sdf_fn, R):
    """FP32 grid of the surface's signed distance at each cell centre."""
    return sdf_fn(_centre_grid(R)).astype(np.float32)


def near_surface_mask(sdf_fn, R):
    """uint8 [R, R, R]: 1 where the cell meets the surface, by the paper's
    test (Sec. 4.1): the distance from the cell centre to the surface is at
    most half the cell's diagonal, sqrt(3)/R for cells of side 2/R."""
    return (np.abs(sdf_fn(_centre_grid(R))) <= np.sqrt(3.0) / R).astype(np.uint8)
