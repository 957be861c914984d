"""FP64 reference for building a volumetric network-depth map (test
infrastructure only).

What is computed (Sec. 3.2, Eq. 5-7), on a dense R^3 grid of voxels over
[-1, 1]^3 (voxel (ix, iy, iz) is the box [-1 + 2 i/R, -1 + 2 (i+1)/R) per
axis, flat index (ix R + iy) R + iz):

1. Required depth of one point x from its accumulated outputs y_1..y_L
   (Eq. 5, near-surface case):
       d(x) = min { i : |y_L(x) - y_i(x)| < r  and  sign(y_i(x)) = sign(y_L(x)) },
   where sign is the three-valued sign (-1, 0, +1). i = L always qualifies
   (|y_L - y_L| = 0 < r), so 1 <= d(x) <= L.
2. Sample points of a voxel: the s^3 centres of its s x s x s sub-cells,
   x = -1 + (2/R) (i + (k + 1/2)/s) per axis, k = 0..s-1. (The paper pools
   over "all points" of a leaf without naming them; with R = 128 and s = 4
   these are exactly the 512^3 grid's cell centres that fall in the voxel.)
3. Map (Eq. 6-7): a near-surface voxel (near[v] = 1) stores the maximum
   required depth over its samples; a far voxel stores depth 0 and the SDF
   at its centre, supplied by the caller (the paper takes it from the
   shape's ground truth); near voxels store far value 0.

Which voxels are near-surface is an input (the paper tests whether the
distance from a voxel's centre to the surface is at most half the voxel's
diagonal, against the shape; the generators in synth/ do the same test
against the analytic scene).

Pins (tests/oracle_pins.py): required_depth against a pure-Python
loop over the definition on adversarial y rows (ties at r, zeros, sign
flips); invariants (range, monotone in r, truncated models whose tails
beyond layer k vanish give d <= k, with equality where the k-th tail moves
y by more than r); sample points against the 512^3 lattice; the map
against brute force with the scalar twin on a tiny model.
"""

import numpy as np

from .tmlp import forward_all_tails


def required_depth(y_all, r):
    """Eq. 5 (near case) per row of y_all = [n, L] accumulated outputs."""
    y = np.asarray(y_all, dtype=np.float64)
    n, L = y.shape
    yL = y[:, L - 1:L]
    ok = (np.abs(yL - y) < r) & (np.sign(y) == np.sign(yL))
    # the first qualifying layer (column L-1 always qualifies)
    return (np.argmax(ok, axis=1) + 1).astype(np.int64)


def sample_points(R, voxels, s):
    """The s^3 sub-cell centres of each voxel in `voxels` (flat indexes),
    float64 [len(voxels) * s^3, 3], voxel-major, sub-cells in (kx, ky, kz)
    C order."""
    v = np.asarray(voxels, dtype=np.int64)
    ix, iy, iz = v // (R * R), (v // R) % R, v % R
    k = (np.arange(s, dtype=np.float64) + 0.5) / s
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    sub = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)        # [s^3, 3]
    base = np.stack([ix, iy, iz], axis=1).astype(np.float64)           # [m, 3]
    pts = (base[:, None, :] + sub[None, :, :]) * (2.0 / R) - 1.0
    return pts.reshape(-1, 3)


def voxel_depths(model, R, voxels, s, r):
    """Max-pooled required depth (Eq. 6) of each listed voxel, int64."""
    v = np.asarray(voxels, dtype=np.int64)
    if v.size == 0:
        return np.zeros(0, dtype=np.int64)
    y_all = forward_all_tails(model, sample_points(R, v, s))
    d = required_depth(y_all, r).reshape(v.size, s ** 3)
    return d.max(axis=1)


def construct(model, R, near, center_sdf, s, r):
    """Eq. 6-7 on the dense grid: (depth uint8 [R^3], far float64 [R^3])."""
    near = np.asarray(near).reshape(-1).astype(bool)
    depth = np.zeros(R ** 3, dtype=np.uint8)
    far = np.where(near, 0.0, np.asarray(center_sdf, dtype=np.float64).reshape(-1))
    idx = np.nonzero(near)[0]
    depth[idx] = voxel_depths(model, R, idx, s, r)
    return depth, far
