"""Seeded query point sets (FP32 coordinates in [-1, 1]^3, shape [n, 3]).

* the G^3 grid of cell centres, C order (x slowest, z fastest), as used by a
  marching-cubes pass over the cube (Sec. 4.1 queries a 512^3 grid);
* uniform subsamples of such a grid;
* near-surface points, contiguous grid slabs and camera-ray samples for the
  served and differentiated workloads.
"""

import math

import numpy as np


def grid_points_at(G, idx):
    """Cell-centre coordinates of linear grid indices ``idx`` (C order).

    Coordinate along an axis: (2i+1)/G - 1, exact in FP32 for G <= 2^23.
    """
    idx = np.asarray(idx, dtype=np.int64)
    ix = idx // (G * G)
    iy = (idx // G) % G
    iz = idx % G
    f = lambda i: ((2.0 * i + 1.0) / G - 1.0).astype(np.float32)
    return np.stack([f(ix), f(iy), f(iz)], axis=-1)


def grid_points(G):
    """All G^3 cell centres, [G^3, 3] float32."""
    c = ((2.0 * np.arange(G) + 1.0) / G - 1.0).astype(np.float32)
    out = np.empty((G, G, G, 3), dtype=np.float32)
    out[..., 0] = c[:, None, None]
    out[..., 1] = c[None, :, None]
    out[..., 2] = c[None, None, :]
    return out.reshape(-1, 3)


def grid_points_torch(G, device):
    """The same grid built directly on a torch device (identical values)."""
    import torch
    c = (torch.arange(G, dtype=torch.float64, device=device) * 2.0 + 1.0) / G - 1.0
    c = c.to(torch.float32)
    out = torch.empty((G, G, G, 3), dtype=torch.float32, device=device)
    out[..., 0] = c[:, None, None]
    out[..., 1] = c[None, :, None]
    out[..., 2] = c[None, None, :]
    return out.reshape(-1, 3)


def sample_indices(n, k, seed):
    """``k`` distinct indices drawn uniformly from range(n), sorted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if k >= n:
        return np.arange(n, dtype=np.int64)
    if n <= 1 << 24:
        return np.sort(rng.choice(n, size=k, replace=False))
    got = np.unique(rng.integers(0, n, size=int(k * 1.05) + 64))
    while got.size < k:
        got = np.unique(np.concatenate([got, rng.integers(0, n, size=k)]))
    return np.sort(rng.permutation(got)[:k])


def near_surface_points(prims, n, seed, band=0.05, sigma=0.02, pool=1 << 16):
    """Points jittered around the surface.

    Rejection-sample uniform points with |sdf| < band, move each onto the
    surface with three steps p <- p - sdf(p) * grad sdf(p), then add
    isotropic Gaussian noise N(0, sigma^2); clipped to [-1, 1].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    got = []
    have = 0
    while have < n:
        p = rng.uniform(-1.0, 1.0, size=(pool, 3))
        keep = p[np.abs(prims.sdf(p)) < band]
        got.append(keep)
        have += keep.shape[0]
    p = np.concatenate(got)[:n]
    for _ in range(3):
        g = prims.grad(p)
        g /= np.maximum(np.linalg.norm(g, axis=1, keepdims=True), 1e-12)
        p = p - prims.sdf(p)[:, None] * g
    p = p + rng.normal(0.0, sigma, size=p.shape)
    return np.clip(p, -1.0, 1.0).astype(np.float32)


def slab_points(G, n, seed):
    """A contiguous run of ``n`` grid points in C order from a random start."""
    rng = np.random.Generator(np.random.PCG64(seed))
    start = int(rng.integers(0, G ** 3 - n + 1))
    return grid_points_at(G, np.arange(start, start + n, dtype=np.int64))


def _look_at_basis(eye):
    fwd = -eye / np.linalg.norm(eye)
    up0 = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) < 0.9 else np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up0)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return fwd, right, up


def camera_ray_points(prims, seed, width=1920, height=1080, distance=2.5,
                      fov_deg=40.0, sigma=0.03, max_steps=96):
    """One sample per pixel along rays of a pinhole camera looking at the origin.

    The eye sits at ``distance`` in a seeded uniform direction, vertical field
    of view ``fov_deg``. Each ray is sphere-traced (FP64) against the analytic
    surface; a hit point is moved along its ray by N(0, sigma^2). A miss takes
    t uniform in the ray's span inside [-1, 1]^3, or t = |eye| if the ray does
    not meet the cube. Returns float32 [height*width, 3] clipped to the cube.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=3)
    eye = distance * v / np.linalg.norm(v)
    fwd, right, up = _look_at_basis(eye)
    tan_half = math.tan(math.radians(fov_deg) / 2.0)
    aspect = width / height
    ys = (1.0 - 2.0 * (np.arange(height) + 0.5) / height) * tan_half
    xs = (2.0 * (np.arange(width) + 0.5) / width - 1.0) * tan_half * aspect
    dirs = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
            + ys[:, None, None] * up[None, None, :]).reshape(-1, 3)
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    n = dirs.shape[0]
    # slab test against the cube
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / dirs
        t0 = (-1.0 - eye[None, :]) * inv
        t1 = (1.0 - eye[None, :]) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=1)
    in_box = tmax > np.maximum(tmin, 0.0)
    t = np.where(in_box, np.maximum(tmin, 0.0), 0.0)
    hit = np.zeros(n, dtype=bool)
    active = in_box.copy()
    for _ in range(max_steps):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        p = eye[None, :] + t[idx, None] * dirs[idx]
        d = prims.sdf(p)
        done = d < 1e-5
        hit[idx[done]] = True
        t[idx] += np.where(done, 0.0, d)
        out = t[idx] > tmax[idx]
        active[idx[done | out]] = False
    t_out = np.empty(n)
    t_out[hit] = t[hit] + rng.normal(0.0, sigma, size=int(hit.sum()))
    miss = ~hit
    lo = np.maximum(tmin, 0.0)
    u = rng.uniform(0.0, 1.0, size=n)
    t_miss = np.where(in_box, lo + u * (tmax - lo), np.linalg.norm(eye))
    t_out[miss] = t_miss[miss]
    pts = eye[None, :] + t_out[:, None] * dirs
    return np.clip(pts, -1.0, 1.0).astype(np.float32)
