"""Analytic synthetic surfaces (FP64 signed distance functions).

They stand in for the paper's scanned and Thingi meshes, which are not
available: a single sphere for the small case and a union of seeded spheres
and tori for the large ones. Only used to shape depth maps and query sets.
"""

import dataclasses

import numpy as np


def sphere_sdf(p, centre=(0.0, 0.0, 0.0), radius=0.5):
    p = np.asarray(p, dtype=np.float64)
    return np.linalg.norm(p - np.asarray(centre, dtype=np.float64), axis=-1) - radius


def _random_rotation(rng):
    """Uniform random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


@dataclasses.dataclass
class Primitives:
    """Union of spheres and tori; ``sdf`` is the minimum of their SDFs."""
    sphere_centres: np.ndarray   # [S, 3]
    sphere_radii: np.ndarray     # [S]
    torus_centres: np.ndarray    # [T, 3]
    torus_rot: np.ndarray        # [T, 3, 3], world -> local is R^T (p - c)
    torus_major: np.ndarray      # [T]
    torus_minor: np.ndarray      # [T]

    def sdf(self, p, chunk=1 << 20):
        p = np.asarray(p, dtype=np.float64)
        shape = p.shape[:-1]
        flat = p.reshape(-1, 3)
        out = np.empty(flat.shape[0], dtype=np.float64)
        for s in range(0, flat.shape[0], chunk):
            q = flat[s:s + chunk]
            d = np.full(q.shape[0], np.inf)
            for c, r in zip(self.sphere_centres, self.sphere_radii):
                d = np.minimum(d, np.linalg.norm(q - c, axis=1) - r)
            for c, rot, big, small in zip(self.torus_centres, self.torus_rot,
                                          self.torus_major, self.torus_minor):
                loc = (q - c) @ rot  # = (R^T (q - c))^T
                rad = np.hypot(loc[:, 0], loc[:, 1]) - big
                d = np.minimum(d, np.hypot(rad, loc[:, 2]) - small)
            out[s:s + chunk] = d
        return out.reshape(shape)

    def grad(self, p, h=1e-6):
        """Central-difference gradient of ``sdf`` (generator use only)."""
        p = np.asarray(p, dtype=np.float64)
        g = np.empty(p.shape, dtype=np.float64)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            g[..., a] = (self.sdf(p + e) - self.sdf(p - e)) / (2 * h)
        return g


def random_primitives(seed, count=12):
    """``count`` primitives alternating sphere, torus, sphere, ... .

    Spheres: centre U[-0.55, 0.55]^3, radius U[0.12, 0.30].
    Tori: centre as above, uniform random rotation, major radius U[0.15, 0.30],
    minor radius U[0.03, 0.08]. Draw order follows the primitive order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sc, sr, tc, tr, tM, tm = [], [], [], [], [], []
    for k in range(count):
        c = rng.uniform(-0.55, 0.55, size=3)
        if k % 2 == 0:
            sc.append(c)
            sr.append(rng.uniform(0.12, 0.30))
        else:
            tc.append(c)
            tr.append(_random_rotation(rng))
            tM.append(rng.uniform(0.15, 0.30))
            tm.append(rng.uniform(0.03, 0.08))
    arr = lambda x, s: np.asarray(x, dtype=np.float64).reshape(s)
    return Primitives(arr(sc, (-1, 3)), arr(sr, (-1,)), arr(tc, (-1, 3)),
                      arr(tr, (-1, 3, 3)), arr(tM, (-1,)), arr(tm, (-1,)))
