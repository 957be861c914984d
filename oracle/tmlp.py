"""FP64 reference for the SAND query path (test infrastructure only).

What is computed, per query point x (FP32 or FP64 coordinates, widened exactly to FP64):

1. Cell of x in a dense R^3 network-depth map over [-1, 1]^3 (R a power of
   two). Cell i along an axis is the half-open interval
   [-1 + 2i/R, -1 + 2(i+1)/R); points beyond the cube fall into the border
   cell and a NaN coordinate into cell 0. With s = R/2 a power of two the
   product x*s is exact, so i = floor(x*s) + s (clamped) is the exact cell.
2. Exit depth d(x): the map value (adaptive), L (full depth) or a given
   value (forced); then the level-of-detail clamp d <- min(d, max_depth)
   when max_depth > 0 (Sec. 3.4, last paragraph).
3. d = 0 marks a far-field cell: the value stored for that cell is returned
   and no network runs (Sec. 3.2, Eq. 7; Sec. 3.4).
4. Otherwise the T-MLP of Eq. 2 runs to layer d: h_0 = x,
   z_j = W_j h_{j-1} + b_j, h_j = sigma_j(z_j), tail t_j from h_j -- linear a.h + c, or for the multiplicative design of Eq. 3
   (a0.h + c0)(a1.h + c1) -- and the output is the accumulated
   y_d = t_1 + ... + t_d (Eq. 2; the overview figure's caption: the
   accumulated output up to the exit depth is the prediction).
   The activation sigma_j is the backbone's (Sec. 4.1 runs SAND on SIREN and
   on FINER and restates neither; both definitions are their own papers'):
     sine  (SIREN):  sigma_j(z) = sin(omega_j z);
     finer (FINER, variable-periodic sine): sigma_j(z) = sin(omega_j (|z| + 1) z).
5. Input gradient of y_d with d held fixed (the map is piecewise constant):
   reverse accumulation from the exit tail,
     g_d = dt_d/dh_d,  delta_j = sigma_j'(z_j) * g_j,
     g_{j-1} = W_j^T delta_j + dt_{j-1}/dh_{j-1},  grad_x = W_1^T delta_1,
   with dt/dh = a (linear) or (a1.h + c1) a0 + (a0.h + c0) a1 (Eq. 3), and
   sigma_j'(z) = omega_j cos(omega_j z) (sine) or
   omega_j (2|z| + 1) cos(omega_j (|z| + 1) z) (finer: d/dz of (|z| + 1) z
   is 2|z| + 1). A far-field point's value is constant within its cell:
   gradient 0.

Pins (tests/test_oracle_pins.py): the cell rule against exact rational box
membership; forward against the textbook MLP of Eq. 1 (intermediate tails
zeroed) built from torch.nn layers; the quadratic-form identity of the
appendix for the multiplicative tail; truncation (exit at k equals the
k-layer network at full depth); an all-L map equals full depth; a pure-Python
scalar twin on tiny inputs; 50-digit mpmath spot values; the gradient against
torch autograd and against central differences. The FINER activation:
its zeros and extrema at the roots of omega (|z| + 1) z = k pi / 2 solved
at 50 digits (odd in z), its slope against central differences, and the
scalar twin, mpmath, truncation and gradient pins on FINER models.
"""

import numpy as np

MODE_ADAPTIVE = 0
MODE_FULL = 1
MODE_FORCED = 2


def voxel_index(xyz, R):
    """Exact cell indices [n, 3] (int64) of points in an R^3 map."""
    if R < 2 or (R & (R - 1)) != 0:
        raise ValueError("R must be a power of two >= 2")
    x = np.asarray(xyz, dtype=np.float64)
    s = R // 2
    with np.errstate(invalid="ignore"):
        v = np.floor(x * s)
    v = np.where(np.isnan(v), -s, v)
    v = np.clip(v, -s, s - 1) + s
    return v.astype(np.int64)


def lookup_depth(xyz, dmap, L, mode=MODE_ADAPTIVE, forced=None, max_depth=0):
    """Exit depth per point (int64 [n]); see step 2 of the module header."""
    n = np.asarray(xyz).shape[0]
    if mode == MODE_FULL:
        d = np.full(n, L, dtype=np.int64)
    elif mode == MODE_FORCED:
        d = np.asarray(forced, dtype=np.int64).copy()
    else:
        R = dmap.shape[0]
        i = voxel_index(xyz, R)
        d = dmap[i[:, 0], i[:, 1], i[:, 2]].astype(np.int64)
    if max_depth > 0:
        d = np.minimum(d, max_depth)
    return d


def activation(model, j, z):
    """h_j = sigma_j(z_j) for the pre-activation z_j of layer j (step 4)."""
    om = model["omega"][j - 1]
    if model["activation"] == "finer":
        return np.sin(om * (np.abs(z) + 1.0) * z)
    return np.sin(om * z)


def activation_slope(model, j, z):
    """sigma_j'(z_j), the derivative of the activation (step 5)."""
    om = model["omega"][j - 1]
    if model["activation"] == "finer":
        return om * (2.0 * np.abs(z) + 1.0) * np.cos(om * (np.abs(z) + 1.0) * z)
    return om * np.cos(om * z)


def _tail(t, h):
    if t[0] == "linear":
        _, a, c = t
        return h @ a + c
    _, a0, c0, a1, c1 = t
    return (h @ a0 + c0) * (h @ a1 + c1)


def _tail_grad(t, h):
    if t[0] == "linear":
        return np.broadcast_to(t[1], h.shape)
    _, a0, c0, a1, c1 = t
    return (h @ a1 + c1)[:, None] * a0[None, :] + (h @ a0 + c0)[:, None] * a1[None, :]


def forward(model, xyz, d, far=None):
    """y_{d(x)} in float64 [n] for exit depths ``d`` (int array [n]).

    ``far``: FP32 [R, R, R] far-field values, read for points with d = 0.
    """
    x = np.asarray(xyz, dtype=np.float64)
    d = np.asarray(d, dtype=np.int64)
    n = x.shape[0]
    if np.any(d < 0) or np.any(d > model["L"]):
        raise ValueError("exit depth out of range")
    y = np.zeros(n, dtype=np.float64)
    zero = np.nonzero(d == 0)[0]
    if zero.size:
        if far is None:
            raise ValueError("depth-0 points need a far-field grid")
        i = voxel_index(x[zero], far.shape[0])
        y[zero] = far[i[:, 0], i[:, 1], i[:, 2]].astype(np.float64)
    rows = np.nonzero(d >= 1)[0]
    h = x[rows]
    for j in range(1, model["L"] + 1):
        if rows.size == 0:
            break
        z = h @ model["W_"][j - 1].T + model["b_"][j - 1]
        h = activation(model, j, z)
        y[rows] += _tail(model["tails"][j - 1], h)
        keep = d[rows] > j
        rows, h = rows[keep], h[keep]
    return y


def forward_all_tails(model, xyz):
    """All accumulated outputs y_1..y_L, float64 [n, L] (Eq. 2)."""
    h = np.asarray(xyz, dtype=np.float64)
    out = np.zeros((h.shape[0], model["L"]), dtype=np.float64)
    y = np.zeros(h.shape[0], dtype=np.float64)
    for j in range(1, model["L"] + 1):
        z = h @ model["W_"][j - 1].T + model["b_"][j - 1]
        h = activation(model, j, z)
        y = y + _tail(model["tails"][j - 1], h)
        out[:, j - 1] = y
    return out


def gradient(model, xyz, d):
    """grad_x y_{d(x)} with d held fixed, float64 [n, 3]."""
    x = np.asarray(xyz, dtype=np.float64)
    d = np.asarray(d, dtype=np.int64)
    g_out = np.zeros_like(x)
    for k in np.unique(d):
        if k <= 0:
            continue
        rows = np.nonzero(d == k)[0]
        hs, zs = [x[rows]], []
        for j in range(1, k + 1):
            z = hs[-1] @ model["W_"][j - 1].T + model["b_"][j - 1]
            zs.append(z)
            hs.append(activation(model, j, z))
        g = np.array(_tail_grad(model["tails"][k - 1], hs[k]))
        for j in range(k, 0, -1):
            delta = activation_slope(model, j, zs[j - 1]) * g
            g = delta @ model["W_"][j - 1]
            if j > 1:
                g = g + _tail_grad(model["tails"][j - 2], hs[j - 1])
        g_out[rows] = g
    return g_out
