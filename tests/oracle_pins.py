"""Checks that pin the FP64 oracle to facts outside itself.

Each ``check_*`` raises AssertionError when the oracle disagrees with what the
paper or the mathematics fixes. ``test_oracle_pins.py`` runs them on the real
oracle; ``test_oracle_mutants.py`` plants plausible mistakes in the oracle
and asserts that some check fails for each.
"""

import math
from fractions import Fraction

import mpmath
import numpy as np
import torch

import oracle
import oracle.depthmap as D
import oracle.dynamic as DY
import oracle.octree as OT
import oracle.scalar
import oracle.tmlp as T
import synth


def tiny_model(seed, L, W, tails="mult", scale="plain", activation="sine"):
    return oracle.parse_blob(synth.write_blob(
        synth.siren_tmlp(seed, L, W, tails=tails, scale=scale, activation=activation)))


# -- cell rule ---------------------------------------------------------------

def edge_coordinates(R):
    """FP32 coordinates on, beside and beyond every cell face of an R-map."""
    vals = [0.0, -0.0, 1.0, -1.0, 1e-30, -1e-30, 1.5, -1.5, 3e38, -3e38,
            float("inf"), float("-inf"), float("nan")]
    for i in range(R + 1):
        f = np.float32(-1.0 + 2.0 * i / R)
        vals += [float(f), float(np.nextafter(f, np.float32(2))),
                 float(np.nextafter(f, np.float32(-2)))]
    rng = np.random.Generator(np.random.PCG64(7))
    vals += list(rng.uniform(-1.1, 1.1, size=200).astype(np.float32))
    return np.array(vals, dtype=np.float32)


def cell_by_rational_box(x, R):
    """Cell of one coordinate by exact half-open interval membership."""
    if math.isnan(x):
        return 0
    if x == float("inf"):
        return R - 1
    if x == float("-inf"):
        return 0
    q = Fraction(float(x))
    for i in range(R):
        lo = Fraction(-1) + Fraction(2 * i, R)
        hi = Fraction(-1) + Fraction(2 * (i + 1), R)
        if lo <= q < hi:
            return i
    return 0 if q < -1 else R - 1


def check_cell_rule(R):
    xs = edge_coordinates(R)
    pts = np.stack([xs, xs[::-1], np.roll(xs, 5)], axis=1)
    got = T.voxel_index(pts, R)
    for a in range(3):
        want = [cell_by_rational_box(float(v), R) for v in pts[:, a]]
        assert np.array_equal(got[:, a], want), f"cell rule wrong for R={R}"


# -- forward pass --------------------------------------------------------------

def torch_textbook_mlp(model):
    """Eq. 1 MLP from torch.nn layers: Linear/sin stack + a Linear output.

    Uses the model's hidden layers and its last tail (which must be linear)
    as the output layer; intermediate tails play no part.
    """
    L, W = model["L"], model["W"]
    layers = []
    for j in range(L):
        fan_in = 3 if j == 0 else W
        lin = torch.nn.Linear(fan_in, W, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(model["W_"][j]))
            lin.bias.copy_(torch.from_numpy(model["b_"][j]))
        layers.append((lin, model["omega"][j]))
    kind, a, c = model["tails"][L - 1]
    assert kind == "linear"
    out = torch.nn.Linear(W, 1, dtype=torch.float64)
    with torch.no_grad():
        out.weight.copy_(torch.from_numpy(a)[None, :])
        out.bias.fill_(float(c))

    def f(x):
        h = x
        for lin, om in layers:
            h = torch.sin(om * lin(h))
        return out(h)[:, 0]
    return f


def with_zeroed_intermediate_tails(model):
    m = dict(model)
    tails = []
    for i, t in enumerate(model["tails"]):
        if i < model["L"] - 1:
            z = np.zeros(model["W"])
            tails.append(("linear", z, 0.0) if t[0] == "linear" else ("mult", z, 0.0, z, 0.0))
        else:
            tails.append(("linear", t[1], t[2]) if t[0] == "linear" else None)
    m["tails"] = tails
    return m


def check_textbook_mlp(seed=3, L=4, W=16, n=300):
    model = with_zeroed_intermediate_tails(tiny_model(seed, L, W, tails="linear"))
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    want = torch_textbook_mlp(model)(torch.from_numpy(x)).detach().numpy()
    got = T.forward(model, x, np.full(n, L))
    assert np.allclose(got, want, rtol=0, atol=1e-12), "textbook MLP reduction"


def check_quadratic_form(seed=5, W=24, n=50):
    """Appendix: (a.h + c)(b.h + d) = h^T Q h + u^T h + s,
    Q = a b^T, u = d a + c b, s = c d."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a, b = rng.normal(size=W), rng.normal(size=W)
    c, d = rng.normal(), rng.normal()
    h = rng.uniform(-1, 1, size=(n, W))
    Q = np.outer(a, b)
    u = d * a + c * b
    s = c * d
    want = np.einsum("ni,ij,nj->n", h, Q, h) + h @ u + s
    got = T._tail(("mult", a, c, b, d), h)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12), "quadratic form"


def truncated(model, k):
    return {"L": k, "W": model["W"], "omega": model["omega"][:k],
            "activation": model["activation"],
            "W_": model["W_"][:k], "b_": model["b_"][:k], "tails": model["tails"][:k]}


def check_truncation(seed=11, L=5, W=12, n=200, activation="sine"):
    model = tiny_model(seed, L, W, activation=activation)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    d = rng.integers(1, L + 1, size=n)
    got = T.forward(model, x, d)
    for k in range(1, L + 1):
        sel = d == k
        want = T.forward(truncated(model, k), x[sel], np.full(sel.sum(), k))
        assert np.allclose(got[sel], want, rtol=0, atol=1e-13), f"exit at {k}"
    allt = T.forward_all_tails(model, x)
    assert np.allclose(got, allt[np.arange(n), d - 1], rtol=0, atol=1e-13)


def check_accumulation(seed=13, L=5, W=12, n=100):
    """Only tail k non-zero: y_d = 0 for d < k and y_d = t_k for every d >= k."""
    base = tiny_model(seed, L, W)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    for k in range(1, L + 1):
        m = dict(base)
        z = np.zeros(W)
        m["tails"] = [t if i == k - 1 else ("linear", z, 0.0)
                      for i, t in enumerate(base["tails"])]
        ys = [T.forward(m, x, np.full(n, d)) for d in range(1, L + 1)]
        for d in range(1, k):
            assert np.all(ys[d - 1] == 0.0), "tail contributes before its layer"
        tk = [oracle.scalar.forward_point(m, x[i], k) for i in range(5)]
        for d in range(k, L + 1):
            assert np.allclose(ys[d - 1], ys[k - 1], rtol=0, atol=0), "not cumulative"
        assert np.allclose(ys[k - 1][:5], tk, rtol=0, atol=1e-13)
        assert np.any(ys[k - 1] != 0.0)


def check_scalar_twin(seed=17, L=3, W=8, activation="sine"):
    model = tiny_model(seed, L, W, activation=activation)
    x = synth.grid_points(8).astype(np.float64)
    d = (np.arange(x.shape[0]) % L) + 1
    got = T.forward(model, x, d)
    want = np.array([oracle.scalar.forward_point(model, x[i], int(d[i]))
                     for i in range(x.shape[0])])
    assert np.allclose(got, want, rtol=0, atol=1e-12), "scalar twin"


def check_mpmath(seed=19, L=2, W=6, n=10, activation="sine"):
    """Closed form at 50 digits: y_2 = sum of both tails of a 2-layer net."""
    model = tiny_model(seed, L, W, activation=activation)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    got = T.forward(model, x, np.full(n, L))
    mpmath.mp.dps = 50
    mp = mpmath.mpf
    for i in range(n):
        h = [mp(float(v)) for v in x[i]]
        y = mp(0)
        for j in range(L):
            Wj, bj, om = model["W_"][j], model["b_"][j], mp(model["omega"][j])
            z = [mpmath.fsum(mp(float(Wj[u, k])) * h[k] for k in range(len(h))) + mp(float(bj[u]))
                 for u in range(W)]
            if activation == "finer":
                h = [mpmath.sin(om * (abs(v) + 1) * v) for v in z]
            else:
                h = [mpmath.sin(om * v) for v in z]
            t = model["tails"][j]
            dot = lambda v: mpmath.fsum(mp(float(v[k])) * h[k] for k in range(W))
            if t[0] == "linear":
                y += dot(t[1]) + mp(float(t[2]))
            else:
                y += (dot(t[1]) + mp(float(t[2]))) * (dot(t[3]) + mp(float(t[4])))
        assert abs(float(y) - got[i]) < 1e-13, "mpmath spot value"


def check_lod_and_far(seed=23, L=4, W=8, R=8):
    model = tiny_model(seed, L, W)
    rng = np.random.Generator(np.random.PCG64(seed))
    dmap = rng.integers(0, L + 1, size=(R, R, R)).astype(np.uint8)
    far = rng.normal(size=(R, R, R)).astype(np.float32)
    x = synth.grid_points(16).astype(np.float64)
    d = T.lookup_depth(x, dmap, L)
    i = T.voxel_index(x, R)
    assert np.array_equal(d, dmap[i[:, 0], i[:, 1], i[:, 2]])
    y = T.forward(model, x, d, far=far)
    zero = d == 0
    assert np.array_equal(y[zero], far[i[zero, 0], i[zero, 1], i[zero, 2]].astype(np.float64))
    allt = T.forward_all_tails(model, x)
    for m in range(1, L + 1):
        dm = T.lookup_depth(x, dmap, L, max_depth=m)
        assert np.array_equal(dm, np.minimum(d, m))
        ym = T.forward(model, x, dm, far=far)
        nz = dm > 0
        assert np.allclose(ym[nz], allt[nz, dm[nz] - 1], rtol=0, atol=1e-13)
    full = T.lookup_depth(x, dmap, L, mode=T.MODE_FULL)
    assert np.all(full == L)
    allL = np.full((R, R, R), L, dtype=np.uint8)
    assert np.array_equal(T.lookup_depth(x, allL, L), full)
    assert np.allclose(T.forward(model, x, full), allt[:, L - 1], rtol=0, atol=1e-13)


# -- gradient ------------------------------------------------------------------

def torch_tmlp(model):
    Ws = [torch.from_numpy(w) for w in model["W_"]]
    bs = [torch.from_numpy(b) for b in model["b_"]]
    finer = model["activation"] == "finer"

    def f(x, k):
        h, y = x, torch.zeros(x.shape[0], dtype=torch.float64)
        for j in range(k):
            z = h @ Ws[j].T + bs[j]
            h = torch.sin(model["omega"][j] * ((torch.abs(z) + 1) * z if finer else z))
            t = model["tails"][j]
            if t[0] == "linear":
                y = y + h @ torch.from_numpy(t[1]) + t[2]
            else:
                y = y + (h @ torch.from_numpy(t[1]) + t[2]) * (h @ torch.from_numpy(t[3]) + t[4])
        return y
    return f


def check_gradient_autograd(seed=29, L=4, W=16, n=120, activation="sine"):
    model = tiny_model(seed, L, W, activation=activation)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    d = rng.integers(1, L + 1, size=n)
    got = T.gradient(model, x, d)
    f = torch_tmlp(model)
    for k in range(1, L + 1):
        sel = np.nonzero(d == k)[0]
        xt = torch.from_numpy(x[sel]).requires_grad_(True)
        f(xt, k).sum().backward()
        assert np.allclose(got[sel], xt.grad.numpy(), rtol=1e-10, atol=1e-10), f"grad depth {k}"


def check_gradient_fd(seed=31, L=3, W=10, n=60, h=1e-6, activation="sine"):
    model = tiny_model(seed, L, W, activation=activation)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    d = rng.integers(1, L + 1, size=n)
    got = T.gradient(model, x, d)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (T.forward(model, x + e, d) - T.forward(model, x - e, d)) / (2 * h)
        scale = 1.0 + np.abs(got[:, a])
        assert np.all(np.abs(fd - got[:, a]) <= 1e-6 * scale), "central difference"


# -- FINER activation (SAND-FINER backbone, Sec. 4.1) --------------------------

def _finer_root(om, k):
    """The positive z with om (z + 1) z = k pi / 2, solved at 50 digits."""
    mpmath.mp.dps = 50
    c = mpmath.mpf(k) * mpmath.pi / 2 / mpmath.mpf(om)
    return float((mpmath.sqrt(1 + 4 * c) - 1) / 2)


def check_finer_roots():
    """sin(om (|z| + 1) z) is 0 where om (|z| + 1) z = m pi, (-1)^m where it
    is (m + 1/2) pi, and odd in z: at the roots of the quadratic, not by
    evaluating the formula."""
    for om in (30.0, 7.5, 1.0):
        m = {"L": 1, "omega": [om], "activation": "finer"}
        for k in range(1, 81):
            z = _finer_root(om, k)
            v = T.activation(m, 1, np.array([z, -z, 0.0]))
            assert v[2] == 0.0
            assert v[1] == -v[0], "FINER activation must be odd"
            if k % 2 == 0:
                assert abs(v[0]) <= 2e-13, f"om={om}: zero at k={k}: {v[0]}"
            else:
                want = (-1.0) ** ((k - 1) // 2)
                assert abs(v[0] - want) <= 1e-12, f"om={om}: extremum at k={k}: {v[0]}"


def check_finer_slope():
    """The activation's derivative against fourth-order central differences
    of the activation itself (away from the kink of |z| at 0, where the
    slope is om)."""
    rng = np.random.Generator(np.random.PCG64(71))
    z = np.concatenate([rng.uniform(-2, -0.01, 300), rng.uniform(0.01, 2, 300)])
    for act in ("finer", "sine"):
        for om in (30.0, 2.5):
            m = {"L": 1, "omega": [om], "activation": act}
            h = 1e-4
            f = lambda v: T.activation(m, 1, v)
            fd = (8 * (f(z + h) - f(z - h)) - (f(z + 2 * h) - f(z - 2 * h))) / (12 * h)
            got = T.activation_slope(m, 1, z)
            assert np.all(np.abs(fd - got) <= 1e-6 * (1 + np.abs(got))), f"{act} slope, om={om}"
            assert abs(T.activation_slope(m, 1, np.array([0.0]))[0] - om) < 1e-12


# -- network-depth map construction (Sec. 3.2, Eq. 5-7) ----------------------

def _sign(v):
    return (v > 0) - (v < 0)


def required_depth_loop(row, r):
    """Eq. 5 (near case) written out for one point, pure Python."""
    yL = float(row[-1])
    for i, v in enumerate(row):
        if abs(yL - float(v)) < r and _sign(float(v)) == _sign(yL):
            return i + 1
    raise AssertionError("the last layer always qualifies")


def check_required_depth_definition(seed=37, n=3000, L=6, r=0.25):
    """Values on a lattice of r/2 (exact in binary), so ties |y_L - y_i| = r,
    zeros and sign changes all occur."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = rng.integers(-6, 7, size=(n, L)).astype(np.float64) * (r / 2)
    got = D.required_depth(y, r)
    exp = np.array([required_depth_loop(row, r) for row in y])
    assert np.array_equal(got, exp), f"{int((got != exp).sum())} rows differ from Eq. 5"


def check_required_depth_extremes(L=5, r=1e-3):
    rows = np.array([
        [0.3] * L,                        # every layer already at y_L: depth 1
        [1.0, 2.0, 3.0, 4.0, 5.0],        # nothing close before the last: depth L
        [-0.3, 0.3, 0.3, 0.3, 0.3],       # right value only from layer 2
        [0.3 + 5e-4, 0.3, -0.2, 0.3, 0.3],  # close at 1, far at 3: still depth 1 (min)
        [-1e-4, 2e-4, 0.0, 3e-4, 5e-5],   # within r of y_L but wrong sign until layer 2
        [0.0, 0.0, 0.0, 0.0, 0.0],        # sign(0) = sign(0): depth 1
    ])
    got = D.required_depth(rows, r)
    assert list(got) == [1, L, 2, 1, 2, 1], f"got {list(got)}"


def check_required_depth_monotone(seed=41, n=2000, L=8):
    rng = np.random.Generator(np.random.PCG64(seed))
    y = np.cumsum(rng.normal(0, 1, size=(n, L)) * 0.5 ** np.arange(L), axis=1)
    prev = None
    for r in (1e-6, 1e-3, 1e-2, 1e-1, 1.0, 10.0):
        d = D.required_depth(y, r)
        assert d.min() >= 1 and d.max() <= L, "depth outside 1..L"
        if prev is not None:
            assert np.all(d <= prev), "a larger threshold never needs more layers"
        prev = d


def check_vanishing_tails(seed=43, L=6, W=12, k=3, n=400):
    """Tails beyond layer k zero: y_i = y_k for i >= k, so d(x) <= k for any
    r > 0, and d(x) = k when r is below every earlier gap."""
    model = tiny_model(seed, L, W)
    tails = list(model["tails"])
    for j in range(k, L):
        t = tails[j]
        tails[j] = ("mult", np.zeros_like(t[1]), 0.0, np.zeros_like(t[3]), 0.0)
    model = dict(model, tails=tails)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    y = T.forward_all_tails(model, x)
    assert np.all(D.required_depth(y, 1e-3) <= k), "vanishing tails must cap the depth"
    d = D.required_depth(y, 1e-13)
    gaps = np.abs(y[:, k - 1:k] - y[:, :k - 1]).min(axis=1)
    sure = gaps > 1e-12
    assert sure.mean() > 0.99 and np.all(d[sure] == k), "depth must be exactly k"


def check_sample_lattice(R=128, s=4, seed=45):
    """With R = 128 and s = 4 the samples are the 512^3 grid's cell centres
    (2m+1)/512 - 1, m = 4 i + k, each inside its voxel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vox = np.concatenate([[0, R ** 3 - 1, R * R * 5 + R * 7 + 3],
                          rng.integers(0, R ** 3, size=60)])
    pts = D.sample_points(R, vox, s)
    assert pts.shape == (vox.size * s ** 3, 3)
    m = (pts + 1.0) * 256.0 - 0.5
    assert np.array_equal(m, np.round(m)), "samples off the 512^3 cell centres"
    m = m.astype(np.int64).reshape(vox.size, s ** 3, 3)
    ijk = np.stack([vox // (R * R), (vox // R) % R, vox % R], axis=1)
    assert np.all(m // s == ijk[:, None, :]), "a sample outside its voxel"
    for row in m:
        assert len({tuple(p) for p in row}) == s ** 3, "repeated sample in a voxel"
    first = m[:, 0, :] - s * ijk
    assert np.all(first == 0) and np.all(m[:, -1, :] - s * ijk == s - 1)


def check_construct_brute_force(seed=47, L=3, W=8, R=4, s=2, r=0.4):
    """Eq. 6-7 by brute force with the scalar twin on every sample."""
    model = tiny_model(seed, L, W)
    rng = np.random.Generator(np.random.PCG64(seed))
    near = rng.integers(0, 2, size=R ** 3).astype(np.uint8)
    csdf = rng.normal(0, 0.5, size=R ** 3)
    depth, far = D.construct(model, R, near, csdf, s, r)
    ambiguous = 0
    for v in range(R ** 3):
        if not near[v]:
            assert depth[v] == 0 and far[v] == csdf[v], f"far voxel {v}"
            continue
        assert far[v] == 0.0
        i = (v // (R * R), (v // R) % R, v % R)
        best = 0
        for kx in range(s):
            for ky in range(s):
                for kz in range(s):
                    x = [-1.0 + (2.0 / R) * (i[a] + (k + 0.5) / s)
                         for a, k in enumerate((kx, ky, kz))]
                    ys = [oracle.scalar.forward_point(model, x, j) for j in range(1, L + 1)]
                    if min(abs(abs(ys[-1] - yj) - r) for yj in ys) < 1e-9:
                        ambiguous += 1
                    best = max(best, required_depth_loop(ys, r))
        assert depth[v] == best, f"voxel {v}: {depth[v]} vs brute force {best}"
    assert ambiguous == 0, "a sample sits on the threshold; pick another r"
    assert len(set(depth[near == 1].tolist())) > 1, "the case should exercise several depths"


# -- map-free dynamic early exit (Sec. 4.4 ablation) ------------------------

def dynamic_exit_loop(trow, r, max_depth=0):
    """The exit rule written out for one point, pure Python."""
    L = len(trow)
    d = L
    for i in range(2, L + 1):
        if abs(float(trow[i - 1])) < r:
            d = i
            break
    return min(d, max_depth) if max_depth > 0 else d


def check_dynamic_definition(seed=53, n=3000, L=6, r=0.25):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = rng.integers(-4, 5, size=(n, L)).astype(np.float64) * (r / 2)
    for md in (0, 3):
        got = DY.exit_from_tails(t, r, md)
        exp = np.array([dynamic_exit_loop(row, r, md) for row in t])
        assert np.array_equal(got, exp), f"{int((got != exp).sum())} rows differ (max_depth {md})"


def check_dynamic_hand_cases(r=1e-3):
    t = np.array([
        [0.0, 0.0, 0.0, 0.0],      # layer 1 is never tested: exit at 2
        [0.5, 0.5, 5e-4, 0.0],     # first small residual at 3
        [0.5, -1e-3, 0.5, 0.5],    # |t| = r is not below r: runs to L
        [0.5, 0.5, 0.5, 0.5],      # no small residual: L
        [0.5, -9e-4, 0.0, 0.0],    # negative residual counts by magnitude: 2
    ])
    assert list(DY.exit_from_tails(t, r)) == [2, 3, 4, 4, 2]
    assert list(DY.exit_from_tails(t[:, :1], r)) == [1] * 5, "a one-layer net exits at 1"


def check_dynamic_monotone_and_tails(seed=55, L=6, W=12, n=300):
    model = tiny_model(seed, L, W)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    t = DY.tails(model, x)
    y = T.forward_all_tails(model, x)
    assert np.allclose(np.cumsum(t, axis=1), y, rtol=0, atol=1e-12), "tails must sum to y_i"
    prev = None
    for r in (1e-6, 1e-2, 1e-1, 1.0, 10.0):
        d = DY.exit_from_tails(t, r)
        assert d.min() >= 2 and d.max() <= L
        if prev is not None:
            assert np.all(d <= prev), "a larger threshold never runs deeper"
        prev = d
    yd, dd = DY.dynamic_forward(model, x, 1e-1)
    assert np.array_equal(dd, DY.exit_from_tails(t, 1e-1))
    assert np.allclose(yd, y[np.arange(n), dd - 1], rtol=0, atol=1e-12)


def check_dynamic_vanishing_tails(seed=57, L=6, W=12, k=3, n=300):
    model = tiny_model(seed, L, W)
    tl = list(model["tails"])
    for j in range(k, L):
        t = tl[j]
        tl[j] = ("mult", np.zeros_like(t[1]), 0.0, np.zeros_like(t[3]), 0.0)
    model = dict(model, tails=tl)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-1, 1, size=(n, 3))
    _, d = DY.dynamic_forward(model, x, 1e-13)
    t = DY.tails(model, x)
    sure = (np.abs(t[:, 1:k]) > 1e-12).all(axis=1)
    assert sure.mean() > 0.99 and np.all(d[sure] == k + 1), "exit right after the last live tail"


def check_dynamic_scalar_twin(seed=59, L=4, W=8, r=0.3):
    model = tiny_model(seed, L, W)
    x = synth.grid_points(4).astype(np.float64)
    _, d = DY.dynamic_forward(model, x, r)
    for i, p in enumerate(x):
        ys = [oracle.scalar.forward_point(model, p, j) for j in range(1, L + 1)]
        tr = [ys[0]] + [ys[j] - ys[j - 1] for j in range(1, L)]
        assert min(abs(abs(v) - r) for v in tr[1:]) > 1e-9, "sample on the threshold"
        assert d[i] == dynamic_exit_loop(tr, r), f"point {i}"


# -- sparse network-depth octree (Sec. 3.2, Eq. 5-7) -------------------------

def constant_model(c, L=3, W=8, seed=61):
    """y_i = c for every i: tail 1 is the constant c, later tails vanish."""
    m = tiny_model(seed, L, W)
    tl = [("linear", np.zeros(W), float(c))]
    for t in m["tails"][1:]:
        tl.append(("mult", np.zeros(W), 0.0, np.zeros(W), 0.0))
    return dict(m, tails=tl)


def _brute_tree(model, D, s, r):
    """Top-down recursion with the scalar twin, pure Python."""
    L = model["L"]
    internal = [set() for _ in range(D)]
    leaves = {}

    def yl(p):
        return oracle.scalar.forward_point(model, p, L)

    def visit(l, ijk):
        side = 2.0 / (1 << l)
        c = [-1.0 + (v + 0.5) * side for v in ijk]
        y = yl(c)
        hit = abs(y) <= math.sqrt(3.0) * 2.0 ** (-l)
        assert abs(abs(y) - math.sqrt(3.0) * 2.0 ** (-l)) > 1e-9, "centre on the test boundary"
        if hit and l < D:
            internal[l].add(ijk)
            for a in (0, 1):
                for b in (0, 1):
                    for e in (0, 1):
                        visit(l + 1, (2 * ijk[0] + a, 2 * ijk[1] + b, 2 * ijk[2] + e))
        elif hit:
            best = 0
            for ka in range(s):
                for kb in range(s):
                    for kc in range(s):
                        p = [-1.0 + side * (ijk[ax] + (kk + 0.5) / s)
                             for ax, kk in enumerate((ka, kb, kc))]
                        ys = [oracle.scalar.forward_point(model, p, j) for j in range(1, L + 1)]
                        best = max(best, required_depth_loop(ys, r))
            leaves[(l,) + ijk] = (best, 0.0)
        else:
            leaves[(l,) + ijk] = (0, y)

    visit(0, (0, 0, 0))
    return internal, leaves


def check_octree_brute_force(seed=63, L=3, W=10, D=3, s=2, r=0.3):
    model = tiny_model(seed, L, W)
    tree = OT.build(model, D, s, r)
    internal, leaves = _brute_tree(model, D, s, r)
    for l in range(D):
        assert tree["internal"][l] == internal[l], f"internal nodes differ at level {l}"
    assert set(tree["leaves"]) == set(leaves), "leaf sets differ"
    for k, (d, v) in leaves.items():
        dd, vv = tree["leaves"][k]
        assert dd == d and abs(vv - v) < 1e-12, f"leaf {k}: {tree['leaves'][k]} vs {(d, v)}"
    assert sum(1 for k, (d, _) in leaves.items() if d > 0) > 0, "case should have near leaves"
    assert len({k[0] for k in leaves}) > 1, "case should have leaves on several levels"


def check_octree_constant_models(D=3):
    t = OT.build(constant_model(2.0), D, 1, 1e-3)
    assert t["leaves"] == {(0, 0, 0, 0): (0, 2.0)} and not t["internal"][0]
    d, v, lv = OT.lookup(t, np.array([[0.1, -0.7, 0.99]]))
    assert (d[0], v[0], lv[0]) == (0, 2.0, 0)
    t = OT.build(constant_model(0.0), D, 2, 1e-3)
    assert len(t["leaves"]) == 8 ** D and all(k[0] == D and dv == (1, 0.0)
                                              for k, dv in t["leaves"].items())
    t = OT.build(constant_model(0.3), D, 1, 1e-3)          # h = 1.73, .87, .43 > .3 > .22
    assert len(t["leaves"]) == 8 ** 3 and all(k[0] == 3 and dv == (0, 0.3)
                                              for k, dv in t["leaves"].items())
    c = OT.SQRT3 * 0.25                                    # |y| = h exactly at level 2
    t = OT.build(constant_model(c), D, 1, 1e-3)
    assert len(t["internal"][2]) == 64 and all(k[0] == 3 for k in t["leaves"]), \
        "a centre exactly half a diagonal away intersects"


def check_octree_invariants(seed=65, L=3, W=10, D=4, s=1, r=0.3):
    model = tiny_model(seed, L, W)
    t = OT.build(model, D, s, r)
    vol = sum(8 ** (D - k[0]) for k in t["leaves"])
    assert vol == 8 ** D, "leaves must tile the cube exactly"
    for (l, i, j, k), (d, v) in t["leaves"].items():
        if l > 0:
            assert (i // 2, j // 2, k // 2) in t["internal"][l - 1], "a leaf's parent is internal"
        c = OT.centres(l, [[i, j, k]])
        y = OT.y_last(model, c)[0]
        if d > 0:
            assert l == D and abs(y) <= OT.SQRT3 * 2.0 ** (-l), "near leaves sit at level D"
        else:
            assert abs(v - y) < 1e-12, "far leaves store y_L at their centre"
            assert l == D or abs(y) > OT.SQRT3 * 2.0 ** (-l), "a far leaf above D misses the shape"
    for l in range(D):
        for ijk in t["internal"][l]:
            y = OT.y_last(model, OT.centres(l, [ijk]))[0]
            assert abs(y) <= OT.SQRT3 * 2.0 ** (-l)


def check_octree_lookup(seed=67, L=3, W=10, D=4, n=400):
    model = tiny_model(seed, L, W)
    t = OT.build(model, D, 1, 0.3)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.concatenate([rng.uniform(-1, 1, size=(n, 3)), edge_coordinates(1 << D)[:60, None]
                        * np.ones((1, 3))])
    d, v, lv = OT.lookup(t, x)
    for q in range(x.shape[0]):
        l = int(lv[q])
        ijk = tuple(T.voxel_index(x[q:q + 1], 1 << l)[0]) if l > 0 else (0, 0, 0)
        assert (l,) + tuple(int(a) for a in ijk) in t["leaves"], f"point {q}: not its leaf"
        assert t["leaves"][(l,) + tuple(int(a) for a in ijk)] == (d[q], v[q])


ALL_CHECKS = [
    lambda: [check_cell_rule(R) for R in (2, 4, 32, 128)],
    check_textbook_mlp, check_quadratic_form, check_truncation,
    check_accumulation, check_scalar_twin, check_mpmath, check_lod_and_far,
    check_gradient_autograd, check_gradient_fd,
    check_required_depth_definition, check_required_depth_extremes,
    check_required_depth_monotone, check_vanishing_tails, check_sample_lattice,
    check_construct_brute_force,
    check_dynamic_definition, check_dynamic_hand_cases, check_dynamic_monotone_and_tails,
    check_dynamic_vanishing_tails, check_dynamic_scalar_twin,
    check_octree_brute_force, check_octree_constant_models, check_octree_invariants,
    check_octree_lookup,
    check_finer_roots, check_finer_slope,
    lambda: check_scalar_twin(activation="finer"),
    lambda: check_mpmath(activation="finer"),
    lambda: check_truncation(activation="finer"),
    lambda: check_gradient_autograd(activation="finer"),
    lambda: check_gradient_fd(activation="finer"),
]
