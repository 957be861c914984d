"""SAND-FINER: the query path on the FINER backbone (Sec. 4.1, Table 1's
SAND-FINER rows), h = sin(omega (|z| + 1) z), against the FP64 oracle
(needs an MI355X).

Every part of the path that evaluates the network runs with the model's
activation: adaptive, full, forced and dynamic queries, the input
gradient, the serving loop (which must not batch models of different
activations into one launch), and the octree built from the network.
Bars as for the SIREN backbone: exit depths bit-exact, values within 1e-5
(FP32) and 2e-3 (BF16/FP16) of the oracle, gradients within the per-point
bounds of the gradient tests.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.dynamic as DY
import oracle.octree as OT
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c2_blob, c2_map, c2_points, finer_blob

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GTOL = {"fp32": (1e-4, 1e-4), "bf16": (3e-2, 1e-2), "fp16": (1e-2, 5e-3)}


def say(msg):
    print(msg, flush=True)


def run(model, dm, x, **kw):
    xyz = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    depth = torch.full((len(x),), 255, dtype=torch.uint8, device=DEV)
    y = sand.query(model, dm, xyz, depth_out=depth, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), depth.cpu().numpy().astype(np.int64)


def assert_close(got, want, tol, what):
    assert not np.isnan(got).any(), f"{what}: NaN"
    err = np.abs(got - want)
    say(f"  {what}: n={got.size} max|err|={err.max():.3e} mean={err.mean():.3e}")
    assert err.max() <= tol, f"{what}: max |err| {err.max():.3e} > {tol:.1e}"


def check_grad(got, want, prec, what):
    rel, ab = GTOL[prec]
    err = np.linalg.norm(got - want, axis=1)
    nrm = np.linalg.norm(want, axis=1)
    ratio = err / (rel * nrm + ab)
    say(f"  {what}: n={len(err)} max|dg|/|g|={np.max(err / np.maximum(nrm, 1e-12)):.3e} "
        f"mean|g|={nrm.mean():.3f} worst/tol={ratio.max():.3f}")
    assert ratio.max() <= 1.0, f"{what}: gradient error over tolerance"


@pytest.fixture(scope="module")
def c2f():
    blob = finer_blob(256)
    ref = oracle.parse_blob(blob)
    assert ref["activation"] == "finer"
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    return blob, ref, model, dmap, sand.build_depthmap(model, dmap)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_finer_8x256_adaptive_and_full(c2f, prec):
    blob, ref, model, dmap, dm = c2f
    x = c2_points(65536, seed=41)
    say(f"case: FINER 8x256 residual tails, 128^3 map, 65536 points, {prec} adaptive")
    y, d = run(model, dm, x, precision=prec)
    want_d = oracle.lookup_depth(x, dmap, 8)
    assert np.array_equal(d, want_d)
    assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"FINER 8x256 {prec} adaptive")
    xs = x[:8192]
    y, _ = run(model, dm, xs, precision=prec, mode="full")
    assert_close(y, oracle.forward(ref, xs, np.full(len(xs), 8)), TOL[prec],
                 f"FINER 8x256 {prec} full")


def test_finer_differs_from_siren(c2f):
    """The same weights on the two backbones give different outputs, and
    each matches its own oracle: the activation byte is honoured."""
    blob, ref, model, dmap, dm = c2f
    sblob = c2_blob(256)
    sref = oracle.parse_blob(sblob)
    x = c2_points(4096, seed=5)
    forced = torch.full((len(x),), 8, dtype=torch.uint8, device=DEV)
    yf, _ = run(model, None, x, precision="fp32", mode="forced", forced_depth=forced)
    ys = oracle.forward(sref, x, np.full(len(x), 8))
    assert np.abs(yf - ys).max() > 1e-2, "FINER model evaluated with the SIREN sine"
    assert_close(yf, oracle.forward(ref, x, np.full(len(x), 8)), TOL["fp32"], "forced depth 8")


def test_finer_layer1_large_arguments(c2f):
    """Depth 1 at points inside the cube and out to 4 units: the FINER
    argument omega (|z| + 1) z grows quadratically, so the first layer's
    FP32-accurate argument is what keeps the error down in every precision."""
    blob, ref, model, dmap, dm = c2f
    rng = np.random.Generator(np.random.PCG64(57))
    x = np.concatenate([rng.uniform(-1, 1, size=(32768, 3)),
                        rng.uniform(-4, 4, size=(8192, 3))]).astype(np.float32)
    forced = torch.ones(len(x), dtype=torch.uint8, device=DEV)
    want = oracle.forward(ref, x, np.ones(len(x), dtype=np.int64))
    err = {}
    for prec in ("fp32", "bf16", "fp16"):
        y, _ = run(model, None, x, precision=prec, mode="forced", forced_depth=forced)
        err[prec] = float(np.abs(y - want).max())
        say(f"  FINER depth 1, {prec}: max|err| {err[prec]:.3e}")
    inside = slice(0, 32768)
    y, _ = run(model, None, x[inside], precision="fp32", mode="forced", forced_depth=forced[inside])
    assert_close(y, want[inside], TOL["fp32"], "FINER depth 1 inside the cube")
    for prec in ("bf16", "fp16"):
        assert err[prec] <= 2.0 * err["fp32"] + 1e-6, (prec, err)


@pytest.mark.parametrize("W", [16, 64, 128, 200, 336])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_finer_widths(W, prec):
    say(f"case: FINER width {W} (padded), 4 layers, {prec}")
    blob = synth.write_blob(synth.siren_tmlp(90 + W, 4, W, tails="mult", activation="finer"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(W))
    dmap = rng.integers(1, 5, size=(16, 16, 16)).astype(np.uint8)
    dm = sand.build_depthmap(model, dmap)
    x = rng.uniform(-1, 1, size=(3000, 3)).astype(np.float32)
    y, d = run(model, dm, x, precision=prec)
    want_d = oracle.lookup_depth(x, dmap, 4)
    assert np.array_equal(d, want_d)
    assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"FINER W={W} {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_finer_gradient_camera_rays(c2f, prec):
    blob, ref, model, dmap, dm = c2f
    x = synth.camera_ray_points(synth.random_primitives(2000), 77, width=240, height=135)
    say(f"case: FINER 8x256 gradient, {len(x)} camera-ray samples, {prec}")
    xyz = torch.from_numpy(x).to(DEV)
    sdf = torch.empty(len(x), dtype=torch.float32, device=DEV)
    g = sand.query_grad(model, dm, xyz, sdf_out=sdf, precision=prec)
    torch.cuda.synchronize()
    d = oracle.lookup_depth(x, dmap, 8)
    check_grad(g.cpu().numpy().astype(np.float64), oracle.gradient(ref, x, d), prec,
               f"FINER 8x256 {prec}")
    q = sand.query(model, dm, xyz, precision=prec)
    assert torch.equal(q, sdf), "the gradient call's values differ from sand_query's"


def test_finer_gradient_central_differences(c2f):
    """FP32 gradient vs Richardson-extrapolated central differences of the
    FP64 oracle (depth frozen)."""
    blob, ref, model, dmap, dm = c2f
    x = synth.camera_ray_points(synth.random_primitives(2000), 5, width=64, height=36)
    x64 = x.astype(np.float64)
    d = oracle.lookup_depth(x64, dmap, 8)
    g = sand.query_grad(model, dm, torch.from_numpy(x).to(DEV), precision="fp32")
    g = g.cpu().numpy().astype(np.float64)

    def fd(h):
        out = np.zeros_like(x64)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            out[:, a] = (oracle.forward(ref, x64 + e, d) - oracle.forward(ref, x64 - e, d)) / (2 * h)
        return out
    rich = (4 * fd(5e-4) - fd(1e-3)) / 3
    nrm = np.linalg.norm(rich, axis=1)
    e_rich = np.linalg.norm(g - rich, axis=1)
    say(f"  FINER FP32 gradient vs Richardson FD: max rel {np.max(e_rich / nrm):.3e}")
    assert np.all(e_rich <= 1e-3 * nrm + 1e-4)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_finer_dynamic_exit(prec):
    """Map-free dynamic exit on a FINER model: the GPU's exits equal the
    oracle's except where a tested tail lies within eps of r (90 % agreement
    for BF16, whose tails carry about 1e-4 of error), and its values equal
    the oracle's output at the GPU's exit depth."""
    r = 0.05
    blob = synth.write_blob(synth.siren_tmlp(73, 4, 64, tails="mult", scale="plain",
                                             activation="finer"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    x = np.random.Generator(np.random.PCG64(73)).uniform(-1, 1, size=(20000, 3)).astype(np.float32)
    say(f"case: FINER 4x64 plain model, dynamic r = {r}, {prec}")
    y, d = run(model, None, x, precision=prec, mode="dynamic", dynamic_r=r)
    t = DY.tails(ref, x.astype(np.float64))
    d_ref = DY.exit_from_tails(t, r, 0)
    upto = np.arange(1, 5)[None, :] <= np.maximum(d_ref, d)[:, None]
    amb = ((np.abs(np.abs(t) - r) < 1e-5) & upto & (np.arange(1, 5)[None, :] >= 2)).any(axis=1)
    diff = d != d_ref
    say(f"  exits {np.bincount(d, minlength=5)[1:].tolist()}, {int(diff.sum())} differ "
        f"({int((diff & amb).sum())} ambiguous)")
    assert len(set(d.tolist())) >= 3
    tol = TOL[prec] if prec == "fp32" else 1.5e-2   # plain (unit-scale) tails in BF16
    assert_close(y, oracle.forward(ref, x, d), tol, f"FINER dynamic {prec}")
    if prec == "fp32":
        assert not (diff & ~amb).any()
    else:
        assert 1.0 - diff.mean() >= 0.9


def test_finer_server_mix(c2f):
    """SIREN and FINER models of the same width in one serving loop: a batch
    holds one activation, and each request's result equals the same query
    alone, bit for bit."""
    blob, ref, model, dmap, dm = c2f
    sblob = c2_blob(256, seed=1001)
    smodel = sand.load_model(sblob, 0)
    sdm = sand.build_depthmap(smodel, dmap)
    pairs = [(model, dm), (smodel, sdm)]
    sizes = [1, 77, 4097, 30000, 5, 123457, 999, 64000, 2, 4096]
    srv = sand.Server(0, budget_bytes=1 << 30, precision="bf16", n_streams=3)
    reqs = []
    for i, n in enumerate(sizes):
        m, mdm = pairs[i % 2]
        x = synth.slab_points(512, n, 300 + i)
        y = np.full(n, np.nan, dtype=np.float32)
        reqs.append((m, mdm, x, y, srv.submit(m, mdm, x, y)))
    for (_, _, _, _, t) in reqs:
        srv.wait(t)
    info = srv.stats()
    say(f"  {len(sizes)} requests alternating FINER/SIREN: batches={info['batches']}")
    for (m, mdm, x, y, _) in reqs:
        want = sand.query(m, mdm, torch.from_numpy(x).to(DEV), precision="bf16").cpu().numpy()
        assert np.array_equal(y, want), f"request of {len(x)} points differs from alone"
    # request 2 went to the FINER model, request 3 to the SIREN one
    for i, r_ in ((2, ref), (3, oracle.parse_blob(sblob))):
        x, y = reqs[i][2], reqs[i][3]
        d = oracle.lookup_depth(x, dmap, 8)
        assert_close(y.astype(np.float64), oracle.forward(r_, x, d), TOL["bf16"],
                     f"served request {i} ({r_['activation']})")
    srv.close()


def test_finer_octree_small():
    """The octree built from a FINER network (intersection tests on y_L at
    node centres, Eq. 5-7 at level D) has the oracle's tree level by level,
    and lookups through it give the oracle's depths and values, with the
    ambiguity rule of the SIREN octree tests."""
    from test_gpu_octree import check_counts, compare, node_values
    D, s, r = 5, 2, 0.3
    blob = synth.write_blob(synth.siren_tmlp(67, 3, 10, tails="mult", scale="plain",
                                             activation="finer"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    say(f"case: FINER 3x10 model, octree D={D}, s={s}, r={r}, fp32")
    dm, info = sand.construct_octree(model, D=D, s=s, r=r)
    tree = OT.build(ref, D, s, r)
    ny = node_values(ref, tree)
    check_counts(tree, info, ny, 1e-5)
    x = np.random.Generator(np.random.PCG64(3)).uniform(-1, 1, size=(20000, 3)).astype(np.float32)
    y, d = run(model, dm, x, precision="fp32")
    # far leaves hold y_L(centre) from the FP32 build, whose FINER error (up to
    # ~7e-6 on this model) is the FP32 path's: their bound is the FP32 one
    compare(ref, tree, x.astype(np.float64), y, d, s, r, "fp32", 1e-5, "FINER tree", ny=ny,
            far_tol=TOL["fp32"])


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_finer_dynamic_compaction_is_exact(prec):
    """Compacted dynamic exit on the FINER 8x256 model (the resumed launch
    runs the FINER kernels too): every checkpoint gives the uncompacted
    run's bits and depths."""
    from test_gpu_dynamic import run_cp
    r = 1.5e-4
    model = sand.load_model(finer_blob(256), 0)
    x = synth.slab_points(512, 200000, 29)
    y0, d0 = run_cp(model, x, r, prec, -1)
    say(f"case: FINER 8x256, {prec}, {len(x)} points, exits "
        f"{np.bincount(d0, minlength=9)[1:].tolist()}")
    for cp in (2, 4, 5):
        y, d = run_cp(model, x, r, prec, cp)
        assert np.array_equal(d, d0)
        assert np.array_equal(y.view(np.uint32), y0.view(np.uint32))


@pytest.mark.parametrize("W,L", [(16, 2), (64, 4), (128, 3), (336, 3)])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_finer_gradient_widths(W, L, prec):
    """The FINER adjoint at every padded width (16 -> 64, 128, 336 -> 352),
    adaptive and full depth, against the oracle gradient."""
    say(f"case: FINER gradient W={W} L={L} {prec}")
    blob = synth.write_blob(synth.siren_tmlp(500 + W, L, W, tails="mult", activation="finer"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(W + 7 * L))
    dmap = rng.integers(1, L + 1, size=(8, 8, 8)).astype(np.uint8)
    dm = sand.build_depthmap(model, dmap)
    x = rng.uniform(-1, 1, size=(2500, 3)).astype(np.float32)
    xyz = torch.from_numpy(x).to(DEV)
    g = sand.query_grad(model, dm, xyz, precision=prec).cpu().numpy().astype(np.float64)
    check_grad(g, oracle.gradient(ref, x, oracle.lookup_depth(x, dmap, L)), prec,
               f"FINER W={W} L={L} {prec}")
    g = sand.query_grad(model, dm, xyz, precision=prec, mode="full").cpu().numpy()
    check_grad(g.astype(np.float64), oracle.gradient(ref, x, np.full(len(x), L)), prec,
               f"FINER W={W} L={L} {prec} full")
