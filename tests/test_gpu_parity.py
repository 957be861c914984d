"""GPU query path vs the FP64 oracle, element by element (needs an MI355X).

Exit depths must match bit for bit; SDF values within the absolute
tolerance of their precision (1e-5 FP32, 2e-3 BF16/FP16). Everything goes
through the C ABI via the ctypes binding.
"""

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c1_case, c2_blob, c2_map, c2_points, edge_points

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def run(model, dm, x, **kw):
    xyz = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    depth = torch.full((len(x),), 255, dtype=torch.uint8, device=DEV)
    y = sand.query(model, dm, xyz, depth_out=depth, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), depth.cpu().numpy().astype(np.int64)


def assert_close(got, want, tol, what):
    nan_g, nan_w = np.isnan(got), np.isnan(want)
    assert np.array_equal(nan_g, nan_w), f"{what}: NaN pattern differs"
    err = np.abs(got - want)[~nan_w]
    mx = float(err.max()) if err.size else 0.0
    say(f"  {what}: n={got.size} max|err|={mx:.3e} mean={float(err.mean()) if err.size else 0:.3e}")
    assert mx <= tol, f"{what}: max |err| {mx:.3e} > {tol:.1e}"


@pytest.fixture(scope="module")
def c1():
    blob, dmap, x = c1_case()
    model = sand.load_model(blob, 0)
    return blob, oracle.parse_blob(blob), model, sand.build_depthmap(model, dmap), dmap, x


def test_c1_all_points_fp32(c1):
    blob, ref, model, dm, dmap, x = c1
    say("case: C1 4x64, 32^3 map, all 64^3 points, fp32 adaptive")
    y, d = run(model, dm, x, precision="fp32")
    want_d = oracle.lookup_depth(x, dmap, 4)
    assert np.array_equal(d, want_d), "exit depths differ"
    assert_close(y, oracle.forward(ref, x, want_d), TOL["fp32"], "C1 fp32 adaptive")


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_c1_modes(c1, prec):
    blob, ref, model, dm, dmap, x = c1
    sub = x[::7]
    say(f"case: C1 modes, {sub.shape[0]} points, {prec}")
    tol = TOL[prec] if prec == "fp32" else 2e-2
    y, d = run(model, dm, sub, precision=prec, mode="full")
    assert np.all(d == 4)
    assert_close(y, oracle.forward(ref, sub, np.full(len(sub), 4)), tol, f"full {prec}")
    for m in (1, 2, 3):
        y, d = run(model, dm, sub, precision=prec, max_depth=m)
        want_d = oracle.lookup_depth(sub, dmap, 4, max_depth=m)
        assert np.array_equal(d, want_d)
        assert_close(y, oracle.forward(ref, sub, want_d), tol, f"lod {m} {prec}")
    rng = np.random.Generator(np.random.PCG64(5))
    forced = rng.integers(1, 5, size=len(sub)).astype(np.uint8)
    y, d = run(model, None, sub, precision=prec, mode="forced",
               forced_depth=torch.from_numpy(forced).to(DEV))
    assert np.array_equal(d, forced)
    assert_close(y, oracle.forward(ref, sub, forced), tol, f"forced {prec}")


def test_far_field_cells():
    say("case: depth-0 cells with stored far values, 3x32 model, R=8")
    blob = synth.write_blob(synth.siren_tmlp(4, 3, 32, tails="mult"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(11))
    dmap = rng.integers(0, 4, size=(8, 8, 8)).astype(np.uint8)
    far = rng.normal(size=(8, 8, 8)).astype(np.float32)
    dm = sand.build_depthmap(model, dmap, far)
    x = synth.grid_points(32)
    y, d = run(model, dm, x)
    want_d = oracle.lookup_depth(x, dmap, 3)
    assert np.array_equal(d, want_d)
    want = oracle.forward(ref, x, want_d, far=far)
    zero = want_d == 0
    assert np.array_equal(y[zero], want[zero]), "far values must be copied exactly"
    assert_close(y, want, TOL["fp32"], "far-field map fp32")
    forced = np.zeros(len(x), dtype=np.uint8)
    y, _ = run(model, None, x, mode="forced", forced_depth=torch.from_numpy(forced).to(DEV))
    assert np.all(np.isnan(y)), "depth 0 without a map has no value"


def test_edge_points_cell_rule(c1):
    blob, ref, model, dm, dmap, _ = c1
    x = edge_points(32)
    say(f"case: {len(x)} edge points (faces, corners, outside, NaN), fp32")
    y, d = run(model, dm, x)
    want_d = oracle.lookup_depth(x, dmap, 4)
    assert np.array_equal(d, want_d), "cell rule differs on edge points"
    assert_close(y, oracle.forward(ref, x, want_d), TOL["fp32"], "edge points")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ragged_sizes(prec):
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    pts = c2_points(12000, seed=21)
    for n in (0, 1, 2, 31, 33, 127, 129, 255, 257, 4095, 4097, 12000):
        x = pts[:n]
        say(f"case: ragged n={n} {prec}")
        if n == 0:
            out = sand.query(model, dm, torch.empty((0, 3), device=DEV), precision=prec)
            assert out.numel() == 0
            continue
        y, d = run(model, dm, x, precision=prec)
        want_d = oracle.lookup_depth(x, dmap, 8)
        assert np.array_equal(d, want_d)
        assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"n={n} {prec}")


@pytest.mark.parametrize("W", [16, 64, 100, 128, 200, 256, 336, 352])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_widths_and_padding(W, prec):
    say(f"case: width {W} (padded), 4 layers, {prec}")
    blob = synth.write_blob(synth.siren_tmlp(50 + W, 4, W, tails="mult"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(W))
    dmap = rng.integers(1, 5, size=(16, 16, 16)).astype(np.uint8)
    dm = sand.build_depthmap(model, dmap)
    x = rng.uniform(-1, 1, size=(3000, 3)).astype(np.float32)
    y, d = run(model, dm, x, precision=prec)
    want_d = oracle.lookup_depth(x, dmap, 4)
    assert np.array_equal(d, want_d)
    assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"W={W} {prec}")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_permutation_and_batch_invariance(prec):
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, c2_map())
    x = c2_points(20000, seed=33)
    say(f"case: permutation / batch invariance, 20000 points, {prec}")
    y, _ = run(model, dm, x, precision=prec)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(x))
    yp, _ = run(model, dm, x[perm], precision=prec)
    assert np.array_equal(yp, y[perm]), "result depends on point order"
    ys, _ = run(model, dm, x[:777], precision=prec)
    assert np.array_equal(ys, y[:777]), "result depends on batch composition"


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_c2_model_medium(prec):
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    x = c2_points(65536, seed=41)
    say(f"case: 8x256 residual tails, 128^3 map, 65536 points, {prec} adaptive")
    y, d = run(model, dm, x, precision=prec)
    want_d = oracle.lookup_depth(x, dmap, 8)
    assert np.array_equal(d, want_d)
    assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"8x256 {prec} adaptive")
    xs = x[:8192]
    y, _ = run(model, dm, xs, precision=prec, mode="full")
    assert_close(y, oracle.forward(ref, xs, np.full(len(xs), 8)), TOL[prec], f"8x256 {prec} full")


def test_layer1_argument_at_fp32_accuracy():
    """Layer 1 of the BF16/FP16 paths (BF16 MFMAs over three-way splits of
    weights and coordinates) must be as accurate as the FP32 path's: at depth
    1 the output is the FP32 first tail of sin of the omega-scaled argument,
    so any loss in that argument shows directly. Points inside the cube and
    out to 8 units from its centre (larger arguments); a plain BF16 or a
    two-way split would miss by 1e-4 and more."""
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(57))
    x = np.concatenate([rng.uniform(-1, 1, size=(49152, 3)),
                        rng.uniform(-8, 8, size=(16384, 3))]).astype(np.float32)
    forced = torch.ones(len(x), dtype=torch.uint8, device=DEV)
    want = oracle.forward(ref, x, np.ones(len(x), dtype=np.int64))
    err = {}
    for prec in ("fp32", "bf16", "fp16"):
        y, _ = run(model, None, x, precision=prec, mode="forced", forced_depth=forced)
        err[prec] = float(np.abs(y - want).max())
        say(f"  depth 1, {prec}: max|err| {err[prec]:.3e}")
    for prec in ("bf16", "fp16"):
        assert err[prec] <= 2.0 * err["fp32"] + 1e-6, (prec, err)


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fp32"])
def test_c3_width336_medium(prec):
    blob = c2_blob(336, seed=1336)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    x = c2_points(32768, seed=43)
    say(f"case: 8x336 residual tails, 32768 points, {prec} adaptive")
    y, d = run(model, dm, x, precision=prec)
    want_d = oracle.lookup_depth(x, dmap, 8)
    assert np.array_equal(d, want_d)
    assert_close(y, oracle.forward(ref, x, want_d), TOL[prec], f"8x336 {prec}")


def test_workspace_and_errors(c1):
    blob, ref, model, dm, dmap, x = c1
    xyz = torch.from_numpy(x[:5000]).to(DEV)
    ws = torch.empty(sand.query_workspace_size(5000), dtype=torch.uint8, device=DEV)
    a = sand.query(model, dm, xyz, workspace=ws)
    b = sand.query(model, dm, xyz)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    small = torch.empty(100, dtype=torch.uint8, device=DEV)
    with pytest.raises(sand.SandError) as e:
        sand.query(model, dm, xyz, workspace=small)
    assert e.value.status == 1
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz)
    other = sand.load_model(blob, 0)
    with pytest.raises(sand.SandError):
        sand.query(other, dm, xyz)
    with pytest.raises(sand.SandError):
        sand.build_depthmap(model, np.full((8, 8, 8), 9, dtype=np.uint8))
    with pytest.raises(sand.SandError):
        sand.build_depthmap(model, np.zeros((8, 8, 8), dtype=np.uint8))
    with pytest.raises(sand.SandError):
        sand.build_depthmap(model, np.ones((6, 6, 6), dtype=np.uint8))


def test_512_grid_bench_configuration():
    """The benchmarked workload at full size: 8x256 model, 128^3 map, all
    134,217,728 cells of the 512^3 grid. Exit depths are compared on every
    point; SDF values on a seeded sample, per precision."""
    G = 512
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    xyz = synth.queries.grid_points_torch(G, DEV)
    n = xyz.shape[0]
    depth = torch.empty(n, dtype=torch.uint8, device=DEV)
    sdf = torch.empty(n, dtype=torch.float32, device=DEV)
    idx = synth.sample_indices(n, 20000, seed=99)
    xs = synth.grid_points_at(G, idx)
    ds = oracle.lookup_depth(xs, dmap, 8)
    for prec in ("bf16", "fp32"):
        say(f"case: 512^3 grid, 8x256, {prec} adaptive (bench launch)")
        sand.query(model, dm, xyz, out=sdf, precision=prec, depth_out=depth)
        torch.cuda.synchronize()
        if prec == "bf16":
            dev_depth = depth.cpu().numpy()
            step = 1 << 23
            for s in range(0, n, step):
                pts = synth.grid_points_at(G, np.arange(s, min(n, s + step), dtype=np.int64))
                want = oracle.lookup_depth(pts, dmap, 8)
                assert np.array_equal(dev_depth[s:s + step], want), f"depth differs in chunk {s}"
            say("  all 134,217,728 exit depths bit-exact")
        got = sdf[torch.from_numpy(idx).to(DEV)].cpu().numpy().astype(np.float64)
        assert_close(got, oracle.forward(ref, xs, ds), TOL[prec], f"512^3 {prec} sample")
    say("case: 512^3 grid, fp32 full depth (plain network)")
    sand.query(model, dm, xyz, out=sdf, precision="fp32", mode="full")
    torch.cuda.synchronize()
    got = sdf[torch.from_numpy(idx[:4000]).to(DEV)].cpu().numpy().astype(np.float64)
    assert_close(got, oracle.forward(ref, xs[:4000], np.full(4000, 8)), TOL["fp32"],
                 "512^3 fp32 full sample")


def test_free_model_before_map():
    """A map may be freed after its model (finalizers of unreachable objects
    run in any order); nothing may leave a device error behind."""
    blob = synth.write_blob(synth.siren_tmlp(3, 2, 32))
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, np.ones((4, 4, 4), dtype=np.uint8))
    model.free()
    dm.free()
    t = torch.full((1000,), 7, dtype=torch.uint8, device=DEV)
    torch.cuda.synchronize()
    assert int(t.sum().item()) == 7000


@pytest.mark.parametrize("kind", ["dense", "octree"])
def test_unaligned_buffers(kind):
    """Points, results and depths at odd offsets (the 4-points-per-thread
    lookup and scatter then take their element-wise paths) give the same bits
    as aligned buffers; sizes not a multiple of 4."""
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    if kind == "dense":
        dm = sand.build_depthmap(model, c2_map())
    else:
        dm, _ = sand.construct_octree(model, D=6, s=1, r=1.5e-4)
    pts = c2_points(20001, seed=41)
    n = len(pts)
    say(f"case: unaligned buffers, {kind} map, n={n}")
    base = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    y_ref = torch.empty(n, device=DEV)
    d_ref = torch.empty(n, dtype=torch.uint8, device=DEV)
    sand.query(model, dm, base, out=y_ref, precision="bf16", depth_out=d_ref)
    xbuf = torch.empty((n + 1, 3), device=DEV)
    xbuf[1:] = base
    ybuf = torch.empty(n + 1, device=DEV)
    dbuf = torch.empty(n + 3, dtype=torch.uint8, device=DEV)
    xs, ys, ds = xbuf[1:], ybuf[1:], dbuf[3:]
    assert xs.data_ptr() % 16 != 0 and ys.data_ptr() % 16 != 0 and ds.data_ptr() % 4 != 0
    sand.query(model, dm, xs, out=ys, precision="bf16", depth_out=ds)
    torch.cuda.synchronize()
    assert torch.equal(ds, d_ref)
    assert torch.equal(ys.view(torch.int32), y_ref.view(torch.int32))
