"""Sparse network-depth octree (Sec. 3.2, Eq. 5-7) built on the GPU, against
the FP64 oracle (needs an MI355X).

The GPU decides the intersection tests on FP32 values, the oracle on FP64
ones, so a point is compared exactly unless a node on its path (root to
leaf) has |y_L(centre)| within EPS of half its diagonal, or one of its
leaf's samples has a required-depth decision within EPS of r or of zero.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.depthmap as OD
import oracle.octree as OT
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c2_blob

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def gpu_query(model, dm, x, prec="fp32"):
    xyz = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    depth = torch.full((len(x),), 255, dtype=torch.uint8, device=DEV)
    y = sand.query(model, dm, xyz, precision=prec, depth_out=depth)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), depth.cpu().numpy().astype(np.int64)


def ambiguous(ref, tree, x, level, s, r, eps):
    """Per point: some decision on its path is within eps of its boundary."""
    D = tree["D"]
    fine = oracle.voxel_index(x, 1 << D)
    amb = np.zeros(len(x), dtype=bool)
    for l in range(0, D + 1):
        ijk = fine >> (D - l)
        c = OT.centres(l, ijk)
        y = OT.y_last(ref, c)
        gap = np.abs(np.abs(y) - OT.SQRT3 * 2.0 ** (-l))
        amb |= (gap < eps) & (level >= l)
    # near leaves: the samples' required-depth decisions
    nearpt = np.nonzero(level == D)[0]
    if nearpt.size:
        R = 1 << D
        vox = (fine[nearpt, 0] * R + fine[nearpt, 1]) * R + fine[nearpt, 2]
        ya = oracle.forward_all_tails(ref, OD.sample_points(R, vox, s))
        g = np.abs(np.abs(ya[:, -1:] - ya) - r)
        z = np.minimum(np.abs(ya), np.abs(ya[:, -1:]))
        bad = ((g < eps) | (z < eps)).any(axis=1).reshape(nearpt.size, s ** 3).any(axis=1)
        amb[nearpt] |= bad
    return amb


def compare(ref, tree, x, y, d, s, r, prec, eps, what, max_diff=0.0):
    de, ve, lv = OT.lookup(tree, x)
    amb = ambiguous(ref, tree, x, lv, s, r, eps)
    far = de == 0
    yo = np.where(far, ve, 0.0)
    if (~far).any():
        yo[~far] = oracle.forward(ref, x[~far], de[~far])
    bad_d = d != de
    err = np.abs(y - yo)
    tol = np.where(far, 2e-6 * (1 + np.abs(yo)), TOL[prec])
    bad_v = (err > tol) & ~bad_d
    say(f"  {what}: n={len(x)}, far {int(far.sum())}, near {int((~far).sum())}, "
        f"leaf levels {np.bincount(lv, minlength=tree['D'] + 1).tolist()}, "
        f"{int(amb.sum())} ambiguous, {int(bad_d.sum())} depths differ, "
        f"max value error {err[~bad_d].max() if (~bad_d).any() else 0:.2e}")
    assert not (bad_d & ~amb).any(), f"{int((bad_d & ~amb).sum())} unambiguous depths differ"
    assert not (bad_v & ~amb).any(), f"{int((bad_v & ~amb).sum())} unambiguous values differ"
    assert bad_d.mean() <= max_diff + 1e-12 or bad_d.mean() <= amb.mean()


def test_small_model_tree():
    D, s, r = 5, 2, 0.3
    say(f"case: 3x10 plain-init model, octree D={D}, s={s}, r={r}, fp32")
    blob = synth.write_blob(synth.siren_tmlp(67, 3, 10, tails="mult", scale="plain"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dm, info = sand.construct_octree(model, D=D, s=s, r=r)
    tree = OT.build(ref, D, s, r)
    say(f"  gpu: internal {info['internal_nodes']}, leaves {info['leaves']}, "
        f"near {info['near_leaves']}, {info['bytes']} bytes")
    exp_int = [len(tree["internal"][l]) for l in range(D)]
    exp_leaves = [sum(1 for k in tree["leaves"] if k[0] == l) for l in range(D + 1)]
    say(f"  oracle: internal {exp_int}, leaves {exp_leaves}")
    assert sum(n * 8 ** (D - l) for l, n in enumerate(info["leaves"])) == 8 ** D
    assert sum(info["depth_counts"]) == sum(info["leaves"])
    rng = np.random.Generator(np.random.PCG64(3))
    c = synth.voxel_centres(1 << D)
    cells = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(-1, 3)
    x = np.concatenate([rng.uniform(-1, 1, size=(20000, 3)), cells,
                        np.repeat(np.array([[1.0], [-1.0], [0.0], [1.5], [-3.0]]), 3, axis=1)]
                       ).astype(np.float32)
    y, d = gpu_query(model, dm, x)
    compare(ref, tree, x.astype(np.float64), y, d, s, r, "fp32", 1e-5, "mixed points")


def test_c2_model_tree():
    D, s, r = 6, 1, 1.5e-4
    say(f"case: 8x256 residual model, octree D={D}, s={s}, r={r}, fp32")
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dm, info = sand.construct_octree(model, D=D, s=s, r=r)
    say(f"  gpu: internal {info['internal_nodes']}, leaves {info['leaves']}, "
        f"near {info['near_leaves']}, depths {info['depth_counts'][:9]}")
    tree = OT.build(ref, D, s, r)
    x = np.random.Generator(np.random.PCG64(4)).uniform(-1, 1, size=(6000, 3))
    x = x.astype(np.float32)
    y, d = gpu_query(model, dm, x)
    compare(ref, tree, x.astype(np.float64), y, d, s, r, "fp32", 4e-6, "uniform points")
    yb, db = gpu_query(model, dm, x, "bf16")
    assert np.array_equal(db, d), "the map, not the precision, sets the depth"
    assert np.abs(yb - y).max() <= 2 * TOL["bf16"]


def test_tree_lod_clamp_and_gradient():
    """Through a tree, a max_depth clamp and a gradient query: the points
    below the tree's dense index are resolved in a second pass, which must
    clamp their depth and give far points a zero gradient like the first."""
    D, s, r = 5, 2, 0.3
    say(f"case: 3x10 plain-init model, octree D={D}, LOD clamp 2 and gradient, fp32")
    blob = synth.write_blob(synth.siren_tmlp(67, 3, 10, tails="mult", scale="plain"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dm, _ = sand.construct_octree(model, D=D, s=s, r=r)
    rng = np.random.Generator(np.random.PCG64(5))
    x = rng.uniform(-1, 1, size=(30000, 3)).astype(np.float32)
    xyz = torch.from_numpy(x).to(DEV)
    y, d = gpu_query(model, dm, x)
    dl = torch.full((len(x),), 255, dtype=torch.uint8, device=DEV)
    yl = sand.query(model, dm, xyz, precision="fp32", max_depth=2, depth_out=dl).cpu().numpy()
    dl = dl.cpu().numpy().astype(np.int64)
    say(f"  depths {np.bincount(d, minlength=4).tolist()} -> clamped {np.bincount(dl, minlength=4).tolist()}")
    assert (d > 2).any() and (d == 0).any()
    assert np.array_equal(dl, np.minimum(d, 2))
    far = d == 0
    assert np.array_equal(yl[far], y[far].astype(np.float32))
    want = oracle.forward(ref, x[~far].astype(np.float64), dl[~far])
    assert np.abs(yl[~far] - want).max() <= TOL["fp32"]
    g = torch.empty((len(x), 3), dtype=torch.float32, device=DEV)
    sand.query_grad(model, dm, xyz, grad_out=g, precision="fp32")
    g = g.cpu().numpy().astype(np.float64)
    assert not g[far].any(), "far points must have a zero gradient"
    gw = oracle.gradient(ref, x[~far].astype(np.float64), d[~far])
    err = np.linalg.norm(g[~far] - gw, axis=1) / (np.linalg.norm(gw, axis=1) + 1.0)
    say(f"  gradient: {int((~far).sum())} near points, max rel err {err.max():.2e}")
    assert err.max() <= 1e-4


def constant_blob(c, L=3, W=16):
    p = synth.siren_tmlp(9, L, W, tails="mult", scale="plain")
    p["tails"] = [{"kind": 0, "a": np.zeros(W), "c": float(c)}] + [
        {"kind": 1, "a0": np.zeros(W), "c0": 0.0, "a1": np.zeros(W), "c1": 0.0}
        for _ in range(L - 1)]
    return synth.write_blob(p)


def test_closed_form_trees_and_server():
    x = np.random.Generator(np.random.PCG64(5)).uniform(-1, 1, size=(5000, 3)).astype(np.float32)
    say("case: constant 2.0 model: the root is one far leaf")
    m = sand.load_model(constant_blob(2.0), 0)
    dm, info = sand.construct_octree(m, D=4, s=1)
    assert info["leaves"][0] == 1 and info["near_leaves"] == 0
    y, d = gpu_query(m, dm, x)
    assert np.all(d == 0) and np.all(y == np.float32(2.0))
    say("case: constant 0 model: every level-D cell is a near leaf of depth 1")
    m = sand.load_model(constant_blob(0.0), 0)
    dm, info = sand.construct_octree(m, D=4, s=2)
    assert info["near_leaves"] == 8 ** 4 and info["depth_counts"][1] == 8 ** 4
    y, d = gpu_query(m, dm, x)
    assert np.all(d == 1) and np.all(y == 0.0)
    say("case: constant 0.3 model: far leaves at level 3 only (half diagonals 1.73, .87, .43, .22)")
    m = sand.load_model(constant_blob(0.3), 0)
    dm, info = sand.construct_octree(m, D=5, s=1)
    assert info["leaves"] == [0, 0, 0, 512, 0, 0] and info["depth_counts"][0] == 512
    y, d = gpu_query(m, dm, x)
    assert np.all(d == 0) and np.all(y == np.float32(0.3))
    say("case: the serving loop on an octree map gives the direct query's values")
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    dm, _ = sand.construct_octree(model, D=6, s=1, r=1.5e-4)
    want, _ = gpu_query(model, dm, x, "bf16")
    srv = sand.Server(0, budget_bytes=256 << 20, precision="bf16", n_streams=2)
    got = np.full(len(x), np.nan, dtype=np.float32)
    srv.wait(srv.submit(model, dm, x, got))
    srv.close()
    assert np.array_equal(got.astype(np.float64), want)
    with pytest.raises(sand.SandError):
        sand.construct_octree(model, D=11)
    with pytest.raises(sand.SandError):
        sand.construct_octree(model, D=4, s=3)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_shallow_trees(D):
    """Trees with no dense top index (D = 1) or a one- or two-level one."""
    s, r = 2, 0.3
    say(f"case: 3x10 plain-init model, octree D={D}, s={s}, r={r}, fp32")
    blob = synth.write_blob(synth.siren_tmlp(67, 3, 10, tails="mult", scale="plain"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dm, info = sand.construct_octree(model, D=D, s=s, r=r)
    tree = OT.build(ref, D, s, r)
    assert [len(tree["internal"][l]) for l in range(D)] == info["internal_nodes"][:D]
    x = np.random.Generator(np.random.PCG64(30 + D)).uniform(-1.05, 1.05, size=(9000, 3))
    x = x.astype(np.float32)
    y, d = gpu_query(model, dm, x)
    compare(ref, tree, x.astype(np.float64), y, d, s, r, "fp32", 1e-5, f"D={D}")
