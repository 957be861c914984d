"""Network-depth map construction on the GPU (Sec. 3.2, Eq. 5-7) against
the FP64 oracle (needs an MI355X).

The GPU decides Eq. 5 on FP32 outputs, the oracle on FP64 ones, so a
voxel is compared exactly unless one of its samples has a decision within
EPS of the threshold r or of a sign change (on the oracle's values, for
the layers up to its required depth); such voxels are counted, and those
that differ must be rare.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.depthmap as OD
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c2_blob

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = 4e-6      # FP32 outputs of these models are within ~1.2e-6 of FP64, so a
                # difference of two of them within ~2.4e-6


def say(msg):
    print(msg, flush=True)


def ambiguous_voxels(model, R, voxels, s, r):
    """Oracle depths of `voxels` and a flag per voxel: some sample decision
    lies within EPS of r or of zero."""
    y = oracle.forward_all_tails(model, OD.sample_points(R, voxels, s))
    d = OD.required_depth(y, r)
    L = y.shape[1]
    gap = np.abs(np.abs(y[:, -1:] - y) - r)
    near_zero = np.minimum(np.abs(y), np.abs(y[:, -1:]))
    upto = np.arange(1, L + 1)[None, :] <= d[:, None]
    amb = (((gap < EPS) | (near_zero < EPS)) & upto).any(axis=1)
    nv = len(voxels)
    return d.reshape(nv, s ** 3).max(axis=1), amb.reshape(nv, s ** 3).any(axis=1)


def compare(gpu_depth, model, R, voxels, s, r, what, max_diff_frac=0.01):
    exp, amb = ambiguous_voxels(model, R, voxels, s, r)
    got = gpu_depth.reshape(-1)[voxels].astype(np.int64)
    diff = got != exp
    bad = diff & ~amb
    say(f"  {what}: {len(voxels)} near voxels compared, {int(amb.sum())} ambiguous, "
        f"{int(diff.sum())} differ, depths "
        f"{np.bincount(exp, minlength=model['L'] + 1)[1:].tolist()}")
    assert not bad.any(), f"{int(bad.sum())} unambiguous voxels differ, e.g. voxel " \
                          f"{voxels[np.argmax(bad)]}: {got[bad][0]} vs {exp[bad][0]}"
    assert diff.mean() <= max_diff_frac


def test_small_model_whole_map():
    R, s, r = 16, 2, 0.05
    say(f"case: 4x64 plain-init model, R={R}, s={s}, r={r}, sphere shell, fp32")
    blob = synth.write_blob(synth.siren_tmlp(61, 4, 64, tails="mult", scale="plain"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    near = synth.near_surface_mask(synth.sphere_sdf, R)
    csdf = synth.far_value_grid(synth.sphere_sdf, R)
    dm, depth, info = sand.construct_depthmap(model, near, csdf, s=s, r=r, precision="fp32")
    nv = int(near.sum())
    assert info["near_voxels"] == nv and info["samples"] == nv * s ** 3
    assert sum(info["depth_counts"]) == R ** 3
    assert info["depth_counts"][0] == R ** 3 - nv
    assert np.all(depth[near == 0] == 0)
    assert np.all((depth[near == 1] >= 1) & (depth[near == 1] <= 4))
    assert np.bincount(depth[near == 1], minlength=5)[1:].tolist() == info["depth_counts"][1:5]
    compare(depth, ref, R, np.nonzero(near.reshape(-1))[0], s, r, "whole map")

    # the map answers queries: far voxels give their centre value (Eq. 7),
    # near voxels the network at the stored depth
    c = synth.voxel_centres(R)
    pts = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(-1, 3).astype(np.float32)
    y = sand.query(model, dm, torch.from_numpy(pts).to(DEV), precision="fp32").cpu().numpy()
    far = near.reshape(-1) == 0
    assert np.array_equal(y[far], csdf.reshape(-1)[far]), "far voxels must return the centre SDF"
    d = depth.reshape(-1).astype(np.int64)
    yo = oracle.forward(ref, pts[~far], d[~far])
    assert np.abs(y[~far] - yo).max() <= TOL["fp32"]


def test_c2_model_sampled_voxels():
    R, s, r, L = 128, 4, 1.5e-4, 8
    say(f"case: 8x256 residual model, analytic scene, R={R}, s={s}, r={r}, fp32")
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    prims = synth.random_primitives(2000)
    near = synth.near_surface_mask(prims.sdf, R)
    csdf = synth.far_value_grid(prims.sdf, R)
    dm, depth, info = sand.construct_depthmap(model, near, csdf, s=s, r=r, precision="fp32")
    say(f"  near voxels {info['near_voxels']}, samples {info['samples']}, "
        f"depth counts {info['depth_counts'][:L + 1]}")
    assert info["samples"] == int(near.sum()) * s ** 3
    assert np.all(depth[near == 0] == 0)
    assert np.all((depth[near == 1] >= 1) & (depth[near == 1] <= L))
    idx = np.nonzero(near.reshape(-1))[0]
    rng = np.random.Generator(np.random.PCG64(4))
    pick = np.sort(rng.choice(idx, size=1500, replace=False))
    compare(depth, ref, R, pick, s, r, "sampled voxels")
    # r large: shallower maps, never deeper
    _, shallow, _ = sand.construct_depthmap(model, near, csdf, s=s, r=1e-2, precision="fp32")
    assert np.all(shallow <= depth) and shallow[near == 1].mean() < depth[near == 1].mean()
    compare(shallow, ref, R, pick, s, 1e-2, "r = 1e-2")


def test_precisions_and_edge_masks():
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    R = 32
    prims = synth.random_primitives(2000)
    near = synth.near_surface_mask(prims.sdf, R)
    csdf = synth.far_value_grid(prims.sdf, R)
    for prec in ("bf16", "fp16"):
        say(f"case: construct at {prec}, R={R}")
        _, depth, info = sand.construct_depthmap(model, near, csdf, s=2, r=1e-2, precision=prec)
        assert np.all(depth[near == 0] == 0)
        assert np.all((depth[near == 1] >= 1) & (depth[near == 1] <= 8))
    say("case: empty mask (every voxel far)")
    dm, depth, info = sand.construct_depthmap(model, np.zeros((8, 8, 8), np.uint8),
                                              np.full((8, 8, 8), 0.25, np.float32), s=4)
    assert info["samples"] == 0 and not depth.any()
    y = sand.query(model, dm, torch.zeros(10, 3, device=DEV)).cpu().numpy()
    assert np.all(y == np.float32(0.25))
    say("case: full mask, R=4, s=1")
    _, depth, info = sand.construct_depthmap(model, np.ones((4, 4, 4), np.uint8),
                                             np.zeros((4, 4, 4), np.float32), s=1, r=1e-2)
    assert info["samples"] == 64 and np.all(depth >= 1)
    ref = oracle.parse_blob(blob)
    compare(depth, ref, 4, np.arange(64), 1, 1e-2, "full mask", 0.05)
    with pytest.raises(sand.SandError):
        sand.construct_depthmap(model, np.ones((4, 4, 4), np.uint8),
                                np.zeros((4, 4, 4), np.float32), s=3)
    with pytest.raises(sand.SandError):
        sand.construct_depthmap(model, np.ones((4, 4, 4), np.uint8),
                                np.zeros((4, 4, 4), np.float32), r=0.0)
    with pytest.raises(sand.SandError):
        sand.construct_depthmap(model, np.ones((6, 6, 6), np.uint8),
                                np.zeros((6, 6, 6), np.float32))
