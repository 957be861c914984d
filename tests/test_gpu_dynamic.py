"""Map-free dynamic early exit (Sec. 4.4 ablation) against the FP64 oracle
(needs an MI355X).

The GPU tests |t_j| < r on FP32 tails, the oracle on FP64 ones: exit depths
must agree except where some tested tail lies within EPS of r; values must
match the oracle's y at the GPU's own exit depth within the precision's
tolerance.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.dynamic as DY
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c2_blob

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def run(model, x, r, prec, max_depth=0):
    xyz = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    depth = torch.full((len(x),), 255, dtype=torch.uint8, device=DEV)
    y = sand.query(model, None, xyz, precision=prec, mode="dynamic", dynamic_r=r,
                   max_depth=max_depth, depth_out=depth)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), depth.cpu().numpy().astype(np.int64)


def check(ref, x, r, y, d, prec, eps, what, max_depth=0, min_agree=1.0):
    t = DY.tails(ref, x.astype(np.float64))
    d_ref = DY.exit_from_tails(t, r, max_depth)
    L = t.shape[1]
    upto = np.arange(1, L + 1)[None, :] <= np.maximum(d_ref, d)[:, None]
    tested = np.arange(1, L + 1)[None, :] >= 2
    amb = ((np.abs(np.abs(t) - r) < eps) & upto & tested).any(axis=1)
    diff = d != d_ref
    err = np.abs(y - oracle.forward(ref, x, d)).max() if len(x) else 0.0
    say(f"  {what}: n={len(x)} exits {np.bincount(d, minlength=L + 1)[1:].tolist()}, "
        f"{int(diff.sum())} differ from the oracle ({int((diff & amb).sum())} ambiguous), "
        f"max|y - y_oracle(d_gpu)| = {err:.3e}")
    assert np.all((d >= 1) & (d <= L))
    if max_depth:
        assert d.max() <= max_depth
    assert err <= TOL[prec], f"{what}: value error {err:.3e}"
    if min_agree >= 1.0:
        assert not (diff & ~amb).any(), f"{what}: {int((diff & ~amb).sum())} unambiguous exits differ"
    else:
        assert 1.0 - diff.mean() >= min_agree, f"{what}: exit agreement {1 - diff.mean():.4f}"


def test_small_model_fp32():
    say("case: 4x64 plain-init model, dynamic r = 0.05, fp32")
    blob = synth.write_blob(synth.siren_tmlp(71, 4, 64, tails="mult", scale="plain"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    x = np.random.Generator(np.random.PCG64(71)).uniform(-1, 1, size=(20000, 3)).astype(np.float32)
    y, d = run(model, x, 0.05, "fp32")
    check(ref, x, 0.05, y, d, "fp32", 1e-5, "r=0.05")
    assert len(set(d.tolist())) >= 3, "the case should exercise several exits"
    y, d = run(model, x, 0.05, "fp32", max_depth=3)
    check(ref, x, 0.05, y, d, "fp32", 1e-5, "r=0.05, max_depth 3", max_depth=3)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c2_model(prec):
    r = 1.5e-4
    say(f"case: 8x256 residual model, dynamic r = {r}, {prec}")
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    x = synth.slab_points(512, 40000, 11)
    y, d = run(model, x, r, prec)
    if prec == "fp32":
        check(ref, x, r, y, d, prec, 4e-6, "512^3 slab")
    else:
        # BF16 tails carry ~1e-4 error: compare values at the GPU's depths,
        # and require most exits to agree
        check(ref, x, r, y, d, prec, 0.0, "512^3 slab", min_agree=0.9)


def test_ragged_and_errors():
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    ref = oracle.parse_blob(blob)
    rng = np.random.Generator(np.random.PCG64(5))
    for n in (1, 33, 257, 4097):
        say(f"case: dynamic, ragged n={n}")
        x = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        y, d = run(model, x, 1e-2, "fp32")
        check(ref, x, 1e-2, y, d, "fp32", 4e-6, f"n={n}")
    xyz = torch.zeros((4, 3), device=DEV)
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz, mode="dynamic", dynamic_r=0.0)
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz, mode="full", dynamic_r=1e-3)
    with pytest.raises(sand.SandError) as e:
        sand.query_grad(model, None, xyz, mode="dynamic")
    assert e.value.status in (sand.sand.ERR_INVALID, sand.sand.ERR_UNSUPPORTED)


def run_cp(model, x, r, prec, cp, max_depth=0):
    xyz = x if isinstance(x, torch.Tensor) else torch.from_numpy(
        np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    depth = torch.full((xyz.shape[0],), 255, dtype=torch.uint8, device=DEV)
    y = sand.query(model, None, xyz, precision=prec, mode="dynamic", dynamic_r=r,
                   max_depth=max_depth, depth_out=depth, dynamic_checkpoint=cp)
    torch.cuda.synchronize()
    return y.cpu().numpy(), depth.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_compaction_is_exact(prec):
    """Compaction only regroups points: every checkpoint gives the same bits
    and depths as the uncompacted run (and the FP32 run matches the oracle)."""
    r = 1.5e-4
    blob = c2_blob(256)
    model = sand.load_model(blob, 0)
    x = synth.slab_points(512, 300000, 21)
    y0, d0 = run_cp(model, x, r, prec, -1)
    say(f"case: 8x256, {prec}, {len(x)} points, exits {np.bincount(d0, minlength=9)[1:].tolist()}")
    for cp in (2, 3, 4, 5, 7):
        y, d = run_cp(model, x, r, prec, cp)
        say(f"  checkpoint {cp}: {int((y != y0).sum())} values and {int((d != d0).sum())} depths differ")
        assert np.array_equal(d, d0)
        assert np.array_equal(y.view(np.uint32), y0.view(np.uint32))
    y, d = run_cp(model, x, r, prec, 4, max_depth=6)
    y6, d6 = run_cp(model, x, r, prec, -1, max_depth=6)
    assert np.array_equal(d, d6) and np.array_equal(y.view(np.uint32), y6.view(np.uint32))
    if prec == "fp32":
        ref = oracle.parse_blob(blob)
        pick = np.random.Generator(np.random.PCG64(22)).choice(len(x), 20000, replace=False)
        y, d = run_cp(model, x, r, prec, 5)
        check(ref, x[pick], r, y[pick].astype(np.float64), d[pick].astype(np.int64), prec, 4e-6,
              "compacted at 5, sample")


def test_compaction_slabs_ragged_and_auto():
    r = 1.5e-4
    model = sand.load_model(c2_blob(256), 0)
    rng = np.random.Generator(np.random.PCG64(23))
    for n in (1, 33, 257, 4097):
        x = rng.uniform(-1, 1, size=(n, 3)).astype(np.float32)
        y0, d0 = run_cp(model, x, 1e-2, "fp32", -1)
        y, d = run_cp(model, x, 1e-2, "fp32", 3)
        say(f"case: compaction at 3, ragged n={n}")
        assert np.array_equal(d, d0) and np.array_equal(y.view(np.uint32), y0.view(np.uint32))
    # FP32 records are 1040 B: 2.2M points need two slabs of the 2 GiB arena
    n = 2_200_000
    say(f"case: compaction at 5, fp32, n={n} (two slabs)")
    xyz = (torch.rand((n, 3), generator=torch.Generator().manual_seed(24)) * 2 - 1).to(DEV)
    y0, d0 = run_cp(model, xyz, r, "fp32", -1)
    y, d = run_cp(model, xyz, r, "fp32", 5)
    assert np.array_equal(d, d0) and np.array_equal(y.view(np.uint32), y0.view(np.uint32))
    # n >= 2^22: the library samples the query and picks a checkpoint itself
    n = (1 << 22) + 1000
    say(f"case: automatic checkpoint, bf16, n={n}")
    xyz = synth.queries.grid_points_torch(256, DEV)[:n]
    y0, d0 = run_cp(model, xyz, r, "bf16", -1)
    y, d = run_cp(model, xyz, r, "bf16", 0)
    assert np.array_equal(d, d0) and np.array_equal(y.view(np.uint32), y0.view(np.uint32))
    xyz = torch.zeros((4, 3), device=DEV)
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz, mode="dynamic", dynamic_r=1e-3, dynamic_checkpoint=1)
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz, mode="dynamic", dynamic_r=1e-3, dynamic_checkpoint=-2)
    with pytest.raises(sand.SandError):
        sand.query(model, None, xyz, mode="full", dynamic_checkpoint=3)
