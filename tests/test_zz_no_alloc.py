"""sand_query_noalloc (the entry point for callers that cannot allocate)
against sand_query through the C ABI (needs an MI355X): two calls in a row,
the second with a smaller input, must give sand_query's results bit for bit,
on a dense map (adaptive BF16), through an octree (adaptive FP32) and in
forced and full modes; sizes beyond the scratch limit and allocating modes
are rejected before any device work."""

import ctypes

import numpy as np
import pytest
import torch

import synth
import paper_2604_25936_amd as sand
from gpu_cases import c2_blob, c2_map, c2_points

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
MAX_POINTS = 13_373_120


def say(msg):
    print(msg, flush=True)


def both(model, dm, x, **kw):
    """(sand_query, sand_query_noalloc) results and exit depths for one input."""
    xyz = x if isinstance(x, torch.Tensor) else torch.from_numpy(
        np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    n = xyz.shape[0]
    d1 = torch.full((n,), 255, dtype=torch.uint8, device=DEV)
    d2 = torch.full((n,), 254, dtype=torch.uint8, device=DEV)
    y1 = torch.full((n,), float("nan"), device=DEV)
    y2 = torch.full((n,), -7.0, device=DEV)
    sand.query(model, dm, xyz, out=y1, depth_out=d1, **kw)
    sand.query_noalloc(model, dm, xyz, out=y2, depth_out=d2, **kw)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), y2.cpu().numpy(), d1.cpu().numpy(), d2.cpu().numpy()


def same(r, what):
    y1, y2, d1, d2 = r
    say(f"  {what}: n={y1.size}, {int((y1.view(np.uint32) != y2.view(np.uint32)).sum())} values "
        f"and {int((d1 != d2).sum())} depths differ")
    assert np.array_equal(d1, d2), f"{what}: exit depths differ"
    assert np.array_equal(y1.view(np.uint32), y2.view(np.uint32)), f"{what}: values differ"


def test_noalloc_equals_query_dense_map():
    model = sand.load_model(c2_blob(256), 0)
    dm = sand.build_depthmap(model, c2_map())
    big = c2_points(300_000, seed=61)
    say("case: noalloc vs sand_query, 8x256, dense map, bf16 adaptive, 300000 then 4097 points")
    same(both(model, dm, big, precision="bf16"), "call 1 (300000)")
    same(both(model, dm, big[:4097], precision="bf16"), "call 2 (4097)")
    say("case: forced fp32 and full fp16, 50000 then 33 points")
    forced = torch.randint(0, 9, (50_000,), dtype=torch.uint8, device=DEV,
                           generator=torch.Generator(device=DEV).manual_seed(3))
    far = np.random.Generator(np.random.PCG64(2)).uniform(-1, 1, (128,) * 3).astype(np.float32)
    dmf = sand.build_depthmap(model, c2_map(), far)
    same(both(model, dmf, big[:50_000], precision="fp32", mode="forced", forced_depth=forced),
         "forced fp32 (50000)")
    same(both(model, dmf, big[:33], precision="fp32", mode="forced", forced_depth=forced[:33]),
         "forced fp32 (33)")
    same(both(model, None, big[:50_000], precision="fp16", mode="full"), "full fp16 (50000)")
    same(both(model, None, big[:33], precision="fp16", mode="full"), "full fp16 (33)")


def test_noalloc_equals_query_octree_and_finer():
    model = sand.load_model(c2_blob(256), 0)
    tree, _ = sand.construct_octree(model, D=8, s=1, r=1.5e-4)
    x = synth.slab_points(512, 200_000, 62)
    say("case: noalloc vs sand_query through a D = 8 octree, fp32, 200000 then 1000 points")
    same(both(model, tree, x, precision="fp32"), "octree call 1")
    same(both(model, tree, x[:1000], precision="fp32"), "octree call 2")
    from gpu_cases import finer_blob
    fm = sand.load_model(finer_blob(256), 0)
    fdm = sand.build_depthmap(fm, c2_map())
    say("case: FINER model, bf16 adaptive, 100000 then 77 points")
    same(both(fm, fdm, x[:100_000], precision="bf16"), "FINER call 1")
    same(both(fm, fdm, x[:77], precision="bf16"), "FINER call 2")
    say("case: dynamic exit without compaction, fp32, 20000 then 500 points")
    same(both(model, None, x[:20_000], precision="fp32", mode="dynamic", dynamic_r=1.5e-4,
              dynamic_checkpoint=-1), "dynamic call 1")
    same(both(model, None, x[:500], precision="fp32", mode="dynamic", dynamic_r=1.5e-4,
              dynamic_checkpoint=-1), "dynamic call 2")


def test_noalloc_limits_and_errors():
    model = sand.load_model(c2_blob(256), 0)
    dm = sand.build_depthmap(model, c2_map())
    lib = sand.library()
    o = sand.sand.QueryOpts()
    lib.sand_query_opts_init(ctypes.byref(o))
    # one point beyond the scratch: rejected before any pointer is touched
    st = lib.sand_query_noalloc(model.handle, dm.handle, ctypes.c_void_p(256), MAX_POINTS + 1,
                                ctypes.c_void_p(256), ctypes.byref(o), None)
    assert st == sand.sand.ERR_INVALID and b"scratch" in lib.sand_last_error()
    assert sand.query_workspace_size(MAX_POINTS) <= 64 << 20 < sand.query_workspace_size(MAX_POINTS + 1)
    x = torch.zeros((8, 3), device=DEV)
    with pytest.raises(sand.SandError):     # compaction would allocate its arena
        sand.query_noalloc(model, None, x, mode="dynamic", dynamic_r=1e-3, dynamic_checkpoint=0)
    with pytest.raises(sand.SandError):
        sand.query_noalloc(model, dm, x, workspace=torch.empty(1 << 20, dtype=torch.uint8,
                                                               device=DEV))
    y = sand.query_noalloc(model, dm, torch.empty((0, 3), device=DEV))
    assert y.numel() == 0
