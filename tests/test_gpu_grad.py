"""Input-gradient (normal) adjoint kernel vs the FP64 oracle and central
differences (needs an MI355X). Exit depths are held fixed, as the oracle's
gradient and the finite differences do."""

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2604_25936_amd as sand
from paper_2604_25936_amd.autograd import sdf as sdf_fn
from gpu_cases import c1_case, c2_blob, c2_map

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# per point: |grad_gpu - grad_oracle| <= REL * |grad_oracle| + ABS
GTOL = {"fp32": (1e-4, 1e-4), "bf16": (3e-2, 1e-2), "fp16": (1e-2, 5e-3)}


def say(msg):
    print(msg, flush=True)


def run_grad(model, dm, x, prec, dy=None, **kw):
    xyz = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(DEV)
    sdf = torch.empty(len(x), dtype=torch.float32, device=DEV)
    dyt = None if dy is None else torch.from_numpy(np.asarray(dy, dtype=np.float32)).to(DEV)
    g = sand.query_grad(model, dm, xyz, dy=dyt, sdf_out=sdf, precision=prec, **kw)
    torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64), sdf.cpu().numpy().astype(np.float64)


def check_grad(got, want, prec, what):
    rel, ab = GTOL[prec]
    err = np.linalg.norm(got - want, axis=1)
    nrm = np.linalg.norm(want, axis=1)
    ratio = err / (rel * nrm + ab)
    say(f"  {what}: n={len(err)} max|dg|={err.max():.3e} max|dg|/|g|={np.max(err / np.maximum(nrm, 1e-12)):.3e} "
        f"mean|g|={nrm.mean():.3f} worst/tol={ratio.max():.3f}")
    assert ratio.max() <= 1.0, f"{what}: gradient error over tolerance"


def ray_points(n_w=240, n_h=135, seed=77):
    return synth.camera_ray_points(synth.random_primitives(2000), seed, width=n_w, height=n_h)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_grad_8x256_camera_rays(prec):
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    x = ray_points()
    say(f"case: 8x256 gradient, {len(x)} camera-ray samples, {prec}")
    g, y = run_grad(model, dm, x, prec)
    d = oracle.lookup_depth(x, dmap, 8)
    check_grad(g, oracle.gradient(ref, x, d), prec, f"8x256 {prec} adaptive")
    q = sand.query(model, dm, torch.from_numpy(x).to(DEV), precision=prec).cpu().numpy()
    assert np.array_equal(q.astype(np.float64), y), "gradient call's values differ from sand_query"


@pytest.mark.parametrize("W,L,tails", [(16, 1, "mult"), (64, 4, "linear"), (100, 3, "mult"),
                                       (128, 2, "mult"), (336, 5, "mult"), (352, 2, "linear")])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_grad_shapes(W, L, tails, prec):
    say(f"case: gradient W={W} L={L} {tails} tails {prec}")
    blob = synth.write_blob(synth.siren_tmlp(300 + W, L, W, tails=tails))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(W + L))
    dmap = rng.integers(1, L + 1, size=(8, 8, 8)).astype(np.uint8)
    dm = sand.build_depthmap(model, dmap)
    x = rng.uniform(-1, 1, size=(2500, 3)).astype(np.float32)
    g, y = run_grad(model, dm, x, prec)
    d = oracle.lookup_depth(x, dmap, L)
    check_grad(g, oracle.gradient(ref, x, d), prec, f"W={W} L={L} {prec}")
    g2, _ = run_grad(model, dm, x, prec, mode="full")
    check_grad(g2, oracle.gradient(ref, x, np.full(len(x), L)), prec, f"W={W} L={L} {prec} full")


def test_grad_central_differences():
    """FP32 gradient vs central differences of the FP64 oracle (h = 1e-3,
    depth frozen): the difference is the O(h^2) truncation error, estimated
    here by Richardson extrapolation."""
    blob = c2_blob(256)
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dmap = c2_map()
    dm = sand.build_depthmap(model, dmap)
    x = ray_points(64, 36, seed=5).astype(np.float64)
    d = oracle.lookup_depth(x, dmap, 8)
    g, _ = run_grad(model, dm, x.astype(np.float32), "fp32")

    def fd(h):
        out = np.zeros_like(x)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            out[:, a] = (oracle.forward(ref, x + e, d) - oracle.forward(ref, x - e, d)) / (2 * h)
        return out
    f1, f2 = fd(1e-3), fd(5e-4)
    rich = (4 * f2 - f1) / 3
    nrm = np.linalg.norm(rich, axis=1)
    e_fd = np.linalg.norm(g - f1, axis=1)
    e_rich = np.linalg.norm(g - rich, axis=1)
    say(f"  FD h=1e-3: max rel {np.max(e_fd / nrm):.3e}; Richardson: max rel {np.max(e_rich / nrm):.3e}")
    assert np.all(e_fd <= 1e-2 * nrm + 1e-3)
    assert np.all(e_rich <= 1e-3 * nrm + 1e-4)


def test_grad_dy_far_field_and_autograd():
    blob = synth.write_blob(synth.siren_tmlp(8, 3, 64, tails="mult"))
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    rng = np.random.Generator(np.random.PCG64(12))
    dmap = rng.integers(0, 4, size=(8, 8, 8)).astype(np.uint8)
    far = rng.normal(size=(8, 8, 8)).astype(np.float32)
    dm = sand.build_depthmap(model, dmap, far)
    x = rng.uniform(-1, 1, size=(3000, 3)).astype(np.float32)
    dy = rng.normal(size=3000).astype(np.float32)
    say("case: gradient with dy, far-field cells and autograd, 3x64, fp32")
    g1, y = run_grad(model, dm, x, "fp32")
    gd, _ = run_grad(model, dm, x, "fp32", dy=dy)
    d = oracle.lookup_depth(x, dmap, 3)
    assert np.all(g1[d == 0] == 0.0), "far-field points have zero gradient"
    assert np.allclose(gd, g1 * dy.astype(np.float64)[:, None], rtol=1e-6, atol=1e-7)
    check_grad(g1, oracle.gradient(ref, x, d), "fp32", "3x64 with far cells")
    assert np.allclose(y, oracle.forward(ref, x, d, far=far), rtol=0, atol=1e-5)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    out = sdf_fn(model, dm, xt)
    (out * torch.from_numpy(dy).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    assert np.allclose(xt.grad.cpu().numpy(), gd, rtol=0, atol=0), "autograd differs from query_grad"


def test_grad_lod_and_forced(c1=None):
    blob, dmap, xg = c1_case()
    ref = oracle.parse_blob(blob)
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, dmap)
    x = xg[::11]
    say(f"case: C1 gradient with LOD clamp and forced depths, {len(x)} points")
    for m in (1, 2, 3):
        g, _ = run_grad(model, dm, x, "fp32", max_depth=m)
        check_grad(g, oracle.gradient(ref, x, oracle.lookup_depth(x, dmap, 4, max_depth=m)), "fp32",
                   f"lod {m}")
    forced = np.random.Generator(np.random.PCG64(2)).integers(1, 5, size=len(x)).astype(np.uint8)
    g, _ = run_grad(model, None, x, "fp32", mode="forced",
                    forced_depth=torch.from_numpy(forced).to(DEV))
    check_grad(g, oracle.gradient(ref, x, forced), "fp32", "forced")
