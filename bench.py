#!/usr/bin/env python3
"""Throughput of the SAND query path on one MI355X.

One step = one sand_query over every cell centre of the 512^3 grid
(134,217,728 points, FP32 coordinates already in HBM): depth lookup and
bucketing, the fused T-MLP to each point's exit depth, and the result
scatter. Workload: 8 sine layers of width 256 (SIREN init, tail 1 linear,
tails 2..8 multiplicative with residual-scaled weights), a 128^3 depth map
built from 12 seeded spheres and tori (distance bands plus a curvature
bump). Headline: adaptive BF16 queries/s. Printed beside it: the plain
full-depth FP32 form and other precisions/modes on the same GPU, the T-MLP
kernel's roofline position (MFMA), and the FP64 oracle on host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

G = 512
L, W = 8, 256
MODEL_SEED, SURFACE_SEED = 1000, 2000
PEAK = {"bf16": 2500.0, "fp16": 2500.0, "fp32": 157.3}   # dense MFMA TFLOP/s, MI355X
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tmlp_bf16_512grid_traffic.json")
KERNEL_SOURCES = ["paper_2604_25936_amd/csrc/tmlp_kernels.h",
                  "paper_2604_25936_amd/csrc/tmlp_sine.hip",
                  "paper_2604_25936_amd/csrc/mfma_common.h",
                  "paper_2604_25936_amd/csrc/sand_internal.h"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    """Hash of the T-MLP kernel's code (comments and blank lines removed, so
    that only a change of code invalidates the committed traffic counters)."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            t = f.read()
        t = re.sub(r"/\*.*?\*/", "", t, flags=re.S)
        t = re.sub(r"//[^\n]*", "", t)
        h.update("\n".join(ln.rstrip() for ln in t.split("\n") if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per T-MLP launch from committed rocprofv3 counters, if they
    were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def hidden_flops(depth_hist, width):
    """Algorithmic hidden-layer MFMA work: sum over points of 2 (d-1) W^2."""
    return sum(int(c) * 2 * max(d - 1, 0) * width * width for d, c in enumerate(depth_hist))


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(blob, dmap, n_sample, target_s=12.0, n_single=1 << 16):
    """The oracle on a uniform sample of the workload; the sample grows
    (up to 2^21 points) until it takes roughly target_s seconds. A smaller
    sample is also timed with one BLAS thread."""
    import oracle
    import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    model = oracle.parse_blob(blob)

    def run(n):
        x = synth.grid_points_at(G, synth.sample_indices(G ** 3, n, seed=5))
        t0 = time.perf_counter()
        d = oracle.lookup_depth(x, dmap, L)
        oracle.forward(model, x, d)
        return time.perf_counter() - t0

    while True:
        dt = run(n_sample)
        if dt >= target_s / 3 or n_sample >= 1 << 21:
            break
        n_sample = min(1 << 21, n_sample * max(2, 1 << int(target_s / max(dt, 1e-3)).bit_length() - 1))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        dt1 = run(n_single)
    # the small case in full: 4x64 linear-tail model, 32^3 sphere band map,
    # all 64^3 cell centres
    m1 = oracle.parse_blob(synth.write_blob(synth.siren_tmlp(1, 4, 64, tails="linear",
                                                             scale="plain")))
    dm1, x1 = synth.band_map_c1(32), synth.grid_points(64)
    t0 = time.perf_counter()
    oracle.forward(m1, x1, oracle.lookup_depth(x1, dm1, 4))
    dt_c1 = time.perf_counter() - t0
    rate = n_sample / dt
    return {"value": rate, "unit": "queries/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n_sample} uniformly sampled cells of the 512^3 grid, same model and "
                      f"map, FP64 numpy (lookup + adaptive forward), {dt:.1f} s",
            "cpu_model": cpu_model_name(), "host_cpus": os.cpu_count(),
            "extrapolated_512grid_s": G ** 3 / rate,
            "extrapolation": "linear in the point count (each query's work is independent)",
            "single_thread": {"value": n_single / dt1, "unit": "queries/s",
                              "sample": f"{n_single} cells, one BLAS thread, {dt1:.1f} s"},
            "small_case_full": {"value": x1.shape[0] / dt_c1, "unit": "queries/s",
                                "sample": f"all {x1.shape[0]} cell centres of the 64^3 grid, "
                                          f"4x64 linear-tail model, 32^3 sphere band map, "
                                          f"{dt_c1:.2f} s"}}


def valu_estimate(depth_hist, width):
    """Algorithmic vector work of one step beside the MFMA work: one sine per
    unit per evaluated layer, and the FP32 tail dot products (tail 1 linear:
    W FMAs; each multiplicative tail: 2W FMAs). Times are at MI355X's vector
    rates for this instruction mix: FP32 FMA without packing, 78.6 TFLOP/s;
    v_sin_f32 at a quarter of the FMA lane rate."""
    sines = sum(int(c) * width * d for d, c in enumerate(depth_hist))
    tail_flop = sum(int(c) * (2 * width + 4 * width * max(d - 1, 0))
                    for d, c in enumerate(depth_hist) if d > 0)
    fma_lanes_per_s = 78.6e12 / 2
    return {"sines": sines, "sine_ms_at_peak": sines / (fma_lanes_per_s / 4) * 1e3,
            "tail_fp32_flop": tail_flop, "tail_ms_at_peak": tail_flop / 78.6e12 * 1e3}


def torch_leg(torch, params, xyz, depth, chunk=1 << 20):
    """The same T-MLP in plain PyTorch FP32 on the same GPU (rocBLAS GEMMs,
    elementwise sine and tails), as context: every point to full depth, and
    adaptive by evaluating layer j only for the points whose exit depth is
    at least j (the points sorted by depth once, so each layer's active set
    is a prefix). Returns timings and the largest difference from the HIP
    kernel's FP32 full-depth result on the first chunk."""
    dev = xyz.device
    n = xyz.shape[0]
    f = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev)
    WsT = [f(w).t().contiguous() for w in params["weights"]]   # [in, out]
    bs = [f(b) for b in params["biases"]]
    om = [float(params["omega_first"])] + [float(params["omega_hidden"])] * (L - 1)
    tails = []
    for t in params["tails"]:
        if "a" in t:
            tails.append((f(t["a"]), float(t["c"]), None, 1.0))
        else:
            tails.append((f(t["a0"]), float(t["c0"]), f(t["a1"]), float(t["c1"])))

    def layer(j, h):
        h = torch.sin(om[j] * torch.addmm(bs[j], h, WsT[j]))
        a0, c0, a1, c1 = tails[j]
        t = h @ a0 + c0
        if a1 is not None:
            t = t * (h @ a1 + c1)
        return h, t

    def full(x):
        h, y = x, None
        for j in range(L):
            h, t = layer(j, h)
            y = t if y is None else y + t
        return y

    out = torch.empty(n, dtype=torch.float32, device=dev)

    def run_full():
        for s in range(0, n, chunk):
            out[s:s + chunk] = full(xyz[s:s + chunk])

    d_sorted, order = torch.sort(depth.to(torch.int32), descending=True)
    counts = [int((d_sorted >= j).sum()) for j in range(1, L + 1)]

    def run_adaptive():
        res = torch.empty(n, dtype=torch.float32, device=dev)
        for s in range(0, n, chunk):
            idx = order[s:s + chunk]
            x = xyz[idx]
            h, y = x, torch.zeros(idx.shape[0], dtype=torch.float32, device=dev)
            for j in range(L):
                m = max(0, min(counts[j] - s, idx.shape[0]))
                if m == 0:
                    break
                h, t = layer(j, h[:m])
                y[:m] += t
            res[idx] = y
        return res

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_full()
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    t0 = time.perf_counter()
    run_adaptive()
    torch.cuda.synchronize()
    t_ad = time.perf_counter() - t0
    return {"full_fp32": {"queries_per_s": n / t_full, "ms_per_step": t_full * 1e3},
            "adaptive_fp32_masked": {"queries_per_s": n / t_ad, "ms_per_step": t_ad * 1e3},
            "first_chunk_out": out[:chunk]}


def _c4_inputs(k):
    """Map and near-surface point pool of serving model k (CPU, generator only)."""
    import synth
    prims = synth.random_primitives(SURFACE_SEED + k)
    dmap = synth.band_map_c2(prims, R=128, L=L)
    pool = synth.near_surface_points(prims, 1 << 15, seed=5000 + k)
    return dmap, pool


def _c5_points():
    import synth
    return synth.camera_ray_points(synth.random_primitives(SURFACE_SEED), 77)


def gen_inputs(legs, n_models):
    """All CPU-side inputs, generated in worker processes before the GPU is used."""
    import concurrent.futures
    import synth
    out = {}
    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers) as ex:
        fut_c2 = ex.submit(synth.band_map_c2, synth.random_primitives(SURFACE_SEED), 128, L)
        fut_c5 = ex.submit(_c5_points) if ("grad" in legs or "finer" in legs) else None
        fut_c4 = [ex.submit(_c4_inputs, k) for k in range(n_models)] if "serving" in legs else []
        out["c2_map"] = fut_c2.result()
        if fut_c5 is not None:
            out["c5_points"] = fut_c5.result()
        out["c4"] = [f.result() for f in fut_c4]
    return out


def mapbuild_leg(sand, torch, model, prims, xyz, R=128, s=4, r=1.5e-4, reps=3):
    """Building the 128^3 network-depth map from the 8x256 model (Sec. 3.2,
    Eq. 5-7): near-surface voxels by the centre / half-diagonal test against
    the analytic scene, 4^3 sub-cell samples each (the 512^3 grid points in
    those voxels), FP32 full-depth pass with every y_i, r = 1.5e-4."""
    import numpy as np
    import synth
    near = synth.near_surface_mask(prims.sdf, R)
    csdf = synth.far_value_grid(prims.sdf, R)
    sand.construct_depthmap(model, near, csdf, s=s, r=r, precision="fp32")   # warm-up
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dm, depth, info = sand.construct_depthmap(model, near, csdf, s=s, r=r, precision="fp32")
        ts.append(time.perf_counter() - t0)
        dm.free()
    t = float(np.median(ts))
    # the 512^3 grid through the map built this way: far voxels return their
    # stored centre value without running the network (Eq. 7)
    dm, depth, info = sand.construct_depthmap(model, near, csdf, s=s, r=r, precision="fp32")
    out = torch.empty(xyz.shape[0], dtype=torch.float32, device=xyz.device)
    q = {}
    for prec in ("bf16", "fp32"):
        tq = time_steps(lambda p=prec: sand.query(model, dm, xyz, out=out, precision=p), 3, 1)
        q[prec] = {"queries_per_s": xyz.shape[0] / tq, "ms_per_step": tq * 1e3}
    dm.free()
    return {"R": R, "samples_per_axis": s, "r": r, "near_voxels": info["near_voxels"],
            "samples": info["samples"], "ms": t * 1e3, "samples_per_s": info["samples"] / t,
            "depth_counts": info["depth_counts"][:L + 1],
            "note": "host-inclusive: mask/centre upload, all kernels, map read-back",
            "query_512grid_with_this_map": q}


def octree_leg(sand, torch, model, xyz, D=9, s=1, r=1.5e-4, reps=3):
    """The paper's own pipeline on this model: build the sparse network-depth
    octree (max depth 9: level-9 leaves are the 512^3 grid's cells, one
    sample each, r = 1.5e-4, FP32), then query the 512^3 grid through it
    (far leaves answer from their stored value)."""
    import numpy as np
    sand.construct_octree(model, D=D, s=s, r=r)            # warm-up
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dm, info = sand.construct_octree(model, D=D, s=s, r=r)
        ts.append(time.perf_counter() - t0)
        dm.free()
    dm, info = sand.construct_octree(model, D=D, s=s, r=r)
    n = xyz.shape[0]
    out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    depth = torch.empty(n, dtype=torch.uint8, device=xyz.device)
    q = {}
    for prec in ("bf16", "fp32"):
        t = time_steps(lambda p=prec: sand.query(model, dm, xyz, out=out, precision=p,
                                                 depth_out=depth), 3, 1)
        q[prec] = {"queries_per_s": n / t, "ms_per_step": t * 1e3}
    hist = torch.bincount(depth.to(torch.int64), minlength=L + 1).cpu().numpy()
    dm.free()
    return {"D": D, "samples_per_axis": s, "r": r, "build_ms": float(np.median(ts)) * 1e3,
            "internal_nodes": info["internal_nodes"], "leaves": info["leaves"],
            "near_leaves": info["near_leaves"], "bytes": info["bytes"],
            "query_512grid": q, "query_exit_histogram": [int(c) for c in hist],
            "note": "build is host-inclusive (one host round trip per level)"}


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def serving_leg(sand, torch, inputs, n_models, n_payloads=128, n_measure=2000):
    """Poisson request stream over n_models resident 8x256 models (BF16)."""
    import numpy as np
    import synth
    rng = np.random.Generator(np.random.PCG64(7))
    models, maps = [], []
    for k in range(n_models):
        blob = synth.write_blob(synth.siren_tmlp(MODEL_SEED + k, L, W, tails="mult",
                                                 scale="residual"))
        m = sand.load_model(blob, 0)
        models.append(m)
        maps.append(sand.build_depthmap(m, inputs["c4"][k][0]))
    sizes = np.exp(rng.uniform(np.log(1e3), np.log(4e6), size=n_payloads)).astype(np.int64)
    payloads = []
    for i, n in enumerate(sizes):
        k = i % n_models
        half = int(n) // 2
        start = int(rng.integers(0, G ** 3 - half))
        slab = synth.grid_points_at(G, np.arange(start, start + half, dtype=np.int64))
        pool = inputs["c4"][k][1]
        near = pool[rng.integers(0, len(pool), size=int(n) - half)]
        x = torch.from_numpy(np.concatenate([slab, near])).pin_memory()
        y = torch.empty(int(n), dtype=torch.float32).pin_memory()
        payloads.append((k, x, y))
    budget = 4 << 30
    srv = sand.Server(0, budget_bytes=budget, precision="bf16", n_streams=3)

    def run(order, gaps):
        tickets = []
        t0 = time.perf_counter()
        t_next = t0
        for j, i in enumerate(order):
            if gaps is not None:
                t_next += gaps[j]
                while time.perf_counter() < t_next:
                    pass
            k, x, y = payloads[i]
            tickets.append((srv.submit(models[k], maps[k], x, y), x.shape[0]))
        st = [srv.wait(t) for t, _ in tickets]
        lat = [s["t_copied"] - s["t_submit"] for s in st]
        pts = sum(n for _, n in tickets)
        span = max(s["t_copied"] for s in st) - min(s["t_submit"] for s in st)
        return lat, pts, span, st

    run(list(range(16)), None)                       # warm-up
    lat, pts, span, _ = run(list(range(n_payloads)), None)   # burst: saturated rate
    sat_qps, sat_rps = pts / span, n_payloads / span
    mean_pts = float(sizes.mean())
    out = {"models": n_models, "payloads": n_payloads, "mean_request_points": mean_pts,
           "hbm_budget_bytes": budget, "streams": 3, "saturated_queries_per_s": sat_qps,
           "saturated_requests_per_s": sat_rps, "loads": {}}
    for load in (0.5, 0.8):
        rate = load * sat_rps
        gaps = rng.exponential(1.0 / rate, size=n_measure)
        order = [int(i) for i in rng.integers(0, n_payloads, size=n_measure)]
        log(f"serving: Poisson {rate:.0f} requests/s ({load}x saturation), {n_measure} requests")
        lat, pts, span, st = run(order, gaps)
        dev = [s["t_done"] - s["t_submit"] for s in st]       # results complete on the device
        d2h = [s["t_copied"] - s["t_done"] for s in st]       # the copy back to the host
        out["loads"][str(load)] = {
            "offered_requests_per_s": rate, "queries_per_s": pts / span,
            "p50_ms": percentile(lat, 50) * 1e3, "p99_ms": percentile(lat, 99) * 1e3,
            "device_p50_ms": percentile(dev, 50) * 1e3, "device_p99_ms": percentile(dev, 99) * 1e3,
            "d2h_p50_ms": percentile(d2h, 50) * 1e3, "d2h_p99_ms": percentile(d2h, 99) * 1e3,
            "mean_batch_requests": float(np.mean([s["batch_size"] for s in st])),
        }
    info = srv.stats()
    out["peak_reserved_bytes"] = info["peak_reserved_bytes"]
    out["batches"] = info["batches"]
    srv.close()
    return out


def grad_leg(sand, torch, inputs, dm_model):
    """Forward + input gradient over 1920x1080 camera-ray samples (8x256)."""
    import numpy as np
    import oracle
    model, dm, blob, dmap = dm_model
    x = inputs["c5_points"]
    xyz = torch.from_numpy(x).to("cuda:0")
    n = xyz.shape[0]
    sdf = torch.empty(n, dtype=torch.float32, device="cuda:0")
    g = torch.empty((n, 3), dtype=torch.float32, device="cuda:0")
    out = {"points": n}
    depth = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    for prec in ("bf16", "fp32"):
        ws = torch.empty(sand.query_grad_workspace_size(model, n, prec), dtype=torch.uint8,
                         device="cuda:0")
        t = time_steps(lambda: sand.query_grad(model, dm, xyz, sdf_out=sdf, grad_out=g,
                                               precision=prec, workspace=ws), 5, 2)
        sand.query_grad(model, dm, xyz, sdf_out=sdf, grad_out=g, precision=prec, workspace=ws,
                        depth_out=depth)
        hist = torch.bincount(depth.to(torch.int64), minlength=L + 1).cpu().numpy()
        # algorithmic MFMA work: the forward and the transposed backward products,
        # 2 (d - 1) W^2 flop each per point (whole step, bucketing included)
        fl = 2 * hidden_flops(hist, W)
        idx = np.random.Generator(np.random.PCG64(3)).choice(n, 4000, replace=False)
        ref = oracle.parse_blob(blob)
        d = oracle.lookup_depth(x[idx], dmap, L)
        want = oracle.gradient(ref, x[idx], d)
        got = g.cpu().numpy()[idx].astype(np.float64)
        rel = np.linalg.norm(got - want, axis=1) / np.maximum(np.linalg.norm(want, axis=1), 1e-12)
        out[prec] = {"queries_per_s": n / t, "ms_per_step": t * 1e3,
                     "mean_exit_depth": float((hist * np.arange(L + 1)).sum() / max(1, hist.sum())),
                     "mfma_tflops_step": fl / t / 1e12, "mfma_frac_step": fl / t / 1e12 / PEAK[prec],
                     "grad_max_rel_err_4k_sample": float(rel.max()),
                     "grad_mean_rel_err_4k_sample": float(rel.mean())}
    return out


def error_sample(n, n_err=1 << 20):
    """The seeded 1M-point uniform subsample of the 512^3 grid (without
    replacement) on which SDF errors are measured: indices and points."""
    import synth
    idx = synth.sample_indices(n, n_err, seed=11)
    return idx, synth.grid_points_at(G, idx)


def error_study(sand, torch, model, dm, blob, dmap, xyz, sample, precs, sdf):
    """Max and mean |SDF - FP64 oracle| of adaptive queries over the whole
    512^3 grid, read at the sample's points, and sign agreement among sample
    points with |y_oracle| < 0.01."""
    import numpy as np
    import oracle
    idx, xs = sample
    ref = oracle.parse_blob(blob)
    want = oracle.forward(ref, xs, oracle.lookup_depth(xs, dmap, L))
    near = np.abs(want) < 0.01
    idx_t = torch.from_numpy(idx).to(xyz.device)
    out = {"sample_points": int(len(idx)), "sample_points_near_surface": int(near.sum())}
    for prec in precs:
        sand.query(model, dm, xyz, out=sdf, precision=prec)
        got = sdf[idx_t].cpu().numpy().astype(np.float64)
        err = np.abs(got - want)
        out[prec] = {"max_abs_err": float(err.max()), "mean_abs_err": float(err.mean()),
                     "sign_agreement_near_surface": float(np.mean(
                         np.sign(got[near]) == np.sign(want[near]))) if near.any() else None}
    return out


def finer_leg(sand, torch, inputs, xyz, dmap, sample, ws):
    """SAND-FINER (Sec. 4.1): the 8x256 model on the FINER backbone,
    sin(omega (|z| + 1) z), same map and grid. Throughput per precision and
    mode, the T-MLP kernel's algorithmic MFMA rate, the 1M-sample error
    study, and forward + gradient over the 1920x1080 camera-ray samples."""
    import numpy as np
    import oracle
    import synth
    blob = synth.write_blob(synth.siren_tmlp(MODEL_SEED, L, W, tails="mult", scale="residual",
                                             activation="finer"))
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, dmap)
    n = xyz.shape[0]
    sdf = torch.empty(n, dtype=torch.float32, device=xyz.device)
    depth = torch.empty(n, dtype=torch.uint8, device=xyz.device)
    sand.query(model, dm, xyz, out=sdf, precision="bf16", depth_out=depth, workspace=ws)
    hist = torch.bincount(depth.to(torch.int64), minlength=L + 1).cpu().numpy()
    out = {"model": "8x256 FINER backbone (first-layer bias U(-1, 1)), same draws otherwise"}
    for prec, mode in (("bf16", "adaptive"), ("fp16", "adaptive"), ("fp32", "adaptive"),
                       ("bf16", "full"), ("fp32", "full")):
        k = 2 if mode == "full" else 5
        t = time_steps(lambda p=prec, m=mode: sand.query(model, dm, xyz, out=sdf, precision=p,
                                                         mode=m, workspace=ws), k, 1)
        _, ms = sand.query_timed(model, dm, xyz, out=sdf, precision=prec, mode=mode, workspace=ws)
        fl = n * 2 * (L - 1) * W * W if mode == "full" else hidden_flops(hist, W)
        out[f"{mode}_{prec}"] = {"queries_per_s": n / t, "ms_per_step": t * 1e3, "tmlp_ms": ms[3],
                                 "mfma_frac": fl / (ms[3] / 1e3) / 1e12 / PEAK[prec]}
    out["errors"] = error_study(sand, torch, model, dm, blob, dmap, xyz, sample,
                                ("bf16", "fp16", "fp32"), sdf)
    out["gradient"] = grad_leg(sand, torch, inputs, (model, dm, blob, dmap))
    return out


def c3_leg(sand, torch, xyz, dmap, n_err=1 << 20):
    """8x336 on the 512^3 grid: throughput per precision and the error study
    (max/mean |SDF error| vs the FP64 oracle on a seeded 1M-point sample, and
    sign agreement among sample points with |y_oracle| < 0.01)."""
    import numpy as np
    import oracle
    import synth
    blob = synth.write_blob(synth.siren_tmlp(MODEL_SEED + 336, L, 336, tails="mult",
                                             scale="residual"))
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, dmap)
    n = xyz.shape[0]
    sdf = torch.empty(n, dtype=torch.float32, device="cuda:0")
    ws = torch.empty(sand.query_workspace_size(n), dtype=torch.uint8, device="cuda:0")
    idx = synth.sample_indices(n, n_err, seed=11)
    xs = synth.grid_points_at(G, idx)
    ref = oracle.parse_blob(blob)
    want = oracle.forward(ref, xs, oracle.lookup_depth(xs, dmap, L))
    near = np.abs(want) < 0.01
    idx_t = torch.from_numpy(idx).to("cuda:0")
    out = {"sample_points": n_err, "sample_points_near_surface": int(near.sum())}
    for prec, mode in (("bf16", "adaptive"), ("fp16", "adaptive"), ("fp32", "adaptive"),
                       ("fp32", "full")):
        k = 2 if mode == "full" else 3
        t = time_steps(lambda: sand.query(model, dm, xyz, out=sdf, precision=prec, mode=mode,
                                          workspace=ws), k, 1)
        r = {"queries_per_s": n / t, "ms_per_step": t * 1e3}
        if mode == "adaptive":
            got = sdf[idx_t].cpu().numpy().astype(np.float64)
            err = np.abs(got - want)
            r.update({"max_abs_err": float(err.max()), "mean_abs_err": float(err.mean()),
                      "sign_agreement_near_surface": float(np.mean(
                          np.sign(got[near]) == np.sign(want[near]))) if near.any() else None})
        out[f"{mode}_{prec}"] = r
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default="all",
                    help="'all', or a comma list of headline,compare,c3,grad,serving,mapbuild,"
                         "octree,cpu,errors,finer")
    ap.add_argument("--cpu-sample", type=int, default=131072)
    ap.add_argument("--serving-models", type=int, default=64)
    ap.add_argument("--headline-mode", default="adaptive", choices=["adaptive", "full"],
                    help="mode of the timed leg (full: every point to depth L; for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a 1 GiB elementwise copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); the query path "
              "shards by splitting the point set, with no exchange, and is not run on several "
              "GPUs here.", file=sys.stderr)
        sys.exit(2)
    legs = {"headline", "compare", "c3", "grad", "serving", "mapbuild", "octree", "cpu",
            "errors", "finer"} \
        if args.legs == "all" else \
        set(args.legs.split(",")) | {"headline"}

    log("generating inputs on the host")
    inputs = gen_inputs(legs, args.serving_models)

    import numpy as np
    import torch
    import synth
    import paper_2604_25936_amd as sand

    dev = "cuda:0"
    log("building inputs: 8x256 T-MLP, 128^3 map, 512^3 grid")
    blob = synth.write_blob(synth.siren_tmlp(MODEL_SEED, L, W, tails="mult", scale="residual"))
    dmap = inputs["c2_map"]
    model = sand.load_model(blob, 0)
    dm = sand.build_depthmap(model, dmap)
    xyz = synth.queries.grid_points_torch(G, dev)
    n = xyz.shape[0]
    sdf = torch.empty(n, dtype=torch.float32, device=dev)
    depth = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = torch.empty(sand.query_workspace_size(n), dtype=torch.uint8, device=dev)

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 3 x (1 GiB read + 1 GiB write) elementwise kernels")

    sand.query(model, dm, xyz, out=sdf, precision="bf16", depth_out=depth, workspace=ws)
    torch.cuda.synchronize()
    hist = torch.bincount(depth.to(torch.int64), minlength=L + 1).cpu().numpy()
    flops = hidden_flops(hist, W)
    full_flops = n * 2 * (L - 1) * W * W

    def step(prec="bf16", mode="adaptive"):
        return lambda: sand.query(model, dm, xyz, out=sdf, precision=prec, mode=mode, workspace=ws)

    hmode = args.headline_mode
    head_flops = full_flops if hmode == "full" else flops
    log(f"headline: {hmode} bf16, {args.steps} steps after {args.warmup} warm-up")
    t_step = time_steps(step(mode=hmode), args.steps, args.warmup)
    # the dominant kernel's own duration, HIP events on the launch stream
    phases = []
    for _ in range(max(3, min(args.steps, 10))):
        _, ms = sand.query_timed(model, dm, xyz, out=sdf, precision="bf16", mode=hmode,
                                 workspace=ws)
        phases.append(ms)
    phases = np.array(phases)
    t_kernel = float(phases[:, 3].mean()) / 1e3
    achieved = head_flops / t_kernel / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK["bf16"],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK["bf16"], 4),
                "traffic": measured_traffic()}

    comparisons = {}
    if "compare" in legs:
        for prec, mode in [("fp32", "full"), ("fp32", "adaptive"), ("bf16", "full"),
                           ("fp16", "adaptive"), ("fp16", "full")]:
            k = 2 if (prec == "fp32" and mode == "full") else 3
            log(f"comparison: {mode} {prec}, {k} steps")
            t = time_steps(step(prec, mode), k, 1)
            _, ms = sand.query_timed(model, dm, xyz, out=sdf, precision=prec, mode=mode,
                                     workspace=ws)
            fl = full_flops if mode == "full" else flops
            comparisons[f"{mode}_{prec}"] = {
                "queries_per_s": n / t, "ms_per_step": t * 1e3,
                "tmlp_ms": ms[3], "mfma_tflops": fl / (ms[3] / 1e3) / 1e12,
                "mfma_frac": fl / (ms[3] / 1e3) / 1e12 / PEAK[prec]}
        comparisons["speedup_adaptive_bf16_vs_full_fp32"] = \
            comparisons["full_fp32"]["ms_per_step"] / (t_step * 1e3)
        # map-free dynamic early exit on |t_j| < r (the Sec. 4.4 ablation), r = 1.5e-4
        # (checkpoint 0: the library picks the compaction layer from a sample;
        # -1: no compaction, a tile runs as deep as its deepest point)
        for prec in ("bf16", "fp32"):
            log(f"comparison: dynamic early exit without a map, {prec}")
            res = {"r": 1.5e-4}
            for name, cp in (("compacted", 0), ("uncompacted", -1)):
                dyn = lambda p=prec, c=cp: sand.query(model, None, xyz, out=sdf, precision=p,
                                                      mode="dynamic", dynamic_r=1.5e-4,
                                                      depth_out=depth, dynamic_checkpoint=c)
                t = time_steps(dyn, 2, 1)
                res[name] = {"queries_per_s": n / t, "ms_per_step": t * 1e3}
            dh = torch.bincount(depth.to(torch.int64), minlength=L + 1).cpu().numpy()
            res["exit_histogram"] = [int(c) for c in dh]
            res["hidden_mfma_flop_algorithmic"] = hidden_flops(dh, W)
            comparisons[f"dynamic_{prec}"] = res
        # restore the headline's depths for anything after
        sand.query(model, dm, xyz, out=sdf, precision="bf16", depth_out=depth, workspace=ws)
        # plain PyTorch FP32 of the same model on this GPU (context)
        try:
            log("comparison: plain PyTorch FP32, full depth and depth-masked")
            params = synth.siren_tmlp(MODEL_SEED, L, W, tails="mult", scale="residual")
            tl = torch_leg(torch, params, xyz, depth)
            ref = tl.pop("first_chunk_out")
            sand.query(model, dm, xyz[:ref.shape[0]], out=sdf[:ref.shape[0]], precision="fp32",
                       mode="full", workspace=ws)
            tl["max_abs_diff_vs_hip_fp32_full_first_chunk"] = float(
                (sdf[:ref.shape[0]] - ref).abs().max())
            comparisons["torch"] = tl
        except Exception as e:  # noqa: BLE001
            log(f"torch comparison failed: {e!r}")
            comparisons["torch"] = {"error": repr(e)}

    line = {
        "metric": f"{hmode} queries/s on 512^3 grid (8x256 SIREN T-MLP, BF16 hidden GEMMs)",
        "value": n / t_step, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "512^3 grid cell centres; 8 sine layers x 256 (SIREN init, tail 1 "
                               "linear, tails 2-8 multiplicative, residual-scaled); 128^3 depth "
                               "map from 12 seeded spheres/tori (bands + curvature bump)",
                   "points": n, "layers": L, "width": W, "map_resolution": 128,
                   "mode": hmode, "precision": "bf16", "parallelism": "single GPU"},
        "roofline": roofline,
        "valu": valu_estimate(hist, W),
        "phases_ms": {k: round(float(v), 4) for k, v in
                      zip(["lookup", "scan", "scatter", "tmlp", "total"], phases.mean(axis=0))},
        "depth_histogram": [int(c) for c in hist],
        "hidden_mfma_flop_per_step": flops,
        "comparisons": comparisons,
    }
    def secondary(name, fn):
        # a failing secondary leg is reported in its entry; the headline stands
        try:
            line[name] = fn()
        except Exception as e:  # noqa: BLE001
            log(f"{name} leg failed: {e!r}")
            line[name] = {"error": repr(e)}

    sample = error_sample(n) if ("errors" in legs or "finer" in legs) else None
    if "errors" in legs:
        log("error study: the headline model, and the same model with unit-scale tails (stress)")

        def errors():
            out = {"headline": error_study(sand, torch, model, dm, blob, dmap, xyz, sample,
                                           ("bf16", "fp16", "fp32"), sdf)}
            sblob = synth.write_blob(synth.siren_tmlp(MODEL_SEED, L, W, tails="mult",
                                                      scale="plain"))
            sm = sand.load_model(sblob, 0)
            out["unit_scale_tails"] = error_study(sand, torch, sm, sand.build_depthmap(sm, dmap),
                                                  sblob, dmap, xyz, sample,
                                                  ("bf16", "fp16", "fp32"), sdf)
            return out
        secondary("errors_1m_sample", errors)
    if "finer" in legs:
        log("FINER leg: the 8x256 model on the FINER backbone")
        secondary("finer", lambda: finer_leg(sand, torch, inputs, xyz, dmap, sample, ws))
    if "c3" in legs:
        log("8x336 leg: throughput per precision and error study")
        secondary("width336", lambda: c3_leg(sand, torch, xyz, dmap))
    del ws
    if "grad" in legs:
        log("gradient leg: 1920x1080 camera-ray samples")
        secondary("gradient", lambda: grad_leg(sand, torch, inputs, (model, dm, blob, dmap)))
    if "mapbuild" in legs:
        log("map construction leg: 128^3 map from the 8x256 model, 4^3 samples per near voxel")
        secondary("mapbuild", lambda: mapbuild_leg(sand, torch, model,
                                                   synth.random_primitives(SURFACE_SEED), xyz))
    if "octree" in legs:
        log("octree leg: max-depth-9 network-depth octree from the 8x256 model, 512^3 queries")
        secondary("octree", lambda: octree_leg(sand, torch, model, xyz))
    if "serving" in legs:
        log(f"serving leg: {args.serving_models} resident models")
        secondary("serving", lambda: serving_leg(sand, torch, inputs, args.serving_models))
    if args.cpu_sample > 0 and "cpu" in legs:
        log(f"cpu baseline: oracle on {args.cpu_sample} sampled points")
        line["cpu_baseline"] = cpu_baseline(blob, dmap, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
