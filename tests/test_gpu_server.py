"""Serving loop on one GPU: batched multi-model launches, HBM admission,
each request's result the same alone and in the mix (needs an MI355X)."""

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2604_25936_amd as sand
from gpu_cases import TOL, c2_blob, c2_map

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def models():
    """Four 8x256 models: two with band maps, two with random 1..8 maps."""
    out = []
    for k in range(4):
        blob = c2_blob(256, seed=1000 + k)
        m = sand.load_model(blob, 0)
        if k < 2:
            dmap = c2_map(seed=2000 + k)
        else:
            dmap = np.random.Generator(np.random.PCG64(k)).integers(
                1, 9, size=(64, 64, 64)).astype(np.uint8)
        out.append((blob, m, dmap, sand.build_depthmap(m, dmap)))
    return out


def request_points(k, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    half = n // 2
    slab = synth.slab_points(512, half, seed)
    pts = rng.uniform(-1, 1, size=(n - half, 3)).astype(np.float32)
    return np.ascontiguousarray(np.concatenate([slab, pts]))


def alone(m, dm, x, prec):
    y = sand.query(m, dm, torch.from_numpy(x).to(DEV), precision=prec)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_mix_equals_alone(models, prec):
    sizes = [1, 2, 77, 1000, 4096, 4097, 30000, 123457, 5, 250000, 999, 64000] * 2
    say(f"case: {len(sizes)} requests over 4 models, {prec}, 3 streams")
    srv = sand.Server(0, budget_bytes=1 << 30, precision=prec, n_streams=3)
    reqs = []
    for i, n in enumerate(sizes):
        k = i % 4
        x = request_points(k, n, seed=100 + i)
        y = np.full(n, np.nan, dtype=np.float32)
        reqs.append((k, x, y, srv.submit(models[k][1], models[k][3], x, y)))
    stats = [srv.wait(t) for (_, _, _, t) in reqs]
    info = srv.stats()
    say(f"  batches={info['batches']} max_batch={info['max_batch_requests']} "
        f"peak={info['peak_reserved_bytes']}")
    assert info["completed"] == len(sizes) and info["reserved_bytes"] == 0
    for (k, x, y, _), st in zip(reqs, stats):
        assert st["n"] == len(x)
        assert st["t_submit"] <= st["t_admit"] <= st["t_launch"] <= st["t_done"] <= st["t_copied"]
        assert np.array_equal(y, alone(models[k][1], models[k][3], x, prec)), \
            f"request of {len(x)} points differs from the same query alone"
    # a few requests against the oracle
    for (k, x, y, _) in reqs[5:8]:
        ref = oracle.parse_blob(models[k][0])
        d = oracle.lookup_depth(x, models[k][2], 8)
        err = np.abs(y.astype(np.float64) - oracle.forward(ref, x, d)).max()
        assert err <= TOL[prec], f"max |err| {err:.3e}"
    srv.close()


def test_batch_point_cap(models):
    """A batch closes at 2M points: a request above that runs alone, the
    others share batches up to it; every result equals the query alone."""
    sizes = [2_500_000, 800_000, 800_000, 800_000, 3, 5000, 700_000, 17]
    say(f"case: batch point cap, requests of {sizes} points, bf16")
    srv = sand.Server(0, budget_bytes=1 << 30, precision="bf16", n_streams=3)
    reqs = []
    for i, n in enumerate(sizes):
        k = i % 4
        x = request_points(k, n, seed=300 + i)
        y = np.full(n, np.nan, dtype=np.float32)
        reqs.append((k, x, y, srv.submit(models[k][1], models[k][3], x, y)))
    stats = [srv.wait(t) for (_, _, _, t) in reqs]
    info = srv.stats()
    say(f"  batches={info['batches']} batch sizes {[st['batch_size'] for st in stats]}")
    assert stats[0]["batch_size"] == 1, "a request above the cap must run alone"
    assert info["batches"] >= 3
    for (k, x, y, _) in reqs:
        assert np.array_equal(y, alone(models[k][1], models[k][3], x, "bf16"))
    srv.close()


def test_budget_admission_and_fifo(models):
    budget = 64 << 20
    srv = sand.Server(0, budget_bytes=budget, precision="bf16", n_streams=2)
    n = 1_000_000
    say(f"case: 12 requests of {n} points under a {budget >> 20} MiB budget")
    xs = [request_points(0, n, seed=300 + i) for i in range(12)]
    ys = [np.empty(n, dtype=np.float32) for _ in range(12)]
    tickets = [srv.submit(models[i % 4][1], models[i % 4][3], xs[i], ys[i]) for i in range(12)]
    st = [srv.wait(t) for t in tickets]
    info = srv.stats()
    say(f"  peak reserved {info['peak_reserved_bytes']} of {budget}, batches {info['batches']}")
    assert 0 < info["peak_reserved_bytes"] <= budget
    admits = [s["t_admit"] for s in st]
    assert admits == sorted(admits), "admission is first-in first-out"
    for i in (0, 5, 11):
        assert np.array_equal(ys[i], alone(models[i % 4][1], models[i % 4][3], xs[i], "bf16"))
    big = np.zeros((4_000_000, 3), dtype=np.float32)
    with pytest.raises(sand.SandError) as e:
        srv.submit(models[0][1], models[0][3], big, np.empty(4_000_000, dtype=np.float32))
    assert e.value.status == sand.sand.ERR_BUDGET
    srv.close()


def test_zero_size_timeout_and_errors(models):
    srv = sand.Server(0, budget_bytes=256 << 20, precision="bf16", n_streams=2)
    t0 = srv.submit(models[0][1], models[0][3], np.zeros((0, 3), np.float32), np.zeros(0, np.float32))
    assert srv.wait(t0)["n"] == 0
    with pytest.raises(sand.SandError) as e:
        srv.wait(123456)
    assert e.value.status == sand.sand.ERR_INVALID
    with pytest.raises(sand.SandError):
        srv.submit(models[0][1], models[1][3], np.zeros((5, 3), np.float32), np.zeros(5, np.float32))
    x = request_points(0, 3_000_000, seed=9)
    y = np.empty(len(x), dtype=np.float32)
    t = srv.submit(models[0][1], models[0][3], x, y)
    try:
        srv.wait(t, timeout=0.0)
        timed_out = False
    except sand.SandError as err:
        assert err.status == sand.sand.ERR_TIMEOUT
        timed_out = True
    if timed_out:
        srv.wait(t)
    say(f"  immediate wait timed out: {timed_out}")
    # an un-waited request is finished by close()
    x2 = request_points(1, 50000, seed=10)
    y2 = np.full(len(x2), np.nan, dtype=np.float32)
    srv.submit(models[1][1], models[1][3], x2, y2)
    srv.close()
    assert not np.any(np.isnan(y2)), "close() finishes queued requests"


def _c4_model(k):
    """Serving model k of the benchmark mix: 8x256 residual model (seed
    1000 + k), its 128^3 band map (surface seed 2000 + k) and a pool of
    near-surface points (generators only)."""
    prims = synth.random_primitives(2000 + k)
    return (c2_blob(256, seed=1000 + k), synth.band_map_c2(prims, R=128, L=8),
            synth.near_surface_points(prims, 1 << 14, seed=5000 + k))


def test_mix_equals_alone_16_models():
    """16 of the benchmark's resident models, requests of log-uniform size in
    [1e3, 4e6] (half a contiguous run of the 512^3 grid, half near-surface
    points), all submitted at once under the benchmark's 4 GB budget: every
    result equals the same query alone, bit for bit; the two smallest are
    checked against the oracle."""
    import concurrent.futures
    n_models, n_req = 16, 40
    with concurrent.futures.ProcessPoolExecutor(max_workers=8) as ex:
        inputs = list(ex.map(_c4_model, range(n_models)))
    ms = []
    for blob, dmap, _ in inputs:
        m = sand.load_model(blob, 0)
        ms.append((m, sand.build_depthmap(m, dmap)))
    rng = np.random.Generator(np.random.PCG64(77))
    sizes = np.exp(rng.uniform(np.log(1e3), np.log(4e6), size=n_req)).astype(np.int64)
    say(f"case: {n_req} requests over {n_models} models, {int(sizes.sum())} points, bf16")
    srv = sand.Server(0, budget_bytes=4 << 30, precision="bf16", n_streams=3)
    reqs = []
    for i, n in enumerate(sizes):
        k = i % n_models
        half = int(n) // 2
        start = int(rng.integers(0, 512 ** 3 - half))
        slab = synth.grid_points_at(512, np.arange(start, start + half, dtype=np.int64))
        pool = inputs[k][2]
        near = pool[rng.integers(0, len(pool), size=int(n) - half)]
        x = np.ascontiguousarray(np.concatenate([slab, near]))
        y = np.full(int(n), np.nan, dtype=np.float32)
        reqs.append((k, x, y, srv.submit(ms[k][0], ms[k][1], x, y)))
    stats = [srv.wait(t) for (_, _, _, t) in reqs]
    info = srv.stats()
    say(f"  batches={info['batches']} max_batch={info['max_batch_requests']} "
        f"peak={info['peak_reserved_bytes']}")
    assert info["completed"] == n_req and info["reserved_bytes"] == 0
    for (k, x, y, _), st in zip(reqs, stats):
        assert st["n"] == len(x)
        assert np.array_equal(y, alone(ms[k][0], ms[k][1], x, "bf16")), \
            f"request of {len(x)} points (model {k}) differs from the same query alone"
    for i in np.argsort(sizes)[:2]:
        k, x, y, _ = reqs[i]
        ref = oracle.parse_blob(inputs[k][0])
        d = oracle.lookup_depth(x, inputs[k][1], 8)
        err = np.abs(y.astype(np.float64) - oracle.forward(ref, x, d)).max()
        say(f"  request of {len(x)} points vs the oracle: max |err| {err:.2e}")
        assert err <= TOL["bf16"]
    srv.close()


def test_one_waiter_per_ticket(models):
    """A second wait on a ticket while another thread waits on it is
    rejected (the request is freed by exactly one waiter)."""
    import threading
    srv = sand.Server(0, budget_bytes=256 << 20, precision="bf16", n_streams=2)
    x = request_points(0, 3_000_000, seed=12)
    y = np.empty(len(x), dtype=np.float32)
    t = srv.submit(models[0][1], models[0][3], x, y)
    got = {}

    def first():
        got["st"] = srv.wait(t, timeout=30.0)

    th = threading.Thread(target=first)
    th.start()
    th.join(0.001)
    with pytest.raises(sand.SandError) as e:
        srv.wait(t, timeout=30.0)
    assert e.value.status == sand.sand.ERR_INVALID
    th.join()
    assert got["st"]["n"] == len(x)
    assert np.array_equal(y, alone(models[0][1], models[0][3], x, "bf16"))
    srv.close()
