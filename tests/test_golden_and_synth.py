"""Stored oracle values and generator shapes (CPU only)."""

import json
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_reproduces_stored_sample():
    with open(os.path.join(HERE, "golden", "c1_oracle_sample.json")) as f:
        g = json.load(f)
    model = oracle.parse_blob(synth.write_blob(
        synth.siren_tmlp(g["model_seed"], 4, 64, tails="linear", scale="plain")))
    x = synth.grid_points_at(g["grid"], np.array(g["index"]))
    d = oracle.lookup_depth(x, synth.band_map_c1(32), 4)
    assert d.tolist() == g["depth"]
    y = oracle.forward(model, x, d)
    want = np.array([float.fromhex(v) for v in g["y"]])
    assert np.allclose(y, want, rtol=0, atol=1e-14)
    gr = oracle.gradient(model, x, d)
    wantg = np.array([[float.fromhex(v) for v in r] for r in g["grad"]])
    assert np.allclose(gr, wantg, rtol=1e-13, atol=1e-13)


def test_c1_band_map_histogram():
    """Depth shares of the 32^3 sphere band map: 61.67/26.25/8.11/3.98 %."""
    m = synth.band_map_c1(32)
    h = np.bincount(m.ravel(), minlength=5) / m.size
    assert np.allclose(h[1:], [0.61669922, 0.26245117, 0.08105469, 0.03979492], atol=1e-8)


def test_grid_points_exact_and_ordered():
    p = synth.grid_points(8)
    assert p.dtype == np.float32 and p.shape == (512, 3)
    assert np.array_equal(p, synth.grid_points_at(8, np.arange(512)))
    c = (2 * np.arange(8) + 1) / 8 - 1
    assert np.array_equal(p[:8, 2], c.astype(np.float32))
    assert np.array_equal(p[::64, 0], c.astype(np.float32))


def test_blob_roundtrip_and_size():
    m = synth.siren_tmlp(3, 3, 32)
    b = synth.write_blob(m)
    assert len(b) == synth.blob_nbytes(3, 32, [0, 1, 1])
    p = oracle.parse_blob(b)
    assert p["L"] == 3 and p["W"] == 32
    assert np.array_equal(p["W_"][1], m["weights"][1].astype(np.float64))
    assert [t[0] for t in p["tails"]] == ["linear", "mult", "mult"]


def test_generators_are_seeded():
    a = synth.write_blob(synth.siren_tmlp(9, 2, 16))
    b = synth.write_blob(synth.siren_tmlp(9, 2, 16))
    c = synth.write_blob(synth.siren_tmlp(10, 2, 16))
    assert a == b and a != c
    assert np.array_equal(synth.sample_indices(1000, 10, 4), synth.sample_indices(1000, 10, 4))
