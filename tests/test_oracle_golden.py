"""Oracle regression against its committed fixture (tests/golden/tiny_oracle.json, written by
tests/golden/make_golden.py from the oracle alone)."""
import json
import os

import numpy as np

import oracle as O
from paper_2602_05492_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_oracle.json")


def test_tiny_oracle_fixture():
    with open(GOLDEN) as f:
        g = json.load(f)
    theta = np.array(g["theta"])
    x = np.array(g["x"])
    wl = W.make_config(1)
    assert np.array_equal(theta, wl.theta_true)           # generator unchanged
    assert np.array_equal(x, wl.samples(0)[:12])
    u = O.evaluate(theta, x, np.array(g["cbar"]), g["S"], g["eps"], g["elems_per_side"])
    assert np.allclose(u, np.array(g["u"]), rtol=1e-13, atol=1e-14)
    grad = O.vjp(theta, x, W.random_vector(g["gbar_seed"], (12, 3)), g["S"], g["eps"], g["elems_per_side"])
    ref = np.array(g["vjp"])
    assert np.abs(grad - ref).max() <= 1e-12 * np.abs(ref).max()
