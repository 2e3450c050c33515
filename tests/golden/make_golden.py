"""Write the oracle regression fixtures of this folder.

Calls only the oracle and the seeded workload generator.  The paper prints no
worked numerical example of any BEM quantity, so these fixtures hold the
oracle's own FP64 values for the tiny workload (4 handles x 32 segments,
eps = 1e-2, 256 elements per side); they guard the oracle against accidental
change, while the identities in test_oracle_*.py pin it to the mathematics.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from paper_2602_05492_amd import workload as W       # noqa: E402


def main():
    wl = W.make_config(1)
    x = wl.samples(0)[:12]
    u = O.evaluate(wl.theta_true, x, wl.cbar_true, wl.S, wl.eps, wl.elems_per_side)
    g = W.random_vector(77, (12, 3))
    grad = O.vjp(wl.theta_true, x, g, wl.S, wl.eps, wl.elems_per_side)
    out = {
        "source": "oracle (FP64 CPU) on the tiny workload, first 12 samples of step 0",
        "S": wl.S, "eps": wl.eps, "elems_per_side": wl.elems_per_side,
        "theta": wl.theta_true.tolist(), "x": x.tolist(), "cbar": wl.cbar_true.tolist(),
        "u": u.tolist(), "gbar_seed": 77, "vjp": grad.tolist(),
    }
    with open(os.path.join(os.path.dirname(__file__), "tiny_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
