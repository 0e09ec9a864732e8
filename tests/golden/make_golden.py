"""Write the stored expected values under tests/golden/ from the float64 oracle.

Only the oracle computes these values; the seeded input generator supplies the
initial fields.  Run from the repository root:

    python tests/golden/make_golden.py

rf256_order2.npz -- a 256 x 256 periodic d2v9 field with the recipe of the
2048 x 2048 workload (n = 1 + 0.01 G, G a periodic Gaussian random field of
correlation length 32 cells, seed 0; drift u_x = 1e-4 c_0; tau = 0.55; second
order), moments n and u0 after 1000, 3000 and 10000 steps, used to measure the
float32 deviation path's error against float64 over a long run.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import theory as th  # noqa: E402
from oracle.lbm import Oracle  # noqa: E402
from paper_1510_07328_amd import inputs  # noqa: E402

RF_N, RF_TAU, RF_CHECKPOINTS = 256, 0.55, (1000, 3000, 10000)


def make_rf256():
    n0, u0 = inputs.perturbed_field((RF_N, RF_N), 0.01, 32.0, (1e-4, 0.0), seed=0)
    o = Oracle(th.make_model("d2v9"), shape=(RF_N, RF_N), tau=RF_TAU, order=2)
    f = o.init(n0, u0)
    out, done = {}, 0
    for t in RF_CHECKPOINTS:
        t0 = time.time()
        o.run(f, t - done)
        done = t
        n, u = o.moments(f)
        out[f"n_{t}"], out[f"u_{t}"] = n, u
        print(f"t={t} ({time.time() - t0:.0f} s)", flush=True)
    out["checkpoints"] = np.array(RF_CHECKPOINTS)
    np.savez_compressed(os.path.join(HERE, "rf256_order2.npz"), **out)


if __name__ == "__main__":
    make_rf256()
