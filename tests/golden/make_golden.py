"""Write the stored expected values under tests/golden/ from the float64 oracle.

Only the oracle computes these values; the seeded input generator supplies the
initial fields.  Run from the repository root:

    python tests/golden/make_golden.py

rf256_order2.npz -- a 256 x 256 periodic d2v9 field with the recipe of the
2048 x 2048 workload (n = 1 + 0.01 G, G a periodic Gaussian random field of
correlation length 32 cells, seed 0; drift u_x = 1e-4 c_0; tau = 0.55; second
order), moments n and u0 after 1000, 3000 and 10000 steps, used to measure the
float32 deviation path's error against float64 over a long run.

rf2048_order2_rows.npz -- the 2048 x 2048 workload itself (same recipe, correlation
length 32 cells), second order, tau = 0.55, after 25, 1000, 3000 and 10000
steps: the full field's largest |n|, |n - 1| and |u0| (the normalisations of
the relative L-infinity errors), and n and u0 on sampled rows: five fixed rows
plus, per checkpoint, the rows holding the largest |u0| and |n - 1|.  Writing
it takes about 15-30 minutes on 8 host threads.

    python tests/golden/make_golden.py rf2048
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


RF2048_N, RF2048_CHECKPOINTS, RF2048_FIXED_ROWS = 2048, (25, 1000, 3000, 10000), (0, 337, 1024, 1361, 2047)


def make_rf2048():
    N = RF2048_N
    n0, u0 = inputs.perturbed_field((N, N), 0.01, 32.0, (1e-4, 0.0), seed=0)
    o = Oracle(th.make_model("d2v9"), shape=(N, N), tau=RF_TAU, order=2)
    f = o.init(n0, u0)
    del n0, u0
    out, done = {}, 0
    for t in RF2048_CHECKPOINTS:
        t0 = time.time()
        o.run(f, t - done)
        done = t
        n, u = o.moments(f)
        n, u = n.reshape(N, N), u.reshape(2, N, N)
        umag = np.abs(u).max(axis=0)
        r_u = int(np.unravel_index(np.argmax(umag), umag.shape)[0])
        r_n = int(np.unravel_index(np.argmax(np.abs(n - 1.0)), n.shape)[0])
        rows = np.array(sorted(set(RF2048_FIXED_ROWS) | {r_u, r_n}), dtype=np.int64)
        out[f"rows_{t}"] = rows
        out[f"n_{t}"] = n[rows]
        out[f"u_{t}"] = u[:, rows]
        out[f"max_n_{t}"] = np.float64(np.abs(n).max())
        out[f"max_dn_{t}"] = np.float64(np.abs(n - 1.0).max())
        out[f"max_u_{t}"] = np.float64(np.abs(u).max())
        print(f"t={t} ({time.time() - t0:.0f} s) rows {rows.tolist()} max|u| {out[f'max_u_{t}']:.6e}",
              flush=True)
        del n, u, umag
    out["checkpoints"] = np.array(RF2048_CHECKPOINTS)
    np.savez_compressed(os.path.join(HERE, "rf2048_order2_rows.npz"), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["rf256"]
    if "rf256" in which:
        make_rf256()
    if "rf2048" in which:
        make_rf2048()
