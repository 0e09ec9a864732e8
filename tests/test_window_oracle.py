"""The light-cone window used to check full-size GPU runs at sample cells gives
exactly the oracle's full-box values (CPU only)."""
import numpy as np

from gpu_helpers import window_oracle
from oracle.lbm import Oracle
from oracle import theory as th
from paper_1510_07328_amd import inputs, lbm


def test_window_oracle_matches_full_box():
    nx, ny, steps = 61, 47, 6
    cfg = lbm.make_config("d2v9", shape=(nx, ny, 1), order=2, tau=0.55)
    n0, u0 = inputs.perturbed_field((ny, nx), 0.02, 4.0, (0.01, 0.0), seed=3)
    o = Oracle(th.make_model("d2v9"), shape=(nx, ny), tau=0.55, order=2)
    f = o.init(n0, u0)
    o.run(f, steps)
    n, u = o.moments(f)
    n, u = n.reshape(ny, nx), u.reshape(2, ny, nx)
    centers = [(0, 0), (60, 46), (30, 2)]
    for c, (wn, wu) in zip(centers, window_oracle(cfg, n0, u0, centers, half=3, steps=steps)):
        ys = np.arange(c[1] - 3, c[1] + 4) % ny
        xs = np.arange(c[0] - 3, c[0] + 4) % nx
        np.testing.assert_array_equal(wn, n[np.ix_(ys, xs)])
        np.testing.assert_array_equal(wu, u[(slice(None),) + np.ix_(ys, xs)])
