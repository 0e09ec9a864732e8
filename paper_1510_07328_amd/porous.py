"""The porous-media (Ohm's law) workload of the paper's section "Numerical
simulations for electrons in metals": electrons flowing through rigid
obstacles at random positions in a periodic box, driven by a constant force;
the steady mean velocity along the force is linear in the force (Ohm's law for
electrons, Darcy's law for a classical fluid).  The paper uses a 700 x 150 box
with 30 discs of radius 3 (porosity 0.992) and tau = 0.7, and fits
<u>/<u>_min = a F/F_min through the origin.

Host driver only: every step runs in the library's porous kernels (solid cells
with halfway bounce-back, body force by the exact difference of equilibria);
the mean velocity comes from lbm_moments.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import inputs, lbm


def mean_velocity(lat, fluid_mask, axis: int = 0) -> float:
    """Mean of the velocity component `axis` over the fluid cells."""
    import torch

    n, u = lat.moments()
    torch.cuda.synchronize()
    ux = u[axis][fluid_mask]
    return float(ux.mean())


def steady_mean_velocity(cfg, solid, chunk: int = 2000, rtol: float = 1e-7, max_steps: int = 400_000,
                         axis: int = 0):
    """Run from rest (n = 1, u = 0) until the fluid-mean velocity along `axis`
    changes by less than rtol (relative) over one chunk of steps.  Returns
    (mean velocity, steps run, seconds of GPU time)."""
    import torch

    cells = cfg.nx * cfg.ny * cfg.nz
    D = lbm.DIM[cfg.lattice]
    lat = lbm.Lattice.create(cfg, np.ones(cells), np.zeros((D, cells)))
    lat.set_solid(solid)
    fluid = torch.as_tensor(np.asarray(solid).reshape(-1) == 0, device=lat.workspace.device)
    prev, steps, t_gpu = None, 0, 0.0
    try:
        while steps < max_steps:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(lat.stream)
            lat.step(chunk)
            e1.record(lat.stream)
            steps += chunk
            cur = mean_velocity(lat, fluid, axis)
            t_gpu += e0.elapsed_time(e1) * 1e-3
            if not math.isfinite(cur):
                raise RuntimeError("porous run broke down")
            if prev is not None and abs(cur - prev) <= rtol * abs(cur):
                break
            prev = cur
    finally:
        lat.free()
    return cur, steps, t_gpu


def fit_through_origin(x, y):
    """Least-squares slope a of y = a x and its standard error."""
    x, y = np.asarray(x, float), np.asarray(y, float)
    a = float(np.dot(x, y) / np.dot(x, x))
    dof = max(1, len(x) - 1)
    resid = y - a * x
    se = float(math.sqrt(np.dot(resid, resid) / dof / np.dot(x, x)))
    return a, se


def ohm_sweep(shape=(700, 150), discs: int = 30, radius: float = 3.0, seed: int = 0, tau: float = 0.7,
              forces=(1e-9, 2e-9, 3e-9, 4e-9, 5e-9), precision=lbm.LBM_FP32_DEV, order: int = 2,
              graph_steps: int = 200, chunk: int = 4000, rtol: float = 1e-7, max_steps: int = 600_000,
              block: int = 0):
    """Steady mean velocity along x for each force (along x) on the seeded
    porous box, and the fit of <u>/<u>_1 against F/F_1 through the origin.

    The cases run concurrently, one context and one stream each (a 700 x 150
    box fills only 150 workgroups); each stops when its fluid-mean velocity
    changes by less than rtol over `chunk` steps."""
    import torch

    solid = inputs.porous_obstacles(shape, discs, radius, seed=seed)
    cells = int(np.prod(shape))
    fluid = torch.as_tensor(np.asarray(solid).reshape(-1) == 0, device="cuda")
    lats, streams = [], []
    for F in forces:
        cfg = lbm.make_config("d2v9", shape=tuple(shape) + (1,), order=order, tau=tau, precision=precision,
                              scheme=lbm.LBM_SCHEME_AA, obstacles=1, force=(F, 0.0, 0.0), graph_steps=graph_steps,
                              block=block)
        st = torch.cuda.Stream()
        lat = lbm.Lattice.create(cfg, np.ones(cells), np.zeros((2, cells)), stream=st)
        lat.set_solid(solid)
        lats.append(lat)
        streams.append(st)
    torch.cuda.synchronize()
    prev = [None] * len(forces)
    cur = [None] * len(forces)
    steps = [0] * len(forces)
    done = [False] * len(forces)
    t0 = time.perf_counter()
    try:
        while not all(done):
            for k, lat in enumerate(lats):
                if not done[k]:
                    lat.step(chunk)
                    steps[k] += chunk
            torch.cuda.synchronize()
            for k, lat in enumerate(lats):
                if done[k]:
                    continue
                cur[k] = mean_velocity(lat, fluid)
                if not math.isfinite(cur[k]):
                    raise RuntimeError("porous run broke down")
                if (prev[k] is not None and abs(cur[k] - prev[k]) <= rtol * abs(cur[k])) or steps[k] >= max_steps:
                    done[k] = True
                prev[k] = cur[k]
        secs = time.perf_counter() - t0
    finally:
        for lat in lats:
            lat.free()
    rows = [{"force": F, "mean_u": u, "steps": n} for F, u, n in zip(forces, cur, steps)]
    x = np.array(forces) / forces[0]
    y = np.array(cur) / cur[0]
    a, se = fit_through_origin(x, y)
    updates = sum(steps) * cells
    return {"porosity": float(1.0 - solid.mean()), "runs": rows, "slope": a, "slope_stderr": se,
            "lattice_updates": updates, "wall_s": secs, "MLUPS": updates / secs / 1e6,
            "converged": all(n < max_steps for n in steps)}
