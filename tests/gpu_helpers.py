"""Helpers shared by the GPU tests: run the HIP path through the C ABI and the
oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np

from oracle import theory as th
from oracle.lbm import Oracle
from oracle.local_weights import LocalOracle
from paper_1510_07328_amd import lbm

FAMILY = {lbm.LBM_W_FD_T0: th.FD_T0, lbm.LBM_W_MB: th.MB}


def gpu_run(cfg, n0, u0, checkpoints):
    """Moments (numpy float64) of the HIP path at each step count in checkpoints."""
    import torch

    lat = lbm.Lattice.create(cfg, n0, u0)
    out, done = [], 0
    for t in checkpoints:
        lat.step(t - done)
        done = t
        n, u = lat.moments()
        torch.cuda.synchronize()
        out.append((n.cpu().numpy(), u.cpu().numpy()))
    lat.free()
    return out


def oracle_model(cfg):
    lat = {lbm.LBM_D1V3: "d1v3", lbm.LBM_D2V9: "d2v9", lbm.LBM_D3V19: "d3v19", lbm.LBM_D2V41: "d2v41"}[cfg.lattice]
    if cfg.weight in (lbm.LBM_W_FD, lbm.LBM_W_BE):
        return th.make_model(lat, th.FD if cfg.weight == lbm.LBM_W_FD else th.BE, z=cfg.fugacity)
    fam = FAMILY[cfg.weight]
    return th.make_model(lat, fam, theta=1.0 / 3.0) if fam == th.MB else th.make_model(lat)


def make_oracle(cfg, shape, bc):
    """The oracle for cfg on a box of `shape`: the C oracle with the constant model,
    or the local-weight oracle (periodic only) for per-cell weights."""
    if cfg.weight == lbm.LBM_W_FD_LOCAL:
        if any(bc):
            raise ValueError("the local-weight oracle is periodic")
        lat = {lbm.LBM_D1V3: "d1v3", lbm.LBM_D2V9: "d2v9", lbm.LBM_D3V19: "d3v19"}[cfg.lattice]
        return LocalOracle(lat, shape, tau=cfg.tau, order=cfg.order, r0=cfg.theta_over_mu,
                           rho_ref=cfg.rho_ref if cfg.rho_ref > 0 else 1.0)
    return Oracle(oracle_model(cfg), shape=shape, bc=bc, tau=cfg.tau, order=cfg.order)


def oracle_run(cfg, n0, u0, checkpoints):
    o = make_oracle(cfg, (cfg.nx, cfg.ny, cfg.nz), tuple(cfg.bc))
    f = o.init(n0, u0)
    out, done = [], 0
    for t in checkpoints:
        f = o.run(f, t - done)
        done = t
        out.append(o.moments(f))
    return out


def rel_linf(a, b):
    """||a - b||_inf / ||b||_inf."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def field_errors(gpu, ref):
    """Relative L-infinity errors: n against max |n|, and each velocity component
    against the largest velocity component of the reference (normwise over the
    velocity field, so a component that is zero up to round-off is measured on
    the flow's scale); "u" is the largest of the components."""
    (n, u), (n_r, u_r) = gpu, ref
    errs = {"n": rel_linf(n, n_r), "dn": rel_linf(n - 1.0, n_r - 1.0) if np.max(np.abs(n_r - 1)) > 0 else 0.0}
    uscale = float(np.max(np.abs(u_r)))
    for d in range(u_r.shape[0]):
        errs[f"u{d}"] = float(np.max(np.abs(u[d] - u_r[d]))) / uscale if uscale > 0 else float(np.max(np.abs(u[d])))
    errs["u"] = max(errs[f"u{d}"] for d in range(u_r.shape[0]))
    return errs


def window_oracle(cfg, n0_full, u0_full, centers, half, steps):
    """Oracle values at sample cells of a periodic box after `steps` steps, from a
    window of side 2 (reach steps + half) + 1 around each sample: information
    travels at most `reach` cells per step (one, four on d2v41), so the window's
    own (wrong) periodic wrap cannot reach its central (2 half + 1)^D cells within
    `steps` steps.  Returns a list of (n, u) over each central block."""
    D = lbm.DIM[cfg.lattice]
    shape_full = (cfg.nz, cfg.ny, cfg.nx)[3 - D:]
    n_full = n0_full.reshape(shape_full)
    u_full = u0_full.reshape((D,) + shape_full)
    r = steps * (4 if cfg.lattice == lbm.LBM_D2V41 else 1) + half
    side = 2 * r + 1
    out = []
    for c in centers:  # c in (x, y[, z]) order
        idx = [np.arange(c[d] - r, c[d] + r + 1) % shape_full[D - 1 - d] for d in range(D)]
        sl = np.ix_(*idx[::-1])
        nw = n_full[sl].reshape(-1)
        uw = np.stack([u_full[d][sl].reshape(-1) for d in range(D)])
        o = make_oracle(cfg, (side,) * D, (0, 0, 0))
        f = o.run(o.init(nw, uw), steps)
        n, u = o.moments(f)
        inner = tuple(slice(r - half, r + half + 1) for _ in range(D))
        out.append((n.reshape((side,) * D)[inner], u.reshape((D,) + (side,) * D)[(slice(None),) + inner]))
    return out


def gpu_window(n, u, cfg, centers, half):
    D = u.shape[0]
    shape_full = (cfg.nz, cfg.ny, cfg.nx)[3 - D:]
    nf, uf = n.reshape(shape_full), u.reshape((D,) + shape_full)
    out = []
    for c in centers:
        idx = [np.arange(c[d] - half, c[d] + half + 1) % shape_full[D - 1 - d] for d in range(D)]
        sl = np.ix_(*idx[::-1])
        out.append((nf[sl], np.stack([uf[d][sl] for d in range(D)])))
    return out


def report_fp32(key, t, n_err, u_err):
    """One line per float32-deviation comparison (relative L-infinity errors), so
    that a run with -s lists every measured value next to its case."""
    print(f"FP32 {key} t={t}: n {n_err:.3e} u {u_err:.3e}", flush=True)
