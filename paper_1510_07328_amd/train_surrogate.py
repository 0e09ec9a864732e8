"""Train the convolutional surrogate on shock-tube trajectories of the batched
lattice sweep and save its parameters.

    python -m paper_1510_07328_amd.train_surrogate [--tubes 20000] [--steps 20000] [--out PATH]

Training data: `tubes` closed tubes of 1024 x 4 cells, n_L = 1, n_R / n_L and tau
drawn uniformly (seeded), snapshots of the row-averaged (n, u_x) every 64
steps for 4096 steps, all generated on the GPU by the batched sweep; tubes that
break down are left out.  Optimiser: Adam on random (snapshot, snapshot + 1)
pairs with a cosine learning-rate decay (forward, loss, backward and Adam all
run in the library's kernels).  The saved file holds the float32 parameter
vector and a JSON record of the settings and of the one-jump error on held-out
tubes.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import surrogate as S

DEFAULT_OUT = S.WEIGHTS


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--tubes", type=int, default=20000)
    ap.add_argument("--snapshots", type=int, default=64)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lambda-mass", type=float, default=1.0)
    ap.add_argument("--pushforward", type=float, default=0.0)
    ap.add_argument("--push-max", type=int, default=1, help="longest own-prediction rollout of a pushforward step")
    ap.add_argument("--push-start", type=float, default=0.5, help="fraction of the steps before pushforward starts")
    ap.add_argument("--data-seed", type=int, default=2)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--heldout-seed", type=int, default=3)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args(argv)

    import torch

    t0 = time.time()
    prof, tau, healthy = S.generate_trajectories(args.tubes, seed=args.data_seed, length=1024,
                                                 snapshots=args.snapshots)
    torch.cuda.synchronize()
    print(f"trajectories: {args.tubes} tubes, {healthy.sum()} healthy, {time.time() - t0:.1f} s", flush=True)
    sur = S.Surrogate(args.batch, 1024, params=S.init_params(args.init_seed))
    t0 = time.time()
    losses = S.train(sur, prof, tau, healthy, args.steps, args.batch, lr=args.lr, lr_final=0.03 * args.lr,
                     lambda_mass=args.lambda_mass, pushforward=args.pushforward, seed=args.init_seed,
                     push_max=args.push_max, push_start=args.push_start,
                     log_every=max(1, min(args.steps // 10, 20000)),
                     report=lambda it, v: print(f"  step {it:6d}  loss {v:.3e}", flush=True))
    torch.cuda.synchronize()
    train_s = time.time() - t0
    del prof
    params = sur.params().cpu().numpy()
    sur.free()
    ev = S.one_jump_errors(params, count=512, seed=args.heldout_seed)
    print(f"held-out one-jump relative L2: n {ev['n']:.2e}  u {ev['u']:.2e}  "
          f"(persistence u {ev['u_persistence']:.2e}); residual <= 1e-4 for {ev['accept_1e-4']:.2f}", flush=True)
    meta = {"tubes": args.tubes, "snapshots": args.snapshots, "steps": args.steps, "batch": args.batch,
            "lr": args.lr, "lambda_mass": args.lambda_mass, "pushforward": args.pushforward,
            "push_max": args.push_max, "push_start": args.push_start,
            "data_seed": args.data_seed, "init_seed": args.init_seed, "train_seconds": round(train_s, 2),
            "final_loss": losses[-1][1] if losses else None, "heldout": ev}
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, params=params.astype(np.float32), meta=np.array(json.dumps(meta)))
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
