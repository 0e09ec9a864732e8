"""Python binding of the convolutional surrogate (the srg_* entry points of
include/srg.h): ctypes marshalling, plus the host-side driver of training
(data generation by the batched lattice sweep, minibatch sampling, the
optimisation loop) and of the hybrid advance.  Every forward, backward, loss,
optimiser and lattice step runs in the HIP library."""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import time

import numpy as np

from . import batch as _batch
from . import inputs
from . import lbm as _lbm
from .lbm import _check, load

_F = C.c_float
_lbm.EXTRA_SIGNATURES += [
    ("srg_param_count", C.c_int, [C.POINTER(C.c_int64)]),
    ("srg_workspace_bytes", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    ("srg_create", C.c_int, [C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("srg_set_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("srg_get_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("srg_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("srg_infer", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("srg_backward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("srg_loss", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, _F, C.c_void_p, C.POINTER(C.c_double)]),
    ("srg_adam", C.c_int, [C.c_void_p, C.c_void_p, _F, _F, _F, _F]),
    ("srg_train_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, _F, _F,
                                 C.POINTER(C.c_double)]),
    ("srg_mass_residual", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    ("srg_hybrid_advance", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, _F,
                                     C.POINTER(C.c_int)]),
    ("srg_free", C.c_int, [C.c_void_p]),
    ("srg_infer_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
]
if _lbm._lib is not None:  # library already loaded: register the new signatures
    for _name, _res, _args in _lbm.EXTRA_SIGNATURES:
        _fn = getattr(_lbm._lib, _name)
        _fn.restype, _fn.argtypes = _res, _args

JUMP_STEPS = 64
MASS_TOL = 1e-4
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "srg_d2v9_L1024_j64.npz")


def _p(t):
    return C.c_void_p(t.data_ptr())


def srg_param_count() -> int:
    n = C.c_int64()
    _check(load().srg_param_count(C.byref(n)), "srg_param_count")
    return n.value


def srg_workspace_bytes(max_batch: int, length: int) -> int:
    b = C.c_size_t()
    _check(load().srg_workspace_bytes(int(max_batch), int(length), C.byref(b)), "srg_workspace_bytes")
    return b.value


def srg_infer_noalloc(params, prof, tau, out, stream=None):
    """Inference with no context and no allocation in the library (srg_infer_noalloc):
    params float32 [srg_param_count], prof and out float32 [batch, 2, L], tau float32
    [batch], all cuda tensors; enqueued on `stream` (torch's current stream if None)."""
    import torch

    B, two, L = prof.shape
    if two != 2 or tuple(out.shape) != tuple(prof.shape) or tau.numel() != B:
        raise ValueError("prof and out must be [batch, 2, L] and tau [batch]")
    s = stream if stream is not None else torch.cuda.current_stream(prof.device)
    _check(load().srg_infer_noalloc(_p(params), _p(prof), _p(tau), int(B), int(L), _p(out),
                                    C.c_void_p(s.cuda_stream)), "srg_infer_noalloc")
    return out


class Surrogate:
    """A surrogate context with its torch-owned workspace.  Profiles are float32
    cuda tensors [batch, 2, L] (n, u_x); tau is float32 [batch]."""

    def __init__(self, max_batch: int, length: int, params=None, stream=None):
        import torch

        load()
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.max_batch, self.L = int(max_batch), int(length)
        nbytes = srg_workspace_bytes(self.max_batch, self.L)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        h = C.c_void_p()
        _check(load().srg_create(self.max_batch, self.L, _p(self.workspace), nbytes, C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h)), "srg_create")
        self.handle = h.value
        self.nparam = srg_param_count()
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        import torch

        p = torch.as_tensor(np.asarray(params, dtype=np.float32) if not torch.is_tensor(params) else params)
        p = p.to(self.dev, torch.float32).contiguous()
        if p.numel() != self.nparam:
            raise ValueError(f"expected {self.nparam} parameters")
        _check(load().srg_set_params(C.c_void_p(self.handle), _p(p)), "srg_set_params")

    def params(self):
        import torch

        out = torch.empty(self.nparam, dtype=torch.float32, device=self.dev)
        _check(load().srg_get_params(C.c_void_p(self.handle), _p(out)), "srg_get_params")
        return out

    def forward(self, prof, tau, out=None):
        import torch

        B = prof.shape[0]
        if out is None:
            out = torch.empty_like(prof)
        _check(load().srg_forward(C.c_void_p(self.handle), _p(prof), _p(tau), B, _p(out)), "srg_forward")
        return out

    def infer(self, prof, tau, out=None):
        """The forward pass in one fused kernel (the same values as forward();
        nothing is kept for backward())."""
        import torch

        B = prof.shape[0]
        if out is None:
            out = torch.empty_like(prof)
        _check(load().srg_infer(C.c_void_p(self.handle), _p(prof), _p(tau), B, _p(out)), "srg_infer")
        return out

    def backward(self, dout):
        import torch

        g = torch.empty(self.nparam, dtype=torch.float32, device=self.dev)
        _check(load().srg_backward(C.c_void_p(self.handle), _p(dout), _p(g)), "srg_backward")
        return g

    def loss(self, out, target, lambda_mass=0.0):
        import torch

        dout = torch.empty_like(out)
        val = C.c_double()
        _check(load().srg_loss(C.c_void_p(self.handle), _p(out), _p(target), out.shape[0], float(lambda_mass),
                               _p(dout), C.byref(val)), "srg_loss")
        return val.value, dout

    def adam(self, grad, lr, b1=0.9, b2=0.999, eps=1e-8):
        _check(load().srg_adam(C.c_void_p(self.handle), _p(grad), float(lr), float(b1), float(b2), float(eps)),
               "srg_adam")

    def train_step(self, prof, tau, target, lr, lambda_mass=0.0, want_loss=True):
        val = C.c_double()
        _check(load().srg_train_step(C.c_void_p(self.handle), _p(prof), _p(tau), _p(target), prof.shape[0],
                                     float(lr), float(lambda_mass), C.byref(val) if want_loss else None),
               "srg_train_step")
        return val.value if want_loss else None

    def mass_residual(self, prof_in, prof_out):
        import torch

        r = torch.empty(prof_in.shape[0], dtype=torch.float32, device=self.dev)
        _check(load().srg_mass_residual(C.c_void_p(self.handle), _p(prof_in), _p(prof_out), prof_in.shape[0], _p(r)),
               "srg_mass_residual")
        return r

    def hybrid_advance(self, b: "_batch.Batch", tau, jumps: int, jump_steps: int = JUMP_STEPS,
                       mass_tol: float = MASS_TOL):
        """Advance the tube batch b by `jumps` coarse jumps; returns the number of
        fallback tubes per jump."""
        nf = (C.c_int * max(1, jumps))()
        _check(load().srg_hybrid_advance(C.c_void_p(self.handle), C.c_void_p(b.handle), _p(tau), b.ntubes, int(jumps),
                                         int(jump_steps), float(mass_tol), nf), "srg_hybrid_advance")
        return np.array(nf[:jumps], dtype=np.int64)

    def free(self):
        if getattr(self, "handle", 0):
            _check(load().srg_free(C.c_void_p(self.handle)), "srg_free")
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# -- training data: trajectories of the batched lattice sweep ------------------

def trajectory_tubes(count: int, seed: int, length: int = 1024, ratio_range=(0.5, 0.95), tau_range=(0.51, 1.0)):
    """Shock tubes of one length with n_R/n_L and tau drawn uniformly."""
    d = inputs.tube_draws(count, seed, nx_range=(length, length), ratio_range=ratio_range, tau_range=tau_range)
    return d


def generate_trajectories(count: int, seed: int, length: int = 1024, snapshots: int = 64,
                          jump_steps: int = JUMP_STEPS, chunk: int = 4096, ratio_range=(0.5, 0.95),
                          tau_range=(0.51, 1.0)):
    """Run `count` shock tubes of `length` x 4 cells (float32 deviation storage,
    second-order equilibrium) and keep the profiles every jump_steps steps.

    Returns (prof [snapshots + 1, count, 2, L] float32 cuda, tau [count] float32
    cuda, healthy [count] bool numpy)."""
    import torch

    d = trajectory_tubes(count, seed, length, ratio_range, tau_range)
    dev = torch.device("cuda", torch.cuda.current_device())
    prof = torch.empty((snapshots + 1, count, 2, length), dtype=torch.float32, device=dev)
    healthy = np.ones(count, dtype=bool)
    for a in range(0, count, chunk):
        b = min(count, a + chunk)
        tubes = _batch.make_tubes(d["nx"][a:b], d["tau"][a:b], d["n_left"][a:b], d["n_right"][a:b], 0)
        bt = _batch.Batch(tubes, _batch.make_options())
        try:
            for s in range(snapshots + 1):
                if s:
                    bt.advance(jump_steps)
                bt.profiles(out=prof[s, a:b])
            healthy[a:b] = bt.health() == 0
        finally:
            bt.free()
    tau = torch.as_tensor(d["tau"], dtype=torch.float32).to(dev)
    return prof, tau, healthy


def train(sur: Surrogate, prof, tau, healthy, steps: int, batch: int, lr: float = 1e-3, lr_final: float = 3e-5,
          lambda_mass: float = 1.0, pushforward: float = 0.0, seed: int = 0, log_every: int = 0, report=None,
          push_max: int = 1, push_start: float = 0.5):
    """Adam on random (trajectory, snapshot) pairs: input snapshot s, target s + 1.

    With probability `pushforward` (from the fraction push_start of the steps
    on) a step instead takes the network's own prediction k jumps on from
    snapshot s as its input (k drawn uniformly from 1 .. push_max, the jumps
    made by the network without gradient) and snapshot s + k + 1 as its
    target, so that it learns to correct the errors of its own rollouts.  The
    learning rate decays by cosine from lr to lr_final.  Returns the losses at
    the logged steps; report(step, loss) is called at each of them when given."""
    import torch

    rng = np.random.default_rng(seed)
    good = np.flatnonzero(healthy)
    S = prof.shape[0] - 1
    losses = []
    pred = None
    for it in range(steps):
        ti = torch.as_tensor(rng.choice(good, batch), device=prof.device)
        t = tau[ti].contiguous()
        push = pushforward > 0 and it >= int(push_start * steps) and rng.random() < pushforward
        if push:
            k = int(rng.integers(1, push_max + 1))
            si = torch.as_tensor(rng.integers(0, S - k, batch), device=prof.device)
            if pred is None or pred.shape[0] != batch:
                pred = torch.empty((2, batch, 2, prof.shape[3]), dtype=torch.float32, device=prof.device)
            x = prof[si, ti].contiguous()
            for j in range(k):
                x = sur.infer(x, t, out=pred[j % 2])
            y = prof[si + k + 1, ti].contiguous()
        else:
            si = torch.as_tensor(rng.integers(0, S, batch), device=prof.device)
            x = prof[si, ti].contiguous()
            y = prof[si + 1, ti].contiguous()
        frac = it / max(1, steps - 1)
        rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
        want = bool(log_every) and (it % log_every == 0 or it == steps - 1)
        v = sur.train_step(x, t, y, rate, lambda_mass, want_loss=want)
        if want:
            losses.append((it, v))
            if report is not None:
                report(it, v)
    return losses


def init_params(seed: int = 0, scale_out: float = 0.1):
    """He-normal initial parameters (std sqrt(2 / fan_in)), zero biases, the last
    layer scaled by scale_out so the untrained network starts near the identity."""
    rng = np.random.default_rng(seed)
    shapes = [((5, 64, 3), 64), ((5, 64, 64), 64), ((5, 64, 64), 64), ((5, 2, 64), 2)]
    out = []
    for i, (ws, nb) in enumerate(shapes):
        w = rng.standard_normal(ws) * math.sqrt(2.0 / (ws[0] * ws[2]))
        if i == 3:
            w *= scale_out
        out += [w.reshape(-1), np.zeros(nb)]
    return np.concatenate(out).astype(np.float32)



def load_weights(path: str = WEIGHTS):
    """(float32 parameter vector, metadata dict) of a file written by train_surrogate."""
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


def one_jump_errors(params, count: int = 512, seed: int = 3, snapshots: int = 16):
    """Relative L2 error of single jumps over held-out trajectories (every
    snapshot s -> s + 1 of `count` tubes), next to the error of persistence
    (predicting no change), and the fraction of jumps whose mass residual is
    within MASS_TOL."""
    import torch

    hp, htau, _ = generate_trajectories(count, seed=seed, length=1024, snapshots=snapshots)
    sur = Surrogate(count, 1024, params=params)
    dn = dd = du = dp = duu = 0.0
    acc = 0
    for s in range(snapshots):
        x, y = hp[s].contiguous(), hp[s + 1]
        out = sur.forward(x, htau)
        acc += int((sur.mass_residual(x, out) <= MASS_TOL).sum())
        e = (out - y).double()
        dn += float((e[:, 0] ** 2).sum())
        dd += float((y[:, 0].double() ** 2).sum())
        du += float((e[:, 1] ** 2).sum())
        duu += float((y[:, 1].double() ** 2).sum())
        dp += float(((x[:, 1] - y[:, 1]).double() ** 2).sum())
    torch.cuda.synchronize()
    sur.free()
    return {"n": math.sqrt(dn / dd), "u": math.sqrt(du / duu), "u_persistence": math.sqrt(dp / duu),
            "accept_1e-4": acc / (count * snapshots), "count": count, "seed": seed}


def hybrid_run(params, count: int = 512, seed: int = 3, jumps: int = 16, jump_steps: int = JUMP_STEPS,
               mass_tol: float = MASS_TOL, repeats: int = 1):
    """The surrogate-accelerated batched run next to the plain batched sweep on
    the same held-out tubes (length 1024, n_L = 1, seeded n_R / n_L and tau).

    Both start from the tubes' initial step; the plain sweep advances
    jumps * jump_steps steps, the hybrid makes `jumps` surrogate jumps with the
    lattice fallback.  Returns timings (best of `repeats`, GPU work bracketed by
    device synchronisation), the fallback fraction, the per-tube relative L2
    errors of n and u against the plain sweep (mean and max), and the number of
    broken-down tubes of each run."""
    import torch

    d = trajectory_tubes(count, seed, 1024)
    tubes = _batch.make_tubes(d["nx"], d["tau"], d["n_left"], d["n_right"], 0)
    tau = torch.as_tensor(d["tau"], dtype=torch.float32).cuda()
    sur = Surrogate(count, 1024, params=params)
    t_plain = t_hyb = float("inf")
    for _ in range(repeats):
        bp = _batch.Batch(tubes, _batch.make_options())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bp.advance(jumps * jump_steps)
        torch.cuda.synchronize()
        t_plain = min(t_plain, time.perf_counter() - t0)
        ref = bp.profiles().double()
        broken_plain = int((bp.health() != 0).sum())
        bp.free()
        bh = _batch.Batch(tubes, _batch.make_options())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nf = sur.hybrid_advance(bh, tau, jumps, jump_steps, mass_tol)
        torch.cuda.synchronize()
        t_hyb = min(t_hyb, time.perf_counter() - t0)
        p = bh.profiles().double()
        broken = int((bh.health() != 0).sum())
        bh.free()
    sur.free()
    en = ((p[:, 0] - ref[:, 0]).norm(dim=1) / ref[:, 0].norm(dim=1)).cpu().numpy()
    eu = ((p[:, 1] - ref[:, 1]).norm(dim=1) / ref[:, 1].norm(dim=1)).cpu().numpy()
    return {"tubes": count, "jumps": jumps, "jump_steps": jump_steps, "mass_tol": mass_tol,
            "ms_plain": t_plain * 1e3, "ms_hybrid": t_hyb * 1e3, "speedup": t_plain / t_hyb,
            "fallback_fraction": float(nf.sum()) / (count * jumps),
            "rel_l2_n_mean": float(np.nanmean(en)), "rel_l2_n_max": float(np.max(en)),
            "rel_l2_u_mean": float(np.nanmean(eu)), "rel_l2_u_max": float(np.max(eu)),
            "broken_hybrid": broken, "broken_plain": broken_plain}
