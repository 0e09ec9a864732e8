"""Python binding of the batched tube sweep (the lbm_batch_* entry points of
include/lbm.h): ctypes marshalling only, torch for the workspace and stream."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lbm as _lbm
from .lbm import _check, load


class lbm_tube(C.Structure):
    _fields_ = [("nx", C.c_int), ("tau", C.c_double), ("n_left", C.c_double), ("n_right", C.c_double),
                ("steps", C.c_int64)]


class lbm_batch_options(C.Structure):
    _fields_ = [("weight", C.c_int), ("J2", C.c_double), ("J4", C.c_double), ("order", C.c_int),
                ("precision", C.c_int), ("rho_ref", C.c_double), ("tile_cols", C.c_int), ("halo", C.c_int),
                ("block", C.c_int), ("use_graph", C.c_int), ("fugacity", C.c_double)]


_TP = C.POINTER(lbm_tube)
_OP = C.POINTER(lbm_batch_options)
_lbm.EXTRA_SIGNATURES += [
    ("lbm_batch_workspace_bytes", C.c_int, [_TP, C.c_int, _OP, C.POINTER(C.c_size_t)]),
    ("lbm_batch_init", C.c_int, [_TP, C.c_int, _OP, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("lbm_batch_run", C.c_int, [C.c_void_p]),
    ("lbm_batch_advance", C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    ("lbm_batch_set_equilibrium", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lbm_batch_moments", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lbm_batch_profiles", C.c_int, [C.c_void_p, C.c_void_p]),
    ("lbm_batch_set_profiles", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lbm_batch_health", C.c_int, [C.c_void_p, C.POINTER(C.c_int)]),
    ("lbm_batch_layout", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("lbm_batch_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int),
                                 C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("lbm_batch_free", C.c_int, [C.c_void_p]),
]
if _lbm._lib is not None:  # library already loaded: register the new signatures
    for _name, _res, _args in _lbm.EXTRA_SIGNATURES:
        _fn = getattr(_lbm._lib, _name)
        _fn.restype, _fn.argtypes = _res, _args


def make_tubes(nx, tau, n_left, n_right, steps):
    nx, tau, nl, nr, st = (np.broadcast_to(np.asarray(a), np.shape(nx)) for a in (nx, tau, n_left, n_right, steps))
    arr = (lbm_tube * len(nx))()
    for i in range(len(nx)):
        arr[i].nx, arr[i].tau = int(nx[i]), float(tau[i])
        arr[i].n_left, arr[i].n_right, arr[i].steps = float(nl[i]), float(nr[i]), int(st[i])
    return arr


def make_options(weight=_lbm.LBM_W_FD_T0, order=2, precision=_lbm.LBM_FP32_DEV, rho_ref=1.0, tile_cols=0, halo=0,
                 block=0, use_graph=1, J2=0.0, J4=0.0, fugacity=0.0):
    o = lbm_batch_options()
    o.weight, o.J2, o.J4, o.order, o.precision, o.rho_ref = weight, J2, J4, order, precision, rho_ref
    o.tile_cols, o.halo, o.block, o.use_graph = tile_cols, halo, block, use_graph
    o.fugacity = fugacity
    return o


def lbm_batch_workspace_bytes(tubes, opt) -> int:
    b = C.c_size_t()
    _check(load().lbm_batch_workspace_bytes(tubes, len(tubes), C.byref(opt), C.byref(b)), "lbm_batch_workspace_bytes")
    return b.value


class Batch:
    """A set of tubes with its torch-owned workspace."""

    def __init__(self, tubes, opt, stream=None):
        import torch

        load()
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.tubes, self.opt = tubes, opt
        self.ntubes = len(tubes)
        nbytes = lbm_batch_workspace_bytes(tubes, opt)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        h = C.c_void_p()
        _check(load().lbm_batch_init(tubes, self.ntubes, C.byref(opt), C.c_void_p(self.workspace.data_ptr()), nbytes,
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h)), "lbm_batch_init")
        self.handle = h.value
        off = (C.c_int64 * (self.ntubes + 1))()
        _check(load().lbm_batch_layout(C.c_void_p(self.handle), off), "lbm_batch_layout")
        self.offsets = np.array(off[:], dtype=np.int64)
        self.cells = int(self.offsets[-1])

    def run(self):
        _check(load().lbm_batch_run(C.c_void_p(self.handle)), "lbm_batch_run")

    def advance(self, nsteps: int, active=None):
        mask = None
        if active is not None:
            mask = np.ascontiguousarray(active, dtype=np.uint8)
        _check(load().lbm_batch_advance(C.c_void_p(self.handle), int(nsteps),
                                        None if mask is None else mask.ctypes.data_as(C.c_void_p)),
               "lbm_batch_advance")

    def set_equilibrium(self, n, u, mask=None):
        """n: float64 cuda tensor [cells]; u: [2, cells]."""
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        _check(load().lbm_batch_set_equilibrium(C.c_void_p(self.handle), C.c_void_p(n.data_ptr()),
                                                C.c_void_p(u.data_ptr()),
                                                None if m is None else m.ctypes.data_as(C.c_void_p)),
               "lbm_batch_set_equilibrium")

    def moments(self):
        import torch

        n = torch.empty(self.cells, dtype=torch.float64, device=self.dev)
        u = torch.empty((2, self.cells), dtype=torch.float64, device=self.dev)
        _check(load().lbm_batch_moments(C.c_void_p(self.handle), C.c_void_p(n.data_ptr()), C.c_void_p(u.data_ptr())),
               "lbm_batch_moments")
        return n, u

    def profiles(self, out=None):
        """Row-averaged float32 profiles [ntubes, 2, nx] (n, u_x) of tubes of equal length."""
        import torch

        nx = (int(self.offsets[1]) - int(self.offsets[0])) // 4
        if out is None:
            out = torch.empty((self.ntubes, 2, nx), dtype=torch.float32, device=self.dev)
        _check(load().lbm_batch_profiles(C.c_void_p(self.handle), C.c_void_p(out.data_ptr())), "lbm_batch_profiles")
        return out

    def set_profiles(self, prof, mask=None):
        """Set the masked tubes to f_eq of float32 profiles [ntubes, 2, nx] on every row."""
        m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        _check(load().lbm_batch_set_profiles(C.c_void_p(self.handle), C.c_void_p(prof.data_ptr()),
                                             None if m is None else m.ctypes.data_as(C.c_void_p)),
               "lbm_batch_set_profiles")

    def tube_fields(self, n, u, t):
        """Views of tube t's fields as [4, nx] arrays (numpy or torch)."""
        a, b = int(self.offsets[t]), int(self.offsets[t + 1])
        nx = (b - a) // 4
        return n[a:b].reshape(4, nx), u[:, a:b].reshape(2, 4, nx)

    def health(self):
        out = (C.c_int * self.ntubes)()
        _check(load().lbm_batch_health(C.c_void_p(self.handle), out), "lbm_batch_health")
        return np.array(out[:], dtype=np.int64)

    def info(self):
        cells, upd = C.c_int64(), C.c_int64()
        rounds, S, H = C.c_int(), C.c_int(), C.c_int()
        _check(load().lbm_batch_info(C.c_void_p(self.handle), C.byref(cells), C.byref(upd), C.byref(rounds),
                                     C.byref(S), C.byref(H)), "lbm_batch_info")
        return {"cells": cells.value, "updates_per_run": upd.value, "rounds": rounds.value, "tile_cols": S.value,
                "halo": H.value}

    def free(self):
        if getattr(self, "handle", 0):
            _check(load().lbm_batch_free(C.c_void_p(self.handle)), "lbm_batch_free")
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
