"""Python binding of liblbm.so: ctypes marshalling of the C ABI in include/lbm.h.

Every function named lbm_* here calls the C entry point of the same name and
does nothing but convert arguments; all of the method's arithmetic runs in the
HIP library.  PyTorch supplies device memory (the workspace and the field
buffers) and the stream.  If the library is missing it is built from source
with hipcc, and so is a library built from other sources than those in the
tree; if that fails, loading raises -- there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

from . import build as _build

LBM_D1V3, LBM_D2V9, LBM_D3V19, LBM_D2V41 = 1, 2, 3, 4
LBM_W_MB, LBM_W_FD_T0, LBM_W_CUSTOM, LBM_W_FD, LBM_W_BE, LBM_W_FD_LOCAL = 0, 1, 2, 3, 4, 5
LBM_FP32_DEV, LBM_FP64 = 0, 1
LBM_PERIODIC, LBM_BOUNCEBACK = 0, 1
LBM_SCHEME_PUSH, LBM_SCHEME_AA = 0, 1

STATUS = {0: "LBM_OK", -1: "LBM_ERR_ARG", -2: "LBM_ERR_UNSUPPORTED", -3: "LBM_ERR_HIP",
          -4: "LBM_ERR_NUMERIC", -5: "LBM_ERR_STATE"}

DIM = {LBM_D1V3: 1, LBM_D2V9: 2, LBM_D3V19: 3, LBM_D2V41: 2}
LATTICE_BY_NAME = {"d1v3": LBM_D1V3, "d2v9": LBM_D2V9, "d3v19": LBM_D3V19, "d2v41": LBM_D2V41}


class LbmError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class lbm_config(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("bc", C.c_int * 3), ("weight", C.c_int), ("J2", C.c_double), ("J4", C.c_double),
        ("order", C.c_int), ("tau", C.c_double), ("precision", C.c_int), ("rho_ref", C.c_double),
        ("scheme", C.c_int), ("block", C.c_int), ("graph_steps", C.c_int),
        ("obstacles", C.c_int), ("force", C.c_double * 3), ("fugacity", C.c_double),
        ("theta_over_mu", C.c_double),
    ]


_lib = None

# (name, restype, argtypes) of every entry point the header declares
_SIGNATURES = [
    ("lbm_coefficients", C.c_int, [C.POINTER(lbm_config), C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]),
    ("lbm_workspace_bytes", C.c_int, [C.POINTER(lbm_config), C.POINTER(C.c_size_t)]),
    ("lbm_init", C.c_int, [C.POINTER(lbm_config), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.POINTER(C.c_void_p)]),
    ("lbm_step", C.c_int, [C.c_void_p, C.c_int64]),
    ("lbm_moments", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lbm_moments_device", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("lbm_totals", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("lbm_get_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("lbm_set_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    ("lbm_steps_done", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("lbm_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int64)]),
    ("lbm_velocities", C.c_int, [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)]),
    ("lbm_set_solid", C.c_int, [C.c_void_p, C.c_void_p]),
    ("lbm_free", C.c_int, [C.c_void_p]),
    ("lbm_last_error", C.c_char_p, []),
]

EXTRA_SIGNATURES = []  # appended by the batched and surrogate bindings


def library_path() -> str:
    """The library to load: $LBM_LIBRARY if set (the sanitizer test points it at
    a build whose host code runs under the sanitizers), else the in-tree build."""
    return os.environ.get("LBM_LIBRARY") or _build.LIB


def load():
    """Load liblbm.so, building it first if it is missing or was built from
    sources other than those in the tree (digest stored beside the library)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if path == _build.LIB and not _build.is_current():
        _build.build()
    # torch (which owns the device memory and streams) loads its own copy of the
    # HIP runtime; importing it first makes the library bind to that same copy
    # (one runtime per process) instead of loading a second one
    import torch  # noqa: F401

    lib = C.CDLL(path)
    for name, res, args in _SIGNATURES + EXTRA_SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        raise LbmError(status, where, load().lbm_last_error().decode())


def make_config(lattice="d2v9", shape=(64, 64, 1), bc=(0, 0, 0), weight=LBM_W_FD_T0, order=3, tau=0.6,
                precision=LBM_FP32_DEV, rho_ref=1.0, scheme=LBM_SCHEME_PUSH, block=0, graph_steps=0,
                J2=0.0, J4=0.0, obstacles=0, force=(0.0, 0.0, 0.0), fugacity=0.0,
                theta_over_mu=0.0) -> lbm_config:
    if isinstance(lattice, str):
        lattice = LATTICE_BY_NAME[lattice]
    nx, ny, nz = (tuple(shape) + (1, 1, 1))[:3]
    cfg = lbm_config()
    cfg.lattice, cfg.nx, cfg.ny, cfg.nz = lattice, nx, ny, nz
    for d in range(3):
        cfg.bc[d] = int(bc[d]) if d < len(bc) else 0
    cfg.weight, cfg.J2, cfg.J4 = weight, J2, J4
    cfg.order, cfg.tau, cfg.precision, cfg.rho_ref = order, tau, precision, rho_ref
    cfg.scheme, cfg.block, cfg.graph_steps = scheme, block, graph_steps
    cfg.obstacles = int(obstacles)
    cfg.fugacity = float(fugacity)
    cfg.theta_over_mu = float(theta_over_mu)
    for d in range(3):
        cfg.force[d] = float(force[d]) if d < len(force) else 0.0
    return cfg


# -- thin wrappers with the C names ------------------------------------------

def lbm_coefficients(cfg: lbm_config):
    out = (C.c_double * 96)()
    n = C.c_int()
    _check(load().lbm_coefficients(C.byref(cfg), out, 96, C.byref(n)), "lbm_coefficients")
    return list(out[: n.value])


def lbm_workspace_bytes(cfg: lbm_config) -> int:
    b = C.c_size_t()
    _check(load().lbm_workspace_bytes(C.byref(cfg), C.byref(b)), "lbm_workspace_bytes")
    return b.value


def lbm_init(cfg, workspace_ptr: int, nbytes: int, stream: int, n0_ptr: int, u0_ptr: int) -> int:
    ctx = C.c_void_p()
    _check(load().lbm_init(C.byref(cfg), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream),
                           C.c_void_p(n0_ptr), C.c_void_p(u0_ptr), C.byref(ctx)), "lbm_init")
    return ctx.value


def lbm_step(ctx: int, nsteps: int):
    _check(load().lbm_step(C.c_void_p(ctx), int(nsteps)), "lbm_step")


def lbm_moments(ctx: int, n_host_ptr: int, u_host_ptr: int):
    _check(load().lbm_moments(C.c_void_p(ctx), C.c_void_p(n_host_ptr), C.c_void_p(u_host_ptr)), "lbm_moments")


def lbm_moments_device(ctx: int, n_dev_ptr: int, u_dev_ptr: int):
    _check(load().lbm_moments_device(C.c_void_p(ctx), C.c_void_p(n_dev_ptr), C.c_void_p(u_dev_ptr)),
           "lbm_moments_device")


def lbm_totals(ctx: int, D: int):
    out = (C.c_double * 4)()
    _check(load().lbm_totals(C.c_void_p(ctx), out), "lbm_totals")
    return list(out[: D + 1])


def lbm_get_state(ctx: int, host_ptr: int, nbytes: int):
    _check(load().lbm_get_state(C.c_void_p(ctx), C.c_void_p(host_ptr), nbytes), "lbm_get_state")


def lbm_set_state(ctx: int, host_ptr: int, nbytes: int):
    _check(load().lbm_set_state(C.c_void_p(ctx), C.c_void_p(host_ptr), nbytes), "lbm_set_state")


def lbm_steps_done(ctx: int) -> int:
    s = C.c_int64()
    _check(load().lbm_steps_done(C.c_void_p(ctx), C.byref(s)), "lbm_steps_done")
    return s.value


def lbm_info(ctx: int):
    cells, Q, b = C.c_int64(), C.c_int(), C.c_int64()
    _check(load().lbm_info(C.c_void_p(ctx), C.byref(cells), C.byref(Q), C.byref(b)), "lbm_info")
    return cells.value, Q.value, b.value


def lbm_velocities(lattice) -> list:
    if isinstance(lattice, str):
        lattice = LATTICE_BY_NAME[lattice]
    e = (C.c_int * 144)()
    Q = C.c_int()
    _check(load().lbm_velocities(lattice, e, 144, C.byref(Q)), "lbm_velocities")
    return [tuple(e[3 * a: 3 * a + 3]) for a in range(Q.value)]


def lbm_set_solid(ctx: int, solid_ptr: int):
    _check(load().lbm_set_solid(C.c_void_p(ctx), C.c_void_p(solid_ptr)), "lbm_set_solid")


def lbm_free(ctx: int):
    _check(load().lbm_free(C.c_void_p(ctx)), "lbm_free")


# -- a context holding its torch-owned buffers --------------------------------

@dataclass
class Lattice:
    """One run: the configuration, the torch-allocated workspace and the context.

    n0 and u0 are float64 torch tensors (any device; copied to the GPU), shaped
    [cells] / [D, cells] or anything with that many elements."""

    cfg: lbm_config
    ctx: int = 0

    @classmethod
    def create(cls, cfg: lbm_config, n0, u0, stream=None):
        import torch

        dev = torch.device("cuda", torch.cuda.current_device())
        D = DIM[cfg.lattice]
        cells = cfg.nx * cfg.ny * cfg.nz
        n0 = torch.as_tensor(n0, dtype=torch.float64).reshape(-1).to(dev).contiguous()
        u0 = torch.as_tensor(u0, dtype=torch.float64).reshape(D, -1).to(dev).contiguous()
        if n0.numel() != cells or u0.shape[1] != cells:
            raise ValueError("field sizes do not match the box")
        nbytes = lbm_workspace_bytes(cfg)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        self = cls(cfg)
        self.workspace, self.stream, self.D, self.cells = ws, s, D, cells
        self.ctx = lbm_init(cfg, ws.data_ptr(), nbytes, s.cuda_stream, n0.data_ptr(), u0.data_ptr())
        self._keep = (n0, u0)
        return self

    def step(self, nsteps: int):
        lbm_step(self.ctx, nsteps)

    def moments(self):
        """Float64 device tensors n [cells] and u0 [D, cells] (lbm_moments_device;
        asynchronous on the context's stream)."""
        import torch

        n = torch.empty(self.cells, dtype=torch.float64, device=self.workspace.device)
        u = torch.empty((self.D, self.cells), dtype=torch.float64, device=self.workspace.device)
        lbm_moments_device(self.ctx, n.data_ptr(), u.data_ptr())
        return n, u

    def moments_host(self):
        """Float64 numpy arrays n [cells] and u0 [D, cells] (lbm_moments; synchronous)."""
        import numpy as np

        n = np.empty(self.cells, dtype=np.float64)
        u = np.empty((self.D, self.cells), dtype=np.float64)
        lbm_moments(self.ctx, n.ctypes.data, u.ctypes.data)
        return n, u

    def totals(self):
        return lbm_totals(self.ctx, self.D)

    def state(self):
        """Stored populations g = f - w rho_ref at their natural slots."""
        import numpy as np

        cells, Q, _ = lbm_info(self.ctx)
        dt = np.float64 if self.cfg.precision == LBM_FP64 else np.float32
        a = np.empty((Q, cells), dtype=dt)
        lbm_get_state(self.ctx, a.ctypes.data, a.nbytes)
        return a

    def set_state(self, a):
        import numpy as np

        dt = np.float64 if self.cfg.precision == LBM_FP64 else np.float32
        a = np.ascontiguousarray(a, dtype=dt)
        lbm_set_state(self.ctx, a.ctypes.data, a.nbytes)

    def set_solid(self, solid):
        """Mark solid cells (any array of cells elements, nonzero = solid)."""
        import torch

        m = torch.as_tensor(solid).reshape(-1).ne(0).to(torch.uint8).to(self.workspace.device).contiguous()
        if m.numel() != self.cells:
            raise ValueError("solid mask size does not match the box")
        lbm_set_solid(self.ctx, m.data_ptr())
        self._solid = m  # kept until the stream has read it

    @property
    def steps_done(self) -> int:
        return lbm_steps_done(self.ctx)

    def free(self):
        if self.ctx:
            lbm_free(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
