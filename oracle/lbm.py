"""ctypes front end of the FP64 C oracle (TEST INFRASTRUCTURE ONLY).

The model (velocities, weights, polynomial coefficients) comes from
oracle/theory.py; the C library runs the lattice BGK iteration with the tensor
expansion of the equilibrium.  Fields use the layout [Q or D][nz][ny][nx] with x
fastest, as float64 numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build
from .theory import LatticeModel, make_model

MAXQ = 48

PERIODIC = 0
BOUNCE_BACK = 1


class _Model(C.Structure):
    _fields_ = [
        ("D", C.c_int), ("Q", C.c_int),
        ("e", (C.c_int * 3) * MAXQ),
        ("w_hat", C.c_double * MAXQ),
        ("opp", C.c_int * MAXQ),
        ("cvel", C.c_double),
        ("I0", C.c_double), ("J2", C.c_double),
        ("c", C.c_double * 5), ("cp", C.c_double * 5), ("cb", C.c_double * 5),
        ("d4", C.c_double), ("dp4", C.c_double), ("db4", C.c_double),
        ("J4", C.c_double), ("I2", C.c_double),
        ("order", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("bc", C.c_int * 3),
        ("tau", C.c_double),
    ]


_lib = None


def library_path() -> str:
    """The oracle library to load: $LBM_ORACLE_LIBRARY if set (the sanitizer
    test points it at a sanitized build), else the in-tree build."""
    return os.environ.get("LBM_ORACLE_LIBRARY") or _build.LIB


def lib():
    global _lib
    if _lib is None:
        path = library_path()
        if path == _build.LIB and not _build.is_current():
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        mp = C.POINTER(_Model)
        L.orc_feq.argtypes = [mp, C.c_double, dp, dp]
        L.orc_init.argtypes = [mp, dp, dp, dp]
        L.orc_moments.argtypes = [mp, dp, dp, dp]
        L.orc_run.argtypes = [mp, dp, C.c_long]
        L.orc_run_porous.argtypes = [mp, C.c_void_p, dp, dp, C.c_long]
        for f in (L.orc_feq, L.orc_init, L.orc_moments, L.orc_run, L.orc_run_porous):
            f.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One lattice run: a model, a box shape, boundary types and tau."""

    def __init__(self, model: LatticeModel | str = "d2v9", shape=(1, 1, 1), bc=(0, 0, 0),
                 tau: float = 0.6, order: int = 3):
        if isinstance(model, str):
            model = make_model(model)
        self.model = model
        nx, ny, nz = (tuple(shape) + (1, 1, 1))[:3]
        m = _Model()
        m.D, m.Q = model.D, model.Q
        for a in range(model.Q):
            for d in range(3):
                m.e[a][d] = int(model.e[a][d]) if d < model.D else 0
            m.w_hat[a] = float(model.w_hat[a])
            m.opp[a] = int(model.opp[a])
        m.cvel = model.cvel
        m.I0, m.J2 = model.co.I0, model.co.J2
        for K in range(5):
            if K in model.co.c:
                m.c[K], m.cp[K], m.cb[K] = model.co.c[K], model.co.cp[K], model.co.cb[K]
        if model.co.d:
            m.d4, m.dp4, m.db4 = model.co.d["d4"], model.co.d["dp4"], model.co.d["db4"]
            m.J4, m.I2 = model.co.J4, model.co.I[2]
        elif order > 3:
            raise ValueError("order 4 needs the moments through I_8")
        m.order = order
        m.nx, m.ny, m.nz = nx, ny, nz
        for d in range(3):
            m.bc[d] = int(bc[d]) if d < len(bc) else 0
        m.tau = tau
        self._m = m
        self.shape = (nx, ny, nz)
        self.cells = nx * ny * nz

    # -- fields ---------------------------------------------------------------
    def feq(self, n: float, u0) -> np.ndarray:
        u = np.zeros(3)
        u[: self.model.D] = u0
        out = np.zeros(self.model.Q)
        rc = lib().orc_feq(C.byref(self._m), float(n), _dp(u), _dp(out))
        if rc:
            raise ValueError("oracle rejected the model")
        return out

    def init(self, n0: np.ndarray, u0: np.ndarray) -> np.ndarray:
        """Populations at equilibrium with the given density and velocity fields.
        n0: [cells] (any shape with that many elements), u0: [D, cells]."""
        n0 = np.ascontiguousarray(n0, dtype=np.float64).reshape(-1)
        u0 = np.ascontiguousarray(u0, dtype=np.float64).reshape(self.model.D, -1)
        if n0.size != self.cells or u0.shape[1] != self.cells:
            raise ValueError("field sizes do not match the box")
        f = np.empty((self.model.Q, self.cells))
        if lib().orc_init(C.byref(self._m), _dp(n0), _dp(u0), _dp(f)):
            raise ValueError("oracle rejected the model")
        return f

    def run(self, f: np.ndarray, steps: int) -> np.ndarray:
        """Advance populations f ([Q, cells], float64) by `steps` steps, in place."""
        if f.shape != (self.model.Q, self.cells):
            raise ValueError("population array has the wrong shape")
        if lib().orc_run(C.byref(self._m), _dp(f), int(steps)):
            raise ValueError("oracle rejected the run")
        return f

    def run_porous(self, f: np.ndarray, steps: int, solid=None, force=(0.0, 0.0, 0.0)) -> np.ndarray:
        """Advance f by `steps` steps with solid cells (bool/uint8 [cells] or the box
        shape [nz][ny][nx]; None = none) and a constant body force, in place."""
        if f.shape != (self.model.Q, self.cells):
            raise ValueError("population array has the wrong shape")
        F = np.zeros(3)
        F[: len(force)] = force
        sp = None
        if solid is not None:
            mask = np.ascontiguousarray(np.asarray(solid).reshape(-1) != 0, dtype=np.uint8)
            if mask.size != self.cells:
                raise ValueError("solid mask size does not match the box")
            sp = mask.ctypes.data_as(C.c_void_p)
        if lib().orc_run_porous(C.byref(self._m), sp, _dp(F), _dp(f), int(steps)):
            raise ValueError("oracle rejected the run")
        return f

    def moments(self, f: np.ndarray):
        n = np.empty(self.cells)
        u = np.empty((self.model.D, self.cells))
        lib().orc_moments(C.byref(self._m), _dp(f), _dp(n), _dp(u))
        return n, u
