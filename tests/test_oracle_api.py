"""The lbm_* call surface of the CPU oracle library (oracle/lbm_oracle_api.c),
on the CPU: its configuration record has the library's layout, its lattice
model equals the Python oracle's (built independently from the same formulas),
its runs equal the oracle's, and the calling conventions hold without a GPU --
argument errors, checkpoint and restore bit for bit, and fault injection
through lbm_set_state (a NaN or a negative density makes lbm_totals return
LBM_ERR_NUMERIC)."""
import ctypes as C

import numpy as np
import pytest

from oracle import lbm as OL
from oracle import theory as th
from paper_1510_07328_amd import inputs
from paper_1510_07328_amd.lbm import lbm_config, make_config

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_NUMERIC = 0, -1, -2, -4
FP32, FP64 = 0, 1


def lib():
    OL.lib()  # builds the library if it is missing or stale
    L = C.CDLL(OL.library_path())
    vp, dp, cp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(lbm_config)
    sig = {
        "lbm_workspace_bytes": [cp, C.POINTER(C.c_size_t)],
        "lbm_init": [cp, vp, C.c_size_t, vp, vp, vp, C.POINTER(vp)],
        "lbm_step": [vp, C.c_int64],
        "lbm_moments": [vp, vp, vp],
        "lbm_moments_device": [vp, vp, vp],
        "lbm_totals": [vp, dp],
        "lbm_get_state": [vp, vp, C.c_size_t],
        "lbm_set_state": [vp, vp, C.c_size_t],
        "lbm_steps_done": [vp, C.POINTER(C.c_int64)],
        "lbm_info": [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int64)],
        "lbm_velocities": [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int)],
        "lbm_free": [vp],
        "orc_api_model": [cp, C.POINTER(OL._Model)],
        "orc_api_config_offset": [C.c_int],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.orc_api_config_size.restype = C.c_size_t
    L.orc_api_config_offset.restype = C.c_size_t
    L.lbm_last_error.restype = C.c_char_p
    return L


class Run:
    """One context over host memory."""

    def __init__(self, cfg, n0, u0):
        self.L = lib()
        b = C.c_size_t()
        assert self.L.lbm_workspace_bytes(C.byref(cfg), C.byref(b)) == OK
        self.ws = np.zeros(b.value // 8, dtype=np.float64)
        self.n0 = np.ascontiguousarray(n0, dtype=np.float64)
        self.u0 = np.ascontiguousarray(u0, dtype=np.float64)
        h = C.c_void_p()
        rc = self.L.lbm_init(C.byref(cfg), self.ws.ctypes.data, b.value, None, self.n0.ctypes.data,
                             self.u0.ctypes.data, C.byref(h))
        assert rc == OK, self.L.lbm_last_error()
        self.h = h
        cells, Q, bps = C.c_int64(), C.c_int(), C.c_int64()
        assert self.L.lbm_info(h, C.byref(cells), C.byref(Q), C.byref(bps)) == OK
        self.cells, self.Q = cells.value, Q.value
        self.D = {1: 1, 2: 2, 3: 3}[cfg.lattice]

    def step(self, n):
        assert self.L.lbm_step(self.h, n) == OK

    def moments(self):
        n = np.empty(self.cells)
        u = np.empty((self.D, self.cells))
        assert self.L.lbm_moments(self.h, n.ctypes.data, u.ctypes.data) == OK
        return n, u

    def state(self):
        g = np.empty((self.Q, self.cells))
        assert self.L.lbm_get_state(self.h, g.ctypes.data, g.nbytes) == OK
        return g

    def set_state(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        return self.L.lbm_set_state(self.h, g.ctypes.data, g.nbytes)

    def totals(self):
        out = (C.c_double * 4)()
        rc = self.L.lbm_totals(self.h, out)
        return rc, list(out[: self.D + 1])

    def free(self):
        self.L.lbm_free(self.h)


def test_config_record_has_the_library_layout():
    L = lib()
    assert L.orc_api_config_size() == C.sizeof(lbm_config)
    for i, name in enumerate(("lattice", "bc", "J2", "tau", "rho_ref", "force", "theta_over_mu")):
        assert L.orc_api_config_offset(i) == getattr(lbm_config, name).offset, name


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("weight", [0, 1, 2])
def test_model_equals_the_python_oracle(lat, weight):
    L = lib()
    D = th.lattice_dim(lat)
    cfg = make_config(lat, shape=(8, 1 if D < 2 else 6, 1 if D < 3 else 5), order=3, tau=0.7, precision=FP64,
                      weight=weight, J2=1.2, J4=1.3)
    m = OL._Model()
    assert L.orc_api_model(C.byref(cfg), C.byref(m)) == OK
    if weight == 0:
        ref = th.make_model(lat, th.MB, theta=1.0 / 3.0)
    elif weight == 1:
        ref = th.make_model(lat)
    else:  # moments with J_2 = 1.2, J_4 = 1.3
        ref = th.model_from_moments(lat, {0: 1.0, 2: 1.0, 4: 1.0 / 1.2, 6: (1.0 / 1.2) ** 2 / 1.3, 8: 1.0})
    assert m.Q == ref.Q and m.D == ref.D
    e = np.array([[m.e[a][d] for d in range(D)] for a in range(m.Q)])
    np.testing.assert_array_equal(e, ref.e)
    np.testing.assert_array_equal([m.opp[a] for a in range(m.Q)], ref.opp)
    np.testing.assert_allclose([m.w_hat[a] for a in range(m.Q)], ref.w_hat, rtol=1e-14, atol=1e-15)
    assert m.cvel == pytest.approx(ref.cvel, rel=1e-14)
    assert m.J2 == pytest.approx(ref.co.J2, rel=1e-14)
    for K in range(4):
        assert m.c[K] == pytest.approx(ref.co.c[K], rel=1e-14)
        assert m.cp[K] == pytest.approx(ref.co.cp[K], rel=1e-14, abs=1e-15)
        assert m.cb[K] == pytest.approx(ref.co.cb[K], rel=1e-14, abs=1e-15)


def test_velocity_order_is_the_oracles():
    L = lib()
    for code, lat in ((1, "d1v3"), (2, "d2v9"), (3, "d3v19")):
        e = (C.c_int * 144)()
        Q = C.c_int()
        assert L.lbm_velocities(code, e, 144, C.byref(Q)) == OK
        D = th.lattice_dim(lat)
        got = np.array([[e[3 * a + d] for d in range(D)] for a in range(Q.value)])
        np.testing.assert_array_equal(got, th.velocity_set(lat))


@pytest.mark.parametrize("lat,shape,bc", [("d2v9", (24, 10, 1), (1, 0, 0)), ("d3v19", (8, 7, 6), (0, 1, 0)),
                                          ("d1v3", (50, 1, 1), (1, 0, 0))])
def test_runs_equal_the_oracle(lat, shape, bc):
    D = th.lattice_dim(lat)
    cfg = make_config(lat, shape=shape, bc=bc, order=2, tau=0.6, precision=FP64)
    grid = tuple(reversed(shape[:D]))
    n0, u0 = inputs.perturbed_field(grid, 0.02, 3.0, (0.01,) + (0.0,) * (D - 1), seed=3)
    r = Run(cfg, n0, u0)
    r.step(17)
    n, u = r.moments()
    r.free()
    o = OL.Oracle(lat, shape=shape, bc=bc, tau=0.6, order=2)
    f = o.init(n0, u0)
    o.run(f, 17)
    n_o, u_o = o.moments(f)
    # the two models differ in the last bits of their weights (closed form here,
    # a least-squares solve of the moment conditions in the Python oracle)
    assert np.abs(n - n_o).max() / np.abs(n_o).max() < 1e-13
    assert np.abs(u - u_o).max() / np.abs(u_o).max() < 1e-13


def test_checkpoint_restores_bit_for_bit():
    cfg = make_config("d2v9", shape=(20, 12, 1), bc=(1, 0, 0), order=3, tau=0.65, precision=FP64)
    n0, u0 = inputs.riemann_step(20, 12, 1.0, 0.8)
    a = Run(cfg, n0, u0)
    a.step(30)
    snap = a.state()
    steps = C.c_int64()
    assert a.L.lbm_steps_done(a.h, C.byref(steps)) == OK and steps.value == 30
    a.step(30)
    want = a.state()
    b = Run(cfg, np.ones(240), np.zeros((2, 240)))
    assert b.set_state(snap) == OK
    b.step(30)
    np.testing.assert_array_equal(b.state(), want)
    a.free()
    b.free()


@pytest.mark.parametrize("poison", ["nan", "negative_density", "inf"])
def test_fault_injection_through_set_state_is_a_numeric_error(poison):
    cfg = make_config("d2v9", shape=(16, 8, 1), order=2, tau=0.7, precision=FP64)
    n0, u0 = inputs.perturbed_field((8, 16), 0.01, 3.0, (0.0, 0.0), seed=1)
    r = Run(cfg, n0, u0)
    rc, _ = r.totals()
    assert rc == OK
    g = r.state()
    if poison == "nan":
        g[3, 77] = np.nan
    elif poison == "inf":
        g[5, 0] = np.inf
    else:
        g[:, 40] = -1.0  # n = rho_ref + sum g < 0 in that cell
    assert r.set_state(g) == OK
    rc, _ = r.totals()
    assert rc == ERR_NUMERIC
    assert b"non" in r.L.lbm_last_error()
    r.free()


def test_argument_errors():
    L = lib()
    b = C.c_size_t()
    good = make_config("d2v9", shape=(16, 8, 1), order=2, tau=0.7, precision=FP64)
    assert L.lbm_workspace_bytes(C.byref(good), C.byref(b)) == OK and b.value == 9 * 128 * 8
    for kw, want in (({"tau": 0.5}, ERR_ARG), ({"precision": FP32}, ERR_UNSUPPORTED), ({"order": 4}, ERR_ARG),
                     ({"lattice": "d2v41"}, ERR_UNSUPPORTED), ({"weight": 5}, ERR_UNSUPPORTED),
                     ({"shape": (16, 8, 2)}, ERR_ARG), ({"force": (1e-5, 0.0, 0.0)}, ERR_UNSUPPORTED)):
        args = dict(lattice="d2v9", shape=(16, 8, 1), order=2, tau=0.7, precision=FP64)
        args.update(kw)
        cfg = make_config(**args)
        assert L.lbm_workspace_bytes(C.byref(cfg), C.byref(b)) == want, kw
    n0, u0 = np.ones(128), np.zeros((2, 128))
    ws = np.zeros(9 * 128)
    h = C.c_void_p()
    assert L.lbm_init(C.byref(good), ws.ctypes.data, ws.nbytes - 8, None, n0.ctypes.data, u0.ctypes.data,
                      C.byref(h)) == ERR_ARG
    assert L.lbm_init(C.byref(good), ws.ctypes.data, ws.nbytes, None, None, u0.ctypes.data, C.byref(h)) == ERR_ARG
    r = Run(good, n0, u0)
    assert r.L.lbm_step(r.h, -1) == ERR_ARG
    g = r.state()
    assert r.L.lbm_set_state(r.h, g.ctypes.data, g.nbytes - 8) == ERR_ARG
    assert r.L.lbm_totals(r.h, None) == ERR_ARG
    r.free()
