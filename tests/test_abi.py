"""CPU checks of the C ABI: the library loads, exports what the headers declare,
its host-side coefficient builder agrees with the oracle, and bad arguments are
rejected with the documented codes.  No GPU is touched."""
import ctypes as C
import glob
import math
import os
import re

import numpy as np
import pytest

from oracle import theory as th
from paper_1510_07328_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b((?:lbm|srg)_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    names = declared_symbols()
    assert "lbm_init" in names and "lbm_step" in names and "lbm_moments" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    bound = {n for n, _, _ in lbm._SIGNATURES + lbm.EXTRA_SIGNATURES}
    # the batched / surrogate bindings register themselves on import
    import importlib

    for mod in ("paper_1510_07328_amd.batch", "paper_1510_07328_amd.surrogate"):
        importlib.import_module(mod)
    bound |= {n for n, _, _ in lbm.EXTRA_SIGNATURES}
    assert set(declared_symbols()) <= bound


def class_polynomial(coefs, k, eu, u2):
    w, l1, q, s, c3, k4 = coefs[6 * k: 6 * k + 6]
    return w, 1.0 + eu * (l1 + c3 * u2 + k4 * eu * eu) + q * eu * eu + s * u2


FAMILIES = [(th.FD_T0, None), (th.MB, None), (th.FD, 148.4131591025766), (th.FD, 0.3), (th.BE, 0.5), (th.BE, 0.9)]


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("family,z", FAMILIES)
def test_host_coefficients_match_oracle_tensor_expansion(lat, order, family, z):
    """Row a0: the library's float64 per-class equilibrium equals the oracle's
    tensor expansion (independent code) at random velocities."""
    weight = {th.FD_T0: lbm.LBM_W_FD_T0, th.MB: lbm.LBM_W_MB, th.FD: lbm.LBM_W_FD, th.BE: lbm.LBM_W_BE}[family]
    D = th.lattice_dim(lat)
    cfg = lbm.make_config(lat, shape=(4, 1 if D == 1 else 4, 1 if D < 3 else 4), weight=weight, order=order,
                          fugacity=z or 0.0)
    coefs = lbm.lbm_coefficients(cfg)
    if family == th.MB:
        model = th.make_model(lat, family, theta=1.0 / 3.0)
    elif family in (th.FD, th.BE):
        model = th.make_model(lat, family, z=z, theta=0.8)
    else:
        model = th.make_model(lat)
    e_lib = np.array(lbm.lbm_velocities(lat))[:, :D]
    rng = np.random.default_rng(12)
    for _ in range(5):
        u0 = 0.12 * rng.standard_normal(D)
        f_or = th.feq_tensor(model, 1.1, u0, order)
        for a, e in enumerate(e_lib):
            b = int(np.flatnonzero((model.e == e).all(axis=1))[0])
            k = int(e @ e)
            w, S = class_polynomial(coefs, k, float(e @ u0), float(u0 @ u0))
            assert 1.1 * w * S == pytest.approx(f_or[b], rel=1e-13, abs=1e-16)
    J2, J4, d2, d4 = coefs[-4:]
    assert J2 == pytest.approx(model.co.J2, rel=1e-14) and J4 == pytest.approx(model.co.J4, rel=1e-14)
    assert d2 == pytest.approx(th.Delta_sq(model.co.I, D, 2), rel=1e-13)


def test_velocity_sets_match_oracle_sets():
    for lat in ("d1v3", "d2v9", "d3v19"):
        D = th.lattice_dim(lat)
        lib_e = {tuple(v[:D]) for v in lbm.lbm_velocities(lat)}
        or_e = {tuple(int(c) for c in v) for v in th.velocity_set(lat)}
        assert lib_e == or_e


@pytest.mark.parametrize("kw,code", [
    (dict(tau=0.5), lbm.LbmError),
    (dict(tau=float("nan")), lbm.LbmError),
    (dict(order=4), lbm.LbmError),
    (dict(shape=(0, 4, 1)), lbm.LbmError),
    (dict(lattice="d1v3", shape=(8, 2, 1)), lbm.LbmError),
    (dict(block=100), lbm.LbmError),
    (dict(graph_steps=3), lbm.LbmError),
    (dict(weight=lbm.LBM_W_CUSTOM, J2=-1.0, J4=1.0), lbm.LbmError),
])
def test_invalid_configs_are_rejected(kw, code):
    cfg = lbm.make_config(**kw)
    with pytest.raises(code) as ei:
        lbm.lbm_workspace_bytes(cfg)
    assert ei.value.status in (-1, -2)


def test_unsupported_order_code():
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_coefficients(lbm.make_config(order=1))
    assert ei.value.status == -2


def test_workspace_bytes():
    cfg = lbm.make_config("d2v9", shape=(2048, 2048, 1))
    b = lbm.lbm_workspace_bytes(cfg)
    assert b >= 2 * 9 * 2048 * 2048 * 4
    cfg.scheme = lbm.LBM_SCHEME_AA
    assert lbm.lbm_workspace_bytes(cfg) < b
    cfg.precision = lbm.LBM_FP64
    assert lbm.lbm_workspace_bytes(cfg) >= 9 * 2048 * 2048 * 8


def test_null_pointers_are_rejected():
    lib = lbm.load()
    cfg = lbm.make_config()
    ctx = C.c_void_p()
    assert lib.lbm_init(C.byref(cfg), None, 0, None, None, None, C.byref(ctx)) == -1
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_free(None) == 0


def test_batch_workspace_and_argument_checks():
    """Host-only checks of the batched sweep's argument validation."""
    import numpy as np

    from paper_1510_07328_amd import batch as B

    tubes = B.make_tubes(np.array([256, 8192]), np.array([0.6, 0.7]), 1.0, np.array([0.8, 0.9]), 100)
    b32 = B.lbm_batch_workspace_bytes(tubes, B.make_options())
    cells = 4 * (256 + 8192)
    assert b32 >= 2 * 9 * cells * 4
    assert B.lbm_batch_workspace_bytes(tubes, B.make_options(precision=lbm.LBM_FP64)) >= 2 * 9 * cells * 8
    for bad_opt in (B.make_options(tile_cols=1100, halo=64), B.make_options(block=100), B.make_options(order=5)):
        with pytest.raises(lbm.LbmError):
            B.lbm_batch_workspace_bytes(tubes, bad_opt)
    for bad_tubes in (B.make_tubes(np.array([1]), 0.6, 1.0, 0.8, 10), B.make_tubes(np.array([64]), 0.5, 1.0, 0.8, 10),
                      B.make_tubes(np.array([64]), 0.6, -1.0, 0.8, 10), B.make_tubes(np.array([64]), 0.6, 1.0, 0.8, -1)):
        with pytest.raises(lbm.LbmError):
            B.lbm_batch_workspace_bytes(bad_tubes, B.make_options())


def test_surrogate_sizes_and_argument_checks():
    from oracle import conv
    from paper_1510_07328_amd import surrogate as S

    assert S.srg_param_count() == conv.param_count()
    small, big = S.srg_workspace_bytes(4, 256), S.srg_workspace_bytes(8, 256)
    assert big > small > 4 * S.srg_param_count() * 4
    for mb, L in [(0, 256), (4, 100), (4, 192), (4, 0), (-1, 128)]:
        with pytest.raises(lbm.LbmError) as e:
            S.srg_workspace_bytes(mb, L)
        assert e.value.status == -1
    h = C.c_void_p()
    assert lbm.load().srg_create(4, 256, None, 1 << 20, None, C.byref(h)) == -1
    assert lbm.load().srg_free(None) == 0
    assert lbm.load().srg_backward(None, None, None) == -1
    assert lbm.load().srg_infer(None, None, None, 1, None) == -1


def test_surrogate_init_matches_reference_initialisation():
    """Same He-normal draws as the float64 reference (both follow numpy's seeded generator)."""
    from oracle import conv
    from paper_1510_07328_amd import surrogate as S

    np.testing.assert_allclose(S.init_params(7), conv.init_params(7), rtol=1e-6, atol=1e-7)


def test_porous_config_workspace_and_checks():
    base = lbm.make_config("d2v9", shape=(100, 30, 1))
    w0 = lbm.lbm_workspace_bytes(base)
    w_obs = lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(100, 30, 1), obstacles=1))
    w_f = lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(100, 30, 1), force=(1e-5, 0, 0)))
    mask = (100 * 30 * 4 + 255) // 256 * 256  # one 32-bit link mask per cell
    assert w_obs - w0 == mask and w_f == w_obs
    for kw, code in [(dict(obstacles=2), -1), (dict(force=(float("nan"), 0, 0)), -1),
                     (dict(force=(0, float("inf"), 0)), -1)]:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(100, 30, 1), **kw))
        assert e.value.status == code
    assert lbm.load().lbm_set_solid(None, None) == -1


@pytest.mark.parametrize("weight,z", [(lbm.LBM_W_FD, 0.0), (lbm.LBM_W_FD, -1.0), (lbm.LBM_W_FD, float("inf")),
                                      (lbm.LBM_W_BE, 1.0), (lbm.LBM_W_BE, 1.5), (lbm.LBM_W_BE, 0.0),
                                      (lbm.LBM_W_FD, float("nan"))])
def test_quantum_weight_fugacity_checks(weight, z):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(8, 8, 1), weight=weight, fugacity=z))
    assert e.value.status == -1


@pytest.mark.parametrize("lat", ["d1v3", "d2v9", "d3v19"])
@pytest.mark.parametrize("order", [2, 3])
@pytest.mark.parametrize("r0", [0.0, 0.12, 0.3])
def test_local_weight_reference_coefficients_match_oracle(lat, order, r0):
    """Per-cell weights: lbm_coefficients reports the coefficients of a cell at the
    reference density, which must equal the oracle's tensor expansion with the
    Sommerfeld moments at theta / mu = r0."""
    from oracle.local_weights import local_moments

    D = th.lattice_dim(lat)
    cfg = lbm.make_config(lat, shape=(4, 1 if D == 1 else 4, 1 if D < 3 else 4), weight=lbm.LBM_W_FD_LOCAL,
                          order=order, theta_over_mu=r0)
    coefs = lbm.lbm_coefficients(cfg)
    model = th.model_from_moments(lat, local_moments(D, 1.0, r0))
    assert coefs[-4] == pytest.approx(model.co.J2, rel=1e-14)
    assert coefs[-3] == pytest.approx(model.co.J4, rel=1e-14)
    e_lib = np.array(lbm.lbm_velocities(lat))[:, :D]
    rng = np.random.default_rng(13)
    for _ in range(4):
        u0 = 0.1 * rng.standard_normal(D)
        f_or = th.feq_tensor(model, 0.9, u0, order)
        for a, e in enumerate(e_lib):
            b = int(np.flatnonzero((model.e == e).all(axis=1))[0])
            w, S = class_polynomial(coefs, int(e @ e), float(e @ u0), float(u0 @ u0))
            assert 0.9 * w * S == pytest.approx(f_or[b], rel=1e-13, abs=1e-16)


@pytest.mark.parametrize("kw,code", [({"theta_over_mu": -0.1}, -1), ({"theta_over_mu": 0.6}, -1),
                                     ({"theta_over_mu": float("nan")}, -1),
                                     ({"theta_over_mu": 0.1, "obstacles": 1}, -2),
                                     ({"theta_over_mu": 0.1, "force": (1e-6, 0.0, 0.0)}, -2)])
def test_local_weight_checks(kw, code):
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(8, 8, 1), weight=lbm.LBM_W_FD_LOCAL, **kw))
    assert e.value.status == code


def test_batched_sweep_rejects_local_weights():
    from paper_1510_07328_amd import batch as B

    tubes = B.make_tubes([64], [0.7], [1.0], [0.9], [10])
    with pytest.raises(lbm.LbmError) as e:
        B.lbm_batch_workspace_bytes(tubes, B.make_options(weight=lbm.LBM_W_FD_LOCAL))
    assert e.value.status == -2


@pytest.mark.parametrize("order", [2, 3, 4])
def test_d2v41_host_coefficients_match_oracle(order):
    """The 41-velocity set and the fourth-order expansion: the library's collapsed
    per-class polynomial (closed-form contraction of eqs. H0-H4 with A0-A4) equals
    the oracle's tensor expansion on its own velocity set and scale.  The bound
    is the conditioning of the scale: the weights move about 200 times faster
    than c_0, and each side finds c_0 by its own bisection."""
    m = th.make_model("d2v41")
    co = lbm.lbm_coefficients(lbm.make_config("d2v41", shape=(8, 8, 1), order=order))
    shells = [0, 1, 2, 4, 8, 9, 10, 13, 16]
    assert len(co) == 6 * 9 + 4 + 3 * 9 + 1
    assert co[-1] == pytest.approx(m.cvel / math.sqrt(3 * m.co.I[4] / m.co.I[2]), rel=1e-13)
    e_lib = np.array(lbm.lbm_velocities("d2v41"))[:, :2]
    assert sorted(map(tuple, e_lib)) == sorted(map(tuple, m.e))
    extra = co[6 * 9 + 4:]
    rng = np.random.default_rng(14)
    for _ in range(4):
        u0 = 0.05 * rng.standard_normal(2)
        f_or = th.feq_tensor(m, 1.1, u0, order)
        for e in e_lib:
            b = int(np.flatnonzero((m.e == e).all(axis=1))[0])
            k = shells.index(int(e @ e))
            w, S = class_polynomial(co, k, float(e @ u0), float(u0 @ u0))
            p4, r4, t4 = extra[3 * k: 3 * k + 3]
            eu2, u2 = float(e @ u0) ** 2, float(u0 @ u0)
            S += p4 * eu2 * eu2 + r4 * eu2 * u2 + t4 * u2 * u2
            assert 1.1 * w * S == pytest.approx(f_or[b], rel=2e-12)


@pytest.mark.parametrize("kw,code", [({"bc": (1, 0, 0)}, -2), ({"obstacles": 1}, -2), ({"weight": 0}, -2),
                                     ({"order": 5}, -2), ({"block": 1024}, -1), ({"shape": (3, 8, 1)}, -1)])
def test_d2v41_checks(kw, code):
    args = {"shape": (16, 16, 1), "order": 4}
    args.update(kw)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(lbm.make_config("d2v41", **args))
    assert e.value.status == code


def test_order_four_needs_the_41_velocity_set():
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes(lbm.make_config("d2v9", shape=(8, 8, 1), order=4))
    assert e.value.status == -2
