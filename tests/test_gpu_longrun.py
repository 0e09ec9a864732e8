"""Long-run accuracy of the float32 deviation path against stored float64 oracle
values (tests/golden/rf256_order2.npz, written by tests/golden/make_golden.py
from the oracle alone): a 256 x 256 field with the recipe of the 2048 x 2048
workload, 10000 steps.

Bars: float64 storage within 1e-11 relative (rounding-order differences and the
oracle's A_0 P_0 rounding bias of about 2e-16 per step, over 1e4 steps);
float32 deviations within the 1e-6 relative L-infinity target on n, and on u
within the storage-rounding bound max(1e-6, 10 2^-24 |g|_max sqrt(t + 1) / |u|_max)
(u normwise over the velocity field).  The errors at every checkpoint are
printed so the growth with step count is visible in the log.
"""
import os

import numpy as np
import pytest

from gpu_helpers import field_errors, gpu_run
from paper_1510_07328_amd import inputs, lbm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rf256_order2.npz")


def golden():
    z = np.load(GOLDEN, allow_pickle=False)
    cps = [int(t) for t in z["checkpoints"]]
    return cps, [(z[f"n_{t}"], z[f"u_{t}"]) for t in cps]


@pytest.mark.parametrize("precision", [lbm.LBM_FP64, lbm.LBM_FP32_DEV])
@pytest.mark.parametrize("scheme", [lbm.LBM_SCHEME_PUSH, lbm.LBM_SCHEME_AA])
def test_longrun_against_stored_oracle(gpu, precision, scheme):
    cps, ref = golden()
    n0, u0 = inputs.perturbed_field((256, 256), 0.01, 32.0, (1e-4, 0.0), seed=0)
    cfg = lbm.make_config("d2v9", shape=(256, 256, 1), order=2, tau=0.55, precision=precision, scheme=scheme)
    errs = [field_errors(g, r) for g, r in zip(gpu_run(cfg, n0, u0, cps), ref)]
    for t, e in zip(cps, errs):
        print(f"precision={precision} scheme={scheme} t={t}: n {e['n']:.3e}  u {e['u']:.3e}  "
              f"(n-1) {e['dn']:.3e}", flush=True)
    for t, e, (n_r, u_r) in zip(cps, errs, ref):
        if precision == lbm.LBM_FP64:
            assert e["n"] < 1e-11 and e["u"] < 1e-11, (t, e)
        else:
            g_max = float(np.max(np.abs(n_r - 1.0))) / 6 + float(np.max(np.abs(u_r)))
            bound = max(1e-6, 10 * 2.0 ** -24 * g_max * np.sqrt(t + 1) / float(np.max(np.abs(u_r))))
            print(f"  t={t}: u bound {bound:.2e}", flush=True)
            assert e["n"] < 1e-6 and e["u"] < bound, (t, e)
