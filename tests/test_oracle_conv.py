"""Pins of the float64 surrogate reference (oracle/conv.py) against library
routines and finite differences."""
import math

import numpy as np
import pytest
import torch
from scipy import ndimage, stats

from oracle import conv as C


def test_conv_matches_library_correlation_with_dilated_kernel():
    rng = np.random.default_rng(0)
    B, Cin, Cout, L = 2, 3, 4, 40
    a = rng.standard_normal((B, Cin, L))
    W = rng.standard_normal((C.K, Cout, Cin))
    b = rng.standard_normal(Cout)
    for d in C.DILATIONS[:3]:
        got = C.conv(a, W, b, d)
        for o in range(Cout):
            for i in range(Cin):
                kern = np.zeros(4 * d + 1)
                kern[::d] = W[:, o, i]
                # correlate1d centres the kernel: out[x] = sum_k kern[k] a[x + k - 2d]
                ref_oi = ndimage.correlate1d(a[:, i, :], kern, axis=-1, mode="constant", cval=0.0, origin=0)
                if i == 0:
                    ref = ref_oi
                else:
                    ref = ref + ref_oi
            np.testing.assert_allclose(got[:, o, :], ref + b[o], rtol=1e-12, atol=1e-12)


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(C.gelu(z), z * stats.norm.cdf(z), rtol=1e-13, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(C.gelu_grad(z), (C.gelu(z + h) - C.gelu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(1000) * 10 ** rng.uniform(-5, 3, 1000), [0.0, -0.0, 1.0, 1.00390625]])
    want = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(v), want)


def test_param_count():
    assert C.param_count() == 5 * 64 * 3 + 64 + 2 * (5 * 64 * 64 + 64) + 5 * 2 * 64 + 2 == 42754


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    B, L = 2, 96
    p = C.init_params(3, scale_out=1.0)
    n = 1 + 0.1 * rng.standard_normal((B, L))
    u = 0.05 * rng.standard_normal((B, L))
    tau = np.array([0.6, 0.9])
    wn, wu = rng.standard_normal((B, L)), rng.standard_normal((B, L))

    def loss(params):
        n1, u1, _ = C.forward(params, n, u, tau)
        return float(np.sum(wn * n1) + np.sum(wu * u1))

    _, _, cache = C.forward(p, n, u, tau)
    g = C.backward(cache, wn, wu)
    idx = rng.choice(p.size, size=60, replace=False)
    idx = np.concatenate([idx, [0, 959, 960, 1023, 1024, 21567, 21568, p.size - 3, p.size - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-7), i


def test_identity_at_zero_output_layer():
    """With the last layer zero the network is the identity map (global residual)."""
    p = C.init_params(4)
    layers = C.unpack(p)
    layers[3] = (np.zeros_like(layers[3][0]), np.zeros_like(layers[3][1]))
    rng = np.random.default_rng(5)
    n, u = 1 + 0.1 * rng.standard_normal((1, 64)), 0.05 * rng.standard_normal((1, 64))
    n1, u1, _ = C.forward(C.pack(layers), n, u, np.array([0.7]))
    np.testing.assert_array_equal(n1, n)
    np.testing.assert_array_equal(u1, u)
