"""Float64 reference of the 1D convolutional surrogate (TEST INFRASTRUCTURE ONLY).

The network (the learned part of the workload; the paper has none):

    features  x0 = (n - 1) / 0.25,  x1 = u / 0.25,  x2 = (tau - 0.75) / 0.25
    z1 = conv(x;  W1, b1, dilation 1)   3 -> 64,  a1 = GELU(z1)
    z2 = conv(a1; W2, b2, dilation 3)  64 -> 64,  a2 = GELU(z2)
    z3 = conv(a2; W3, b3, dilation 9)  64 -> 64,  a3 = GELU(z3)
    y  = conv(a3; W4, b4, dilation 27) 64 -> 2
    n' = n + 0.25 y0,  u' = u + 0.25 y1

conv(a; W, b, d)[co, x] = b[co] + sum_{tap, ci} W[tap, co, ci] a[ci, x + (tap - 2) d],
kernel 5, zero outside [0, L).  GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.

`bf16` rounding (round to nearest even of the float32 value) can be applied at
the points where the GPU path stores bfloat16 (weights, z and a of the hidden
layers), so that the two sides take the same quantisation decisions.

Parameters are one flat float vector in the order W1, b1, W2, b2, W3, b3, W4, b4,
each W in [tap][co][ci] order.
"""
from __future__ import annotations

import math

import numpy as np

CH = 64
K = 5
DILATIONS = (1, 3, 9, 27)
SHAPES = [((K, CH, 3), (CH,)), ((K, CH, CH), (CH,)), ((K, CH, CH), (CH,)), ((K, 2, CH), (2,))]
FEATURE_SCALE = 0.25
TAU_CENTER = 0.75


def param_count() -> int:
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in SHAPES)


def unpack(params):
    out, o = [], 0
    for ws, bs in SHAPES:
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        out.append((np.asarray(params[o:o + nw], dtype=np.float64).reshape(ws),
                    np.asarray(params[o + nw:o + nw + nb], dtype=np.float64)))
        o += nw + nb
    return out


def pack(layers):
    return np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in layers])


def bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    from scipy.special import erf

    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    from scipy.special import erf

    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def conv(a, W, b, d):
    """a: [B, Cin, L]; W: [K, Cout, Cin]; b: [Cout] -> [B, Cout, L] (plain loops over taps)."""
    B, Cin, L = a.shape
    out = np.broadcast_to(b[None, :, None], (B, W.shape[1], L)).astype(np.float64).copy()
    for tap in range(K):
        s = (tap - 2) * d
        shifted = np.zeros_like(a)
        lo, hi = max(0, -s), min(L, L - s)
        if hi > lo:
            shifted[:, :, lo:hi] = a[:, :, lo + s:hi + s]
        out += np.einsum("oc,bcl->bol", W[tap], shifted)
    return out


def features(n, u, tau):
    """n, u: [B, L]; tau: [B] -> x: [B, 3, L]."""
    n, u = np.asarray(n, dtype=np.float64), np.asarray(u, dtype=np.float64)
    t = np.broadcast_to(((np.asarray(tau, dtype=np.float64) - TAU_CENTER) / FEATURE_SCALE)[:, None], n.shape)
    return np.stack([(n - 1.0) / FEATURE_SCALE, u / FEATURE_SCALE, t], axis=1)


def forward(params, n, u, tau, quantize=False):
    """Returns (n', u', cache).  quantize=True rounds weights and the hidden
    layers' z and a to bfloat16 where the GPU stores them."""
    q = bf16 if quantize else (lambda v: v)
    layers = [(q(w), b) for w, b in unpack(params)]
    x = features(n, u, tau)
    cache = {"x": x, "layers": layers, "z": [], "a": [x]}
    a = x
    for i, ((W, b), d) in enumerate(zip(layers, DILATIONS)):
        z = conv(a, W, b, d)
        if i < 3:
            zq = q(z)
            a = q(gelu(zq))
            cache["z"].append(zq)
            cache["a"].append(a)
        else:
            y = z
    cache["y"] = y
    return n + FEATURE_SCALE * y[:, 0], u + FEATURE_SCALE * y[:, 1], cache


def backward(cache, dn_out, du_out):
    """Gradients of a scalar loss with dL/dn' = dn_out, dL/du' = du_out ([B, L])
    with respect to the flat parameter vector (same packing as the parameters).
    Uses the cached (possibly quantised) activations; the arithmetic is float64."""
    layers = cache["layers"]
    dy = FEATURE_SCALE * np.stack([dn_out, du_out], axis=1)
    grads = [None] * 4
    dz = dy
    for i in range(3, -1, -1):
        W, b = layers[i]
        d = DILATIONS[i]
        a_in = cache["a"][i]
        B, Cin, L = a_in.shape
        dW = np.zeros_like(W)
        for tap in range(K):
            s = (tap - 2) * d
            shifted = np.zeros_like(a_in)
            lo, hi = max(0, -s), min(L, L - s)
            if hi > lo:
                shifted[:, :, lo:hi] = a_in[:, :, lo + s:hi + s]
            dW[tap] = np.einsum("bol,bcl->oc", dz, shifted)
        db = dz.sum(axis=(0, 2))
        grads[i] = (dW, db)
        if i == 0:
            break
        # d a_in[ci, x] = sum_{tap, co} dz[co, x - (tap - 2) d] W[tap, co, ci]
        da = np.zeros_like(a_in)
        for tap in range(K):
            s = (tap - 2) * d
            contrib = np.einsum("oc,bol->bcl", W[tap], dz)
            lo, hi = max(0, s), min(L, L + s)
            if hi > lo:
                da[:, :, lo:hi] += contrib[:, :, lo - s:hi - s]
        dz = da * gelu_grad(cache["z"][i - 1])
    return pack(grads)


def init_params(seed: int = 0, scale_out: float = 0.1):
    """He-style initialisation (normal, std sqrt(2 / fan_in)); the last layer is
    scaled down so the untrained network starts near the identity map."""
    rng = np.random.default_rng(seed)
    layers = []
    for i, (ws, bs) in enumerate(SHAPES):
        fan_in = ws[0] * ws[2]
        w = rng.standard_normal(ws) * math.sqrt(2.0 / fan_in)
        if i == 3:
            w *= scale_out
        layers.append((w, np.zeros(bs)))
    return pack(layers)
