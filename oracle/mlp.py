"""FP64 reference of the rate surrogate (test infrastructure).

The surrogate is a multilayer perceptron 8 -> 128 -> 128 -> 128 -> 128 -> 1
with hard-swish activations h(z) = z * clip(z/6 + 1/2, 0, 1) on the four
hidden layers.  Parameters are W_l [in x out] and b_l [out]; the forward
pass is z_l = h_{l-1} W_l + b_l.
`quantize=True` emulates the bfloat16 training arithmetic: every operand of a
matrix product is rounded to bfloat16 (round to nearest even) -- the weights and
every layer input in the forward pass, and in the backward pass also the
back-propagated gradient dZ of each layer before it multiplies the layer input
(weight gradient) and the weights (input gradient); accumulation, activations
and the bias gradients (sums of the unrounded dZ) stay in higher precision.
Gradients are back-propagation of the mean-squared error with the rounding
treated as the identity.

Training data: features (log(omega/T), log(kappa/T), log n_e, Z, channel
one-hot) and labels log R, R = Gamma/g^2 from the oracle's rates (Primakoff
with the screening function by angular quadrature; the detailed-balance
absorption rates of the Compton-like, e-Z and e-e brems channels, the brems
ones without the cell's screening-fit factor).
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import load, make_params, _ptr

SIZES = [8, 128, 128, 128, 128, 1]
NCH = 4   # 0 Primakoff, 1 Compton-like, 2 e-Z brems, 3 e-e brems


def to_bf16(a):
    """Round float64/float32 values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    P = []
    for i in range(5):
        fan_in = SIZES[i]
        W = rng.standard_normal((SIZES[i], SIZES[i + 1])) * math.sqrt(1.0 / fan_in)
        b = np.zeros(SIZES[i + 1])
        P.append([W, b])
    return P


def act(z):
    return z * np.clip(z / 6.0 + 0.5, 0.0, 1.0)


def dact(z):
    return np.clip(z / 6.0 + 0.5, 0.0, 1.0) + np.where(np.abs(z) < 3.0, z / 6.0, 0.0)


def forward(P, X, quantize=False):
    h = np.asarray(X, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(P):
        hin = to_bf16(h) if quantize else h
        Wq = to_bf16(W) if quantize else W
        z = hin @ Wq + b
        cache.append((hin, Wq, z))
        h = act(z) if l < 4 else z
    return h[:, 0], cache


def loss_and_grads(P, X, Y, quantize=False):
    y, cache = forward(P, X, quantize)
    B = y.size
    r = y - Y
    loss = float(np.mean(r * r))
    dz = (2.0 / B) * r[:, None]
    grads = [None] * 5
    for l in range(4, -1, -1):
        hin, Wq, z = cache[l]
        if l < 4:
            dz = dz * dact(z)
        dzq = to_bf16(dz) if quantize else dz
        gW = hin.T @ dzq
        gb = dz.sum(axis=0)
        grads[l] = [gW, gb]
        dz = dzq @ Wq.T
    return loss, grads


# ---------------------------------------------------------------- training data

def _declare():
    L = load()
    if not hasattr(L, "_mlp_declared"):
        L.or_surrogate_labels.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.c_void_p]
        L.or_F_quad.restype = C.c_double
        L.or_F_quad.argtypes = [C.c_double]
        L._mlp_declared = True
    return L


def F_quad(s):
    return _declare().or_F_quad(float(s))


def labels(params, T, ne, Z, x, ch):
    """log R for each sample (R = Gamma/g^2 in s^-1 GeV^2 for Primakoff and
    s^-1 for the g_ae channels, with g = 1), and log(kappa/T)."""
    L = _declare()
    n = len(T)
    T = np.ascontiguousarray(T, dtype=np.float64); ne = np.ascontiguousarray(ne, dtype=np.float64)
    Z = np.ascontiguousarray(Z, dtype=np.float64); x = np.ascontiguousarray(x, dtype=np.float64)
    ch = np.ascontiguousarray(ch, dtype=np.int32)
    out = np.zeros(n); lk = np.zeros(n)
    P = make_params(params)
    L.or_surrogate_labels(C.byref(P), n, _ptr(T), _ptr(ne), _ptr(Z), _ptr(x), _ptr(ch), _ptr(out),
                          _ptr(lk))
    return out, lk


def sample_domain(n, seed, box=None):
    """The surrogate's training box (the shared seeded generator)."""
    from paper_2604_24627_amd.inputs import surrogate_samples
    return surrogate_samples(n, seed, box)
