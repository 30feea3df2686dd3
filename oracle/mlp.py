"""FP64 reference of the surrogate network (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline may import
this module. It shares nothing with the HIP kernels.

Network: inputs (ln T1, ln T2, B1), each mapped affinely from the training box
onto [-1, 1]; `depth` hidden layers of width `width` with the exact GELU
z * Phi(z) (Phi the standard normal CDF); a linear output layer of 8 T values.
Output o = c * 4T + p * T + n holds part c (0 real, 1 imaginary) of train p
(0: m, 1: dm/dlnT1, 2: dm/dlnT2, 3: dm/dB1) at TR n, divided by the head
scale s_p (the RMS of that train over the training set).

Loss: the mean over outputs and samples of the squared difference with the
scaled targets (real parts have target 0).

Parameters are packed in one flat vector: W1 [width][3], b1, then for each
further hidden layer W [width][width], b, then Wout [8T][width], bout
(weights row-major [out][in]).
"""
from __future__ import annotations

import math

import numpy as np

_SQRT2 = math.sqrt(2.0)
_SQRT2PI = math.sqrt(2.0 * math.pi)


def _erf(z):
    from scipy.special import erf
    return erf(z)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / _SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) / _SQRT2PI


def shapes(n_tr, width=256, depth=4):
    s = [(width, 3), (width,)]
    for _ in range(depth - 1):
        s += [(width, width), (width,)]
    s += [(8 * n_tr, width), (8 * n_tr,)]
    return s


def n_params(n_tr, width=256, depth=4):
    return int(sum(np.prod(x) for x in shapes(n_tr, width, depth)))


def unpack(flat, n_tr, width=256, depth=4):
    out, o = [], 0
    for s in shapes(n_tr, width, depth):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def normalise_inputs(theta3, lo, hi):
    """theta3 [3][B] = (ln T1, ln T2, B1) -> [-1, 1] over the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)[:, None]
    hi = np.asarray(hi, dtype=np.float64)[:, None]
    return 2.0 * (np.asarray(theta3, dtype=np.float64) - lo) / (hi - lo) - 1.0


def scaled_targets(trains_im, head_scale):
    """trains_im [4][T][B] (imaginary parts) -> targets [8T][B]."""
    P, T, B = trains_im.shape
    t = np.zeros((8 * T, B))
    for p in range(4):
        t[4 * T + p * T: 4 * T + (p + 1) * T] = trains_im[p] / head_scale[p]
    return t


def forward(flat, x, n_tr, width=256, depth=4):
    """x [3][B] normalised inputs -> (y [8T][B], cache)."""
    P = unpack(flat, n_tr, width, depth)
    h = x
    cache = []
    for l in range(depth):
        W, b = P[2 * l], P[2 * l + 1]
        z = W @ h + b[:, None]
        cache.append((h, z))
        h = gelu(z)
    Wo, bo = P[-2], P[-1]
    y = Wo @ h + bo[:, None]
    cache.append((h, None))
    return y, cache


def loss_and_grad(flat, x, target, n_tr, width=256, depth=4):
    """Mean squared error over all outputs and samples, and its gradient in
    the packed parameter layout (backpropagation through the layers)."""
    P = unpack(flat, n_tr, width, depth)
    y, cache = forward(flat, x, n_tr, width, depth)
    diff = y - target
    count = diff.size
    loss = float(np.sum(diff * diff) / count)
    dy = 2.0 * diff / count
    grads = [None] * len(P)
    h_last = cache[-1][0]
    grads[-2] = dy @ h_last.T
    grads[-1] = dy.sum(axis=1)
    dh = P[-2].T @ dy
    for l in range(depth - 1, -1, -1):
        h_in, z = cache[l]
        dz = dh * gelu_grad(z)
        grads[2 * l] = dz @ h_in.T
        grads[2 * l + 1] = dz.sum(axis=1)
        if l > 0:
            dh = P[2 * l].T @ dz
    return loss, np.concatenate([g.reshape(-1) for g in grads])
