"""FP64 reference of the learned projection (TEST INFRASTRUCTURE ONLY).

The paper notes (Section 6) that any non-random hashing can replace the
random projection in front of MSM. The learned form here is a two-layer
network mapping x in R^d to ell bits:

    a1 = x W1 + b1,  g = GELU(a1) (erf form),  a2 = g W2 + b2,  u = tanh(a2)
    bit c = 1 iff a2_c > 0                      (the sign, as in eq. (3))

trained on labelled pairs (y = 1 for an epsilon-pair) with the relaxed
Hamming distance D = (ell - u_i . u_j) / 2 (exactly the Hamming distance of
the sign strings when u is +-1):

    loss = mean over pairs of  y relu(D - h/2)^2 + (1 - y) relu(3h - D)^2
                              + lam (sum_c (1 - |u_ic|)^2 + sum_c (1 - |u_jc|)^2)

and Adam. Parameters are one packed FP64 vector [W1 (d x hid) | b1 | W2
(hid x ell) | b2], row-major, the layout of the GPU library. Only the tests,
the smoke check and the benchmark's CPU leg use this module; it shares no
code with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def sizes(d: int, hid: int, ell: int):
    return [d * hid, hid, hid * ell, ell]


def unpack(params, d: int, hid: int, ell: int):
    p = np.asarray(params, dtype=np.float64)
    o = np.cumsum([0] + sizes(d, hid, ell))
    return (p[o[0]:o[1]].reshape(d, hid), p[o[1]:o[2]], p[o[2]:o[3]].reshape(hid, ell), p[o[3]:o[4]])


def pack(W1, b1, W2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2)]).astype(np.float64)


def gelu(a):
    return 0.5 * a * (1.0 + erf(a / SQRT2))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a / SQRT2)) + a * np.exp(-0.5 * a * a) * INV_SQRT_2PI


def forward(X, params, d, hid, ell):
    """(a1, g, a2, u) for the rows of X, in FP64."""
    W1, b1, W2, b2 = unpack(params, d, hid, ell)
    x = np.asarray(X, dtype=np.float64)
    a1 = x @ W1 + b1
    g = gelu(a1)
    a2 = g @ W2 + b2
    return a1, g, a2, np.tanh(a2)


def loss_and_grad(X, pairs, labels, params, d, hid, ell, h, lam):
    """Mean loss over the pairs and its gradient w.r.t. the packed parameters."""
    W1, b1, W2, b2 = unpack(params, d, hid, ell)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    y = np.asarray(labels, dtype=np.float64)
    B = pairs.shape[0]
    x = np.asarray(X, dtype=np.float64)[pairs.reshape(-1)]  # rows i0, j0, i1, j1, ...
    a1 = x @ W1 + b1
    g = gelu(a1)
    a2 = g @ W2 + b2
    u = np.tanh(a2)
    ui, uj = u[0::2], u[1::2]
    D = 0.5 * (ell - np.sum(ui * uj, axis=1))
    rp = np.maximum(D - 0.5 * h, 0.0)
    rn = np.maximum(3.0 * h - D, 0.0)
    q = np.sum((1.0 - np.abs(u)) ** 2, axis=1)
    loss = np.mean(y * rp ** 2 + (1.0 - y) * rn ** 2 + lam * (q[0::2] + q[1::2]))
    # dloss/dD, then dD/du_i = -u_j / 2
    dD = (2.0 * y * rp - 2.0 * (1.0 - y) * rn) / B
    du = np.empty_like(u)
    du[0::2] = dD[:, None] * (-0.5 * uj)
    du[1::2] = dD[:, None] * (-0.5 * ui)
    du += (lam / B) * (-2.0 * (1.0 - np.abs(u)) * np.sign(u))
    da2 = du * (1.0 - u * u)
    gW2 = g.T @ da2
    gb2 = da2.sum(axis=0)
    dg = da2 @ W2.T
    da1 = dg * gelu_grad(a1)
    gW1 = x.T @ da1
    gb1 = da1.sum(axis=0)
    return float(loss), pack(gW1, gb1, gW2, gb2)


def adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) in FP64; returns (params, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def bits(X, params, d, hid, ell):
    """Sign strings (a2 > 0) packed as uint64 words, and a2 itself."""
    _, _, a2, _ = forward(X, params, d, hid, ell)
    b = (a2 > 0).astype(np.uint8)
    n = b.shape[0]
    W = (ell + 63) // 64
    padded = np.zeros((n, W * 64), dtype=np.uint8)
    padded[:, :ell] = b
    by = np.packbits(padded.reshape(n, W * 8, 8), axis=2, bitorder="little").reshape(n, W * 8)
    return by.view(np.uint64).reshape(n, W).copy(), a2
