"""Oracle of the warm-start network (TEST INFRASTRUCTURE ONLY: used by tests/,
never by the simulation package).

A fully connected network, n_in -> depth x width (GELU) -> n_out (linear),
parameters in one vector: per layer its weight matrix [out x in] row-major
then its bias [out]. Written in float64 numpy, step by step:

  forward   Z_l = X_l W_l^T + b_l, X_{l+1} = gelu(Z_l) (the exact erf form),
            the last layer linear;
  loss      mean of (Y - T)^2 over all outputs of the batch;
  backward  dY = 2 (Y - T) / (batch n_out); per layer from the last:
            dW_l = dZ_l^T X_l, db_l = column sums of dZ_l,
            dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1}),
            gelu'(z) = Phi(z) + z phi(z);
  AdamW     m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
            w -= lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd w).

With exact=False every operand of a matrix product (weights, activations,
deltas) is first rounded to BFloat16 (round to nearest even), as the GPU
network does before its matrix-core products; the products themselves are
summed in float64 here (FP32 on the GPU). With exact=True nothing is rounded.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def bf16_round(a):
    """float32 -> nearest BFloat16 (ties to even) -> float32."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    is_nan = ((u & 0x7F800000) == 0x7F800000) & ((u & 0x007FFFFF) != 0)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(is_nan, (u >> 16) | 0x40, r) & 0xFFFF
    return (r.astype(np.uint32) << 16).view(np.float32).reshape(f.shape)


def dims_of(n_in, width, depth, n_out):
    return [n_in] + [width] * depth + [n_out]


def num_params(dims):
    return sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))


def unpack(params, dims):
    """[(W, b)] per layer (views into params as float64)."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for i in range(len(dims) - 1):
        din, dout = dims[i], dims[i + 1]
        W = p[o:o + din * dout].reshape(dout, din)
        o += din * dout
        b = p[o:o + dout]
        o += dout
        out.append((W, b))
    assert o == p.size
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _q(a, exact):
    """An operand of a matrix product: as is, or rounded to BFloat16."""
    if exact:
        return np.asarray(a, dtype=np.float64)
    return bf16_round(np.asarray(a, dtype=np.float32)).astype(np.float64)


def forward(params, x, dims, exact=False):
    """Output and the per-layer (input, pre-activation) pairs."""
    layers = unpack(params, dims)
    X = np.asarray(x, dtype=np.float64)
    saved = []
    for li, (W, b) in enumerate(layers):
        Z = _q(X, exact) @ _q(W, exact).T + b
        saved.append((X, Z))
        X = Z if li == len(layers) - 1 else gelu(Z)
    return X, saved


def loss_and_grad(params, x, target, dims, exact=False):
    Y, saved = forward(params, x, dims, exact)
    T = np.asarray(target, dtype=np.float64)
    count = Y.size
    loss = float(np.mean((Y - T) ** 2))
    layers = unpack(params, dims)
    grads = [None] * len(layers)
    dZ = 2.0 * (Y - T) / count
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        X, _ = saved[li]
        dW = _q(dZ, exact).T @ _q(X, exact)
        db = dZ.sum(axis=0)
        grads[li] = (dW, db)
        if li > 0:
            _, Zp = saved[li - 1]
            dZ = (_q(dZ, exact) @ _q(W, exact)) * gelu_grad(Zp)
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adamw(params, m, v, g, t, lr, b1, b2, eps, wd):
    """One AdamW step (t counts from 1); returns new (params, m, v)."""
    w = np.asarray(params, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
