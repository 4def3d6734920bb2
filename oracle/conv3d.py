"""FP64 reference of the warm-start network (test infrastructure only).

The learned warm start is an addition to the paper's method (its predictor
step, section 2.4, is where a better initial guess enters): a stack of 3x3x3
convolutions on the node lattice, ReLU between layers, trained with a mean
squared error and Adam.

Layout: activations are channels-last [V][C] with voxel v = i + nx (j + ny k)
(the fluid node numbering); weights W[tap][c_out][c_in] with tap = dx + 3 (dy
+ 3 dz) for the offset (dx - 1, dy - 1, dz - 1); zero "same" padding.

  forward        Y[v, o] = b[o] + sum_tap sum_i X[v + off(tap), i] W[tap, o, i]
  data grad      dX[v, i] = sum_tap sum_o dY[v - off(tap), o] W[tap, o, i]
  weight grad    dW[tap, o, i] = sum_v dY[v, o] X[v + off(tap), i],  db[o] = sum_v dY[v, o]
  Adam           Kingma & Ba: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
                 w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in range(3) for dy in range(3) for dx in range(3)]


def _vol(X, dims):
    nx, ny, nz = dims
    return np.asarray(X, dtype=np.float64).reshape(nz, ny, nx, -1)


def _shifted(Xv, dx, dy, dz):
    """Array S with S[k, j, i] = X[k + dz - 1, j + dy - 1, i + dx - 1] (0 outside)."""
    P = np.pad(Xv, ((1, 1), (1, 1), (1, 1), (0, 0)))
    nz, ny, nx = Xv.shape[:3]
    return P[dz:dz + nz, dy:dy + ny, dx:dx + nx, :]


def _unshifted(Yv, dx, dy, dz):
    """Array S with S[k, j, i] = Y[k - dz + 1, j - dy + 1, i - dx + 1] (0 outside)."""
    return _shifted(Yv, 2 - dx, 2 - dy, 2 - dz)


def conv_forward(X, W, b, dims):
    Xv = _vol(X, dims)
    W = np.asarray(W, dtype=np.float64)
    Y = np.zeros(Xv.shape[:3] + (W.shape[1],))
    for t, (dx, dy, dz) in enumerate(TAPS):
        Y += _shifted(Xv, dx, dy, dz) @ W[t].T
    Y += np.asarray(b, dtype=np.float64)
    return Y.reshape(-1, W.shape[1])


def conv_backward_data(dY, W, dims):
    dYv = _vol(dY, dims)
    W = np.asarray(W, dtype=np.float64)
    dX = np.zeros(dYv.shape[:3] + (W.shape[2],))
    for t, (dx, dy, dz) in enumerate(TAPS):
        dX += _unshifted(dYv, dx, dy, dz) @ W[t]
    return dX.reshape(-1, W.shape[2])


def conv_backward_weight(dY, X, dims):
    dYv = _vol(dY, dims)
    Xv = _vol(X, dims)
    co, ci = dYv.shape[3], Xv.shape[3]
    dW = np.zeros((27, co, ci))
    for t, (dx, dy, dz) in enumerate(TAPS):
        dW[t] = dYv.reshape(-1, co).T @ _shifted(Xv, dx, dy, dz).reshape(-1, ci)
    db = dYv.reshape(-1, co).sum(axis=0)
    return dW, db


def relu(Z):
    return np.maximum(Z, 0.0)


def net_forward(X, params, dims):
    """params = [(W, b), ...]; ReLU after every layer but the last. Returns (out, cache)."""
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    h = acts[0]
    for li, (W, b) in enumerate(params):
        z = conv_forward(h, W, b, dims)
        pre.append(z)
        h = relu(z) if li < len(params) - 1 else z
        acts.append(h)
    return h, (acts, pre)


def mse(pred, target):
    d = np.asarray(pred) - np.asarray(target)
    return float(np.mean(d * d)), 2.0 * d / d.size


def net_backward(dout, params, cache, dims):
    """Gradients [(dW, db), ...] and dX of the input, given dL/d(out)."""
    acts, pre = cache
    grads = [None] * len(params)
    g = np.asarray(dout, dtype=np.float64)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        if li < len(params) - 1:
            g = g * (pre[li] > 0.0)
        dW, db = conv_backward_weight(g, acts[li], dims)
        grads[li] = (dW, db)
        g = conv_backward_data(g, W, dims)
    return grads, g


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a):
    """Round FP64/FP32 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rounding) >> 16) << 16
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out
