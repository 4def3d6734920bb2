"""Pins of the warm-start network oracle: central finite differences of the loss
(FP64, tiny net), the adjoint relation between forward and data-gradient
convolutions, an identity kernel, Adam's first step, and bf16 rounding."""
import numpy as np

from oracle import conv3d as C


def tiny_net(rng, chans=(3, 4, 2)):
    params = []
    for ci, co in zip(chans[:-1], chans[1:]):
        params.append((rng.standard_normal((27, co, ci)) * 0.3, rng.standard_normal(co) * 0.1))
    return params


def loss_of(params, X, T, dims):
    out, _ = C.net_forward(X, params, dims)
    return C.mse(out, T)[0]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    dims = (5, 4, 3)
    V = 5 * 4 * 3
    params = tiny_net(rng)
    X = rng.standard_normal((V, 3))
    T = rng.standard_normal((V, 2))
    out, cache = C.net_forward(X, params, dims)
    L, dout = C.mse(out, T)
    grads, dX = C.net_backward(dout, params, cache, dims)
    eps = 1e-6
    for li in range(len(params)):
        W, b = params[li]
        for idx in [(13, 0, 0), (0, 1, 2), (26, 1, 1), (5, 0, 1)]:
            idx = tuple(min(i, s - 1) for i, s in zip(idx, W.shape))
            Wp = W.copy(); Wp[idx] += eps
            Wm = W.copy(); Wm[idx] -= eps
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (loss_of(pp, X, T, dims) - loss_of(pm, X, T, dims)) / (2 * eps)
            an = grads[li][0][idx]
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)) + 1e-9, (li, idx, fd, an)
        for o in range(b.size):
            bp = b.copy(); bp[o] += eps
            bm = b.copy(); bm[o] -= eps
            pp = list(params); pp[li] = (W, bp)
            pm = list(params); pm[li] = (W, bm)
            fd = (loss_of(pp, X, T, dims) - loss_of(pm, X, T, dims)) / (2 * eps)
            assert abs(fd - grads[li][1][o]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9
    for v, c in [(0, 0), (17, 2), (V - 1, 1)]:
        Xp = X.copy(); Xp[v, c] += eps
        Xm = X.copy(); Xm[v, c] -= eps
        fd = (loss_of(params, Xp, T, dims) - loss_of(params, Xm, T, dims)) / (2 * eps)
        assert abs(fd - dX[v, c]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_data_gradient_is_the_adjoint_of_the_convolution():
    rng = np.random.default_rng(1)
    dims = (6, 5, 4)
    V = 120
    W = rng.standard_normal((27, 5, 3))
    X = rng.standard_normal((V, 3))
    Y = rng.standard_normal((V, 5))
    lhs = np.sum(C.conv_forward(X, W, np.zeros(5), dims) * Y)
    rhs = np.sum(X * C.conv_backward_data(Y, W, dims))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # weight gradient is the adjoint in W: <conv(X; W'), Y> = <W', dW(Y, X)>
    W2 = rng.standard_normal((27, 5, 3))
    dW, db = C.conv_backward_weight(Y, X, dims)
    assert abs(np.sum(C.conv_forward(X, W2, np.zeros(5), dims) * Y) - np.sum(W2 * dW)) <= 1e-11 * abs(lhs)
    assert np.allclose(db, Y.sum(axis=0))


def test_identity_kernel_and_boundary_padding():
    rng = np.random.default_rng(2)
    dims = (4, 3, 5)
    V = 60
    X = rng.standard_normal((V, 2))
    W = np.zeros((27, 2, 2))
    W[13] = np.eye(2)                     # centre tap
    assert np.allclose(C.conv_forward(X, W, np.zeros(2), dims), X)
    # a +x shift tap reads the right neighbour, zero on the last x layer
    W = np.zeros((27, 1, 1))
    W[14, 0, 0] = 1.0                     # dx = 2 -> offset +1 in x
    Y = C.conv_forward(X[:, :1], W, np.zeros(1), dims).reshape(5, 3, 4)
    Xv = X[:, 0].reshape(5, 3, 4)
    assert np.allclose(Y[:, :, :3], Xv[:, :, 1:])
    assert np.all(Y[:, :, 3] == 0.0)


def test_adam_first_step_moves_by_lr_times_sign():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = C.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(w1, w - 0.01 * np.sign(g))


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -3.140625, 65504.0])
    r = C.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie to even
    assert r[2] == 1.0 + 2.0 ** -7           # above the tie: rounds up
    assert r[3] == -3.140625                 # exactly representable
    rel = np.abs(C.bf16_round(np.random.default_rng(0).standard_normal(1000)) - 0)
    assert np.all(np.isfinite(rel))
