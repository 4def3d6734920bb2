"""GPU parity of the warm-start network kernels against the FP64 oracle
(oracle/conv3d.py).  Operands are rounded to bfloat16 on both sides, so products
are exact in FP32 and only the accumulation order/precision differs: FP32
outputs within 1e-5 relative, bfloat16-stored outputs within 1e-2."""
import numpy as np
import pytest

from oracle import conv3d as C

pytestmark = pytest.mark.gpu


def bf16_bits(a):
    """float64 values (already bf16-representable) -> int16 tensor of bf16 bits on the GPU."""
    import torch
    f = np.asarray(a, dtype=np.float32)
    bits = (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.tensor(bits.ravel(), device="cuda")


def from_bits(t):
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


# (65, 65, 65): the 64^3 workload's node lattice, with the network's padded layer shapes
# (input 32 -> 64, hidden 64 -> 64, output 64 -> 32), as the warm start runs them
@pytest.mark.parametrize("dims,cin,cout", [((7, 5, 6), 32, 64), ((9, 4, 3), 64, 32),
                                           ((5, 5, 5), 64, 96), ((3, 2, 2), 32, 32),
                                           ((65, 65, 65), 32, 64), ((65, 65, 65), 64, 64),
                                           ((65, 65, 65), 64, 32)])
def test_conv_forward_and_data_gradient(dims, cin, cout):
    import torch
    import paper_2601_08266_amd.warmstart as ws
    rng = np.random.default_rng(cin + cout)
    V = int(np.prod(dims))
    X = C.bf16_round(rng.standard_normal((V, cin)))
    W = C.bf16_round(rng.standard_normal((27, cout, cin)) * 0.2)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    Xt, Wt = bf16_bits(X), bf16_bits(W)
    bt = torch.tensor(b, dtype=torch.float32, device="cuda")
    Yf = torch.empty(V * cout, dtype=torch.float32, device="cuda")
    Yb = torch.empty(V * cout, dtype=torch.int16, device="cuda")
    ws.conv3d_fwd(dims, cin, cout, Xt, Wt, bt, relu=False, Ybf=Yb, Yf=Yf)
    ref = C.conv_forward(X, W, b, dims)
    e1 = rel(Yf.cpu().numpy().reshape(V, cout), ref)
    e2 = rel(from_bits(Yb).reshape(V, cout), ref)
    # ReLU variant
    Yr = torch.empty(V * cout, dtype=torch.float32, device="cuda")
    ws.conv3d_fwd(dims, cin, cout, Xt, Wt, bt, relu=True, Yf=Yr)
    e3 = rel(Yr.cpu().numpy().reshape(V, cout), np.maximum(ref, 0))
    # data gradient with a ReLU gate
    dY = C.bf16_round(rng.standard_normal((V, cout)))
    gate = C.bf16_round(rng.standard_normal((V, cin)))
    Wd = torch.empty_like(Wt)
    ws.flip_transpose(cin, cout, Wt, Wd)
    dX = torch.empty(V * cin, dtype=torch.float32, device="cuda")
    ws.conv3d_fwd(dims, cout, cin, bf16_bits(dY), Wd, None, gate=bf16_bits(gate), Yf=dX)
    refd = C.conv_backward_data(dY, W, dims) * (gate > 0)
    e4 = rel(dX.cpu().numpy().reshape(V, cin), refd)
    print(f"conv {dims} {cin}->{cout}: fwd f32 {e1:.2e} bf16 {e2:.2e} relu {e3:.2e} dgrad {e4:.2e}")
    assert e1 <= 1e-5 and e3 <= 1e-5 and e4 <= 1e-5
    assert e2 <= 1e-2


@pytest.mark.parametrize("dims,cin,cout", [((7, 5, 6), 32, 64), ((13, 11, 17), 64, 64),
                                           ((4, 4, 3), 64, 32), ((65, 65, 65), 64, 64),
                                           ((5, 6, 7), 32, 96), ((3, 4, 5), 32, 288)])
def test_conv_weight_gradient(dims, cin, cout):
    import torch
    import paper_2601_08266_amd.warmstart as ws
    rng = np.random.default_rng(7 + cin)
    V = int(np.prod(dims))
    X = C.bf16_round(rng.standard_normal((V, cin)))
    dY = C.bf16_round(rng.standard_normal((V, cout)))
    dW = torch.empty(27 * cout * cin, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    ws.conv3d_wgrad(dims, cin, cout, bf16_bits(dY), bf16_bits(X), dW, db)
    rW, rb = C.conv_backward_weight(dY, X, dims)
    e1 = rel(dW.cpu().numpy().reshape(27, cout, cin), rW)
    e2 = rel(db.cpu().numpy(), rb)
    print(f"wgrad {dims} {cin}->{cout}: dW {e1:.2e} db {e2:.2e}")
    assert e1 <= 1e-5 and e2 <= 1e-5
    # deterministic
    dW2 = torch.empty_like(dW)
    ws.conv3d_wgrad(dims, cin, cout, bf16_bits(dY), bf16_bits(X), dW2, None)
    assert torch.equal(dW, dW2)


def test_mse_adam_pack_moments_unpack():
    import torch
    import paper_2601_08266_amd.warmstart as ws
    rng = np.random.default_rng(3)
    V, c, used = 1000, 32, 4
    pred = rng.standard_normal((V, c)).astype(np.float32)
    targ = rng.standard_normal((V, c)).astype(np.float32)
    dp = torch.empty(V * c, dtype=torch.int16, device="cuda")
    loss = ws.mse_loss(V, c, used, torch.tensor(pred.ravel(), device="cuda"),
                       torch.tensor(targ.ravel(), device="cuda"), dp)
    rl, rg = C.mse(pred[:, :used].astype(np.float64), targ[:, :used].astype(np.float64))
    assert abs(loss - rl) <= 1e-12 * rl
    g = from_bits(dp).reshape(V, c)
    assert rel(g[:, :used], rg) <= 4e-3 and np.all(g[:, used:] == 0)
    # Adam: several steps against the oracle in FP64 (FP32 device arithmetic)
    w = rng.standard_normal(500)
    m = np.zeros(500); v = np.zeros(500)
    tw = torch.tensor(w, dtype=torch.float32, device="cuda")
    tm = torch.zeros(500, device="cuda"); tv = torch.zeros(500, device="cuda")
    for t in range(1, 6):
        gr = rng.standard_normal(500)
        w, m, v = C.adam_step(w, gr, m, v, t, lr=1e-2)
        ws.adam_step(tw, torch.tensor(gr, dtype=torch.float32, device="cuda"), tm, tv, t, lr=1e-2)
    assert rel(tw.cpu().numpy(), w) <= 1e-5
    # pack / moments / unpack
    N = 300
    a = torch.tensor(rng.standard_normal(N), device="cuda", dtype=torch.float64)
    b = torch.tensor(rng.standard_normal(N), device="cuda", dtype=torch.float64)
    out = torch.empty(N * 32, device="cuda")
    ws.pack(N, 32, [([(1.0, a)], 0.0, 0.5, 2.0), ([(1.0, a), (-1.0, b)], 0.0, 0.0, 1.0),
                    ([], 3.0, 1.0, 1.0), ([(2.0, a), (-1.0, b), (0.5, a)], 0.25, 0.0, 1.0)], out)
    o = out.cpu().numpy().reshape(N, 32)
    an, bn = a.cpu().numpy(), b.cpu().numpy()
    assert np.allclose(o[:, 0], (an - 0.5) * 2.0, atol=1e-6)
    assert np.allclose(o[:, 1], an - bn, atol=1e-6)
    assert np.allclose(o[:, 2], 2.0) and np.all(o[:, 4:] == 0)
    assert np.allclose(o[:, 3], 2.5 * an - bn + 0.25, atol=1e-6)
    mom = ws.moments(N, 32, out)
    assert abs(mom[1][0] - float(np.sum(o[:, 1].astype(np.float64)))) <= 1e-9
    assert abs(mom[1][1] - float(np.sum(o[:, 1].astype(np.float64) ** 2))) <= 1e-9
    base = torch.tensor(rng.standard_normal(4 * N), device="cuda", dtype=torch.float64)
    x = torch.empty_like(base)
    ws.unpack(N, 32, out, base, [0.1, 0.2, 0.3, 0.4], [2.0, 2.0, 2.0, 2.0], x)
    exp = base.cpu().numpy().reshape(4, N) + o[:, :4].T.astype(np.float64) / 2.0 + \
        np.array([0.1, 0.2, 0.3, 0.4])[:, None]
    assert np.allclose(x.cpu().numpy().reshape(4, N), exp, atol=1e-12)


def test_network_gradients_against_oracle_and_training_reduces_loss():
    """A 3-layer net on a 9x8x7 lattice: the GPU gradients of the first training step match
    the oracle's (on the same bf16 weights and input) and 60 Adam steps lower the loss."""
    import torch
    import paper_2601_08266_amd.warmstart as ws
    dims = (9, 8, 7)
    V = int(np.prod(dims))
    net = ws.WarmStartNet(dims, in_ch=5, hidden=32, n_hidden=1, out_ch=4, seed=1)
    rng = np.random.default_rng(11)
    Xin = np.zeros((V, 32))
    Xin[:, :5] = C.bf16_round(rng.standard_normal((V, 5)))
    coords = np.stack(np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]),
                                  indexing="ij"), -1).reshape(V, 3)[:, ::-1] / 8.0
    T = np.zeros((V, 32))
    T[:, 0] = np.sin(2 * coords[:, 0]) + Xin[:, 0]
    T[:, 1] = Xin[:, 1] * Xin[:, 2]
    T[:, 2] = coords[:, 2]
    T[:, 3] = np.maximum(Xin[:, 3], 0)
    xb = bf16_bits(Xin)
    tt = torch.tensor(T.ravel(), dtype=torch.float32, device="cuda")
    # oracle gradients on the bf16 weights
    params = []
    for i, lay in enumerate(net.layers):
        w = from_bits(lay.wbf).reshape(27, lay.cout, lay.cin)
        params.append((w, lay.b32.cpu().numpy().astype(np.float64)))
    out_o, cache = C.net_forward(Xin, params, dims)
    loss_o, dout = C.mse(out_o[:, :4], T[:, :4])
    dout_full = np.zeros_like(out_o)
    dout_full[:, :4] = dout
    grads_o, _ = C.net_backward(dout_full, params, cache, dims)
    out = net.forward(xb)
    assert rel(out.cpu().numpy().reshape(V, 32)[:, :4], out_o[:, :4]) <= 2e-2
    loss0 = ws.mse_loss(V, 32, 4, out, tt, net.dout)
    net.backward(net.dout)
    for i, lay in enumerate(net.layers):
        e = rel(lay.gw.cpu().numpy().reshape(27, lay.cout, lay.cin), grads_o[i][0])
        print(f"layer {i}: dW rel err {e:.2e}")
        assert e <= 5e-2
    assert abs(loss0 - loss_o) <= 2e-2 * loss_o
    losses = [net.train_sample(xb, tt, lr=3e-3) for _ in range(60)]
    print(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
