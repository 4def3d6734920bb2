"""Learned warm start: a stack of 3x3x3 convolutions on the fluid node lattice, with its
forward pass, gradients and Adam steps in libfsi.so (argument marshalling only here).
What the network reads and predicts is set by its user (learned.py: the residual of the
extrapolated guess, the previous velocity and s, mapped to the guess's correction).

Architecture (defaults): in_ch input channels, conv layers in_ch -> hidden, then n_hidden
layers hidden -> hidden, then hidden -> out_ch (4), ReLU between layers; channels padded to
multiples of 32 in memory.  The default depth is n_hidden = 2 with hidden = 64 (four
convolutions, a 9-voxel receptive field): with the 19-20 training samples of a run it reaches a
lower training loss and a better guess than deeper stacks (ten convolutions: normalised loss
0.88 against 0.27 at 193^3, 0.89 against 0.21 at 65^3) at about half the inference time.
BF16 weights and activations, FP32 accumulation, FP32 master weights and Adam moments.
Inputs and targets are normalised per channel with statistics of the training set.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field
from typing import List, Optional

import torch

from . import _lib as L
from ._lib import FsiNnPackSpec, FsiNnUnpackSpec

IN_CH = 8         # the learned guess's inputs: residual rows (4), previous velocity (3), s
OUT_CH = 4


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def pad32(c: int) -> int:
    return (c + 31) // 32 * 32


def dims_arg(dims):
    return (ctypes.c_int32 * 3)(*[int(d) for d in dims])


# ------------------------------------------------------------------ thin wrappers
def conv3d_fwd(dims, cin, cout, X, W, bias=None, relu=False, gate=None, Ybf=None, Yf=None,
               stream=None):
    L.check("fsi_conv3d_fwd", L.lib().fsi_conv3d_fwd(
        dims_arg(dims), cin, cout, _p(X), _p(W), _p(bias), 1 if relu else 0, _p(gate), _p(Ybf),
        _p(Yf), _s(stream)))


def conv3d_wgrad(dims, cin, cout, dY, X, dW, db=None, ws=None, stream=None):
    nbytes = int(L.lib().fsi_conv3d_wgrad_workspace(dims_arg(dims), cin, cout))
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dY.device)
    L.check("fsi_conv3d_wgrad", L.lib().fsi_conv3d_wgrad(
        dims_arg(dims), cin, cout, _p(dY), _p(X), _p(dW), _p(db), _p(ws), ws.numel(), _s(stream)))
    return ws


def flip_transpose(cin, cout, W, Wd, stream=None):
    L.check("fsi_conv3d_flip_transpose",
            L.lib().fsi_conv3d_flip_transpose(cin, cout, _p(W), _p(Wd), _s(stream)))


def mse_loss(nvox, c, used, pred, target, dpred=None, ws=None, want_loss=True, stream=None):
    nbytes = int(L.lib().fsi_mse_workspace())
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=pred.device)
    loss = ctypes.c_double(0.0)
    L.check("fsi_mse_loss", L.lib().fsi_mse_loss(
        nvox, c, used, _p(pred), _p(target), _p(dpred), ctypes.byref(loss) if want_loss else None,
        _p(ws), ws.numel(), _s(stream)))
    return float(loss.value)


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, wbf=None, stream=None):
    L.check("fsi_adam_step", L.lib().fsi_adam_step(
        w.numel(), _p(w), _p(g), _p(m), _p(v), _p(wbf), int(t), lr, b1, b2, eps, _s(stream)))


def to_bf16(x, out, stream=None):
    L.check("fsi_to_bf16", L.lib().fsi_to_bf16(x.numel(), _p(x), _p(out), _s(stream)))


def pack(nvox, c, sources, out, stream=None):
    """sources: per channel (terms, cst, shift, scale) with terms a list of up to three
    (coefficient, FP64 field) pairs: channel = (sum coef * field + cst - shift) * scale."""
    spec = FsiNnPackSpec()
    spec.nch = len(sources)
    for i, (terms, cst, shift, scale) in enumerate(sources):
        if len(terms) > 3:
            raise ValueError("at most three fields per channel")
        for slot, (coef, fld) in zip(("a", "b", "c"), terms):
            getattr(spec, slot)[i] = fld.data_ptr()
            getattr(spec, "c" + slot)[i] = float(coef)
        spec.cst[i] = float(cst)
        spec.shift[i] = float(shift)
        spec.scale[i] = float(scale)
    L.check("fsi_nn_pack", L.lib().fsi_nn_pack(nvox, c, ctypes.byref(spec), _p(out), _s(stream)))


def moments(nvox, c, data, stream=None):
    nbytes = int(L.lib().fsi_nn_moments_workspace(c))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=data.device)
    out = (ctypes.c_double * (2 * c))()
    L.check("fsi_nn_moments", L.lib().fsi_nn_moments(nvox, c, _p(data), out, _p(ws), ws.numel(),
                                                     _s(stream)))
    return [(out[2 * i], out[2 * i + 1]) for i in range(c)]


def unpack(nvox, c, out, base, shift, scale, x, mask=None, gD=None, stream=None):
    spec = FsiNnUnpackSpec()
    for i in range(4):
        spec.shift[i] = float(shift[i])
        spec.scale[i] = float(scale[i])
    L.check("fsi_nn_unpack", L.lib().fsi_nn_unpack(nvox, c, _p(out), _p(base), ctypes.byref(spec),
                                                   _p(mask), _p(gD), _p(x), _s(stream)))


# ------------------------------------------------------------------ network
@dataclass
class Layer:
    cin: int
    cout: int
    w32: torch.Tensor          # [27][cout][cin] master weights (float)
    b32: torch.Tensor          # [cout]
    wbf: torch.Tensor          # bf16 bits (int16 storage) of w32
    wd: torch.Tensor           # flipped/transposed bf16 copy for the data gradient
    gw: torch.Tensor
    gb: torch.Tensor
    mw: torch.Tensor
    vw: torch.Tensor
    mb: torch.Tensor
    vb: torch.Tensor


class WarmStartNet:
    """Conv3d stack with FP32 master weights, BF16 compute copies and Adam state."""

    def __init__(self, dims, in_ch=IN_CH, hidden=64, n_hidden=2, out_ch=OUT_CH, seed=0,
                 device="cuda"):
        self.dims = tuple(int(d) for d in dims)
        self.V = self.dims[0] * self.dims[1] * self.dims[2]
        self.in_ch, self.out_ch = in_ch, out_ch
        chans = [in_ch] + [hidden] * (n_hidden + 1) + [out_ch]
        self.layers: List[Layer] = []
        gen = torch.Generator(device="cpu").manual_seed(seed)
        dev = torch.device(device)
        for ci, co in zip(chans[:-1], chans[1:]):
            cin, cout = pad32(ci), pad32(co)
            # He initialisation over the real fan-in; padded rows/columns stay zero
            w = torch.zeros(27, cout, cin)
            std = math.sqrt(2.0 / (27 * ci))
            w[:, :co, :ci] = torch.randn(27, co, ci, generator=gen) * std
            if co == out_ch:
                w *= 0.1
            w = w.to(dev).contiguous()
            b = torch.zeros(cout, device=dev)
            lay = Layer(cin, cout, w, b, torch.empty(w.numel(), dtype=torch.int16, device=dev),
                        torch.empty(w.numel(), dtype=torch.int16, device=dev),
                        torch.zeros_like(w), torch.zeros_like(b), torch.zeros_like(w),
                        torch.zeros_like(w), torch.zeros_like(b), torch.zeros_like(b))
            self.layers.append(lay)
        self.step = 0
        self.refresh()
        self.acts = None
        self.out32 = torch.empty(self.V * self.layers[-1].cout, device=dev)
        self.dout = torch.empty(self.V * self.layers[-1].cout, dtype=torch.int16, device=dev)
        self.g_a = torch.empty(self.V * max(l.cout for l in self.layers), dtype=torch.int16, device=dev)
        self.g_b = torch.empty_like(self.g_a)
        self.wg_ws = None
        self.mse_ws = None

    @property
    def n_params(self):
        real = [self.in_ch] + [l.cout for l in self.layers[:-1]] + [self.out_ch]
        n = 0
        for i, lay in enumerate(self.layers):
            ci = self.in_ch if i == 0 else real[i]
            co = self.out_ch if i == len(self.layers) - 1 else lay.cout
            n += 27 * ci * co + co
        return n

    def refresh(self):
        """BF16 copies and flipped/transposed data-gradient weights from the masters."""
        for lay in self.layers:
            to_bf16(lay.w32, lay.wbf)
            flip_transpose(lay.cin, lay.cout, lay.wbf, lay.wd)

    def _ensure_acts(self):
        if self.acts is None:
            dev = self.layers[0].w32.device
            self.acts = [torch.empty(self.V * self.layers[0].cin, dtype=torch.int16, device=dev)]
            for lay in self.layers[:-1]:
                self.acts.append(torch.empty(self.V * lay.cout, dtype=torch.int16, device=dev))

    def forward(self, x_bf16: torch.Tensor, stream=None) -> torch.Tensor:
        """x_bf16: [V][cin0] bf16 bits.  Returns the FP32 output [V][cout_last]."""
        self._ensure_acts()
        self.acts[0] = x_bf16
        h = x_bf16
        nl = len(self.layers)
        for i, lay in enumerate(self.layers):
            if i < nl - 1:
                conv3d_fwd(self.dims, lay.cin, lay.cout, h, lay.wbf, lay.b32, relu=True,
                           Ybf=self.acts[i + 1], stream=stream)
                h = self.acts[i + 1]
            else:
                conv3d_fwd(self.dims, lay.cin, lay.cout, h, lay.wbf, lay.b32, relu=False,
                           Yf=self.out32, stream=stream)
        return self.out32

    def backward(self, dout_bf16: torch.Tensor, stream=None):
        """Gradients of all layers from dL/d(out) (bf16 [V][cout_last]) into lay.gw / lay.gb."""
        g = dout_bf16
        bufs = [self.g_a, self.g_b]
        for i in range(len(self.layers) - 1, -1, -1):
            lay = self.layers[i]
            self.wg_ws = conv3d_wgrad(self.dims, lay.cin, lay.cout, g, self.acts[i], lay.gw, lay.gb,
                                      ws=self.wg_ws, stream=stream)
            if i > 0:
                nxt = bufs[i % 2]
                # dX of this layer, masked by the ReLU of the previous layer's output
                conv3d_fwd(self.dims, lay.cout, lay.cin, g, lay.wd, None, relu=False,
                           gate=self.acts[i], Ybf=nxt, stream=stream)
                g = nxt

    def adam(self, lr=1e-3, stream=None):
        self.step += 1
        for lay in self.layers:
            adam_step(lay.w32, lay.gw, lay.mw, lay.vw, self.step, lr=lr, wbf=lay.wbf, stream=stream)
            adam_step(lay.b32, lay.gb, lay.mb, lay.vb, self.step, lr=lr, stream=stream)
            flip_transpose(lay.cin, lay.cout, lay.wbf, lay.wd, stream=stream)

    def train_sample(self, x_bf16, target32, lr=1e-3, want_loss=True, stream=None):
        out = self.forward(x_bf16, stream=stream)
        lay = self.layers[-1]
        if self.mse_ws is None:
            self.mse_ws = torch.empty(int(L.lib().fsi_mse_workspace()), dtype=torch.uint8,
                                      device=out.device)
        loss = mse_loss(self.V, lay.cout, self.out_ch, out, target32, self.dout, ws=self.mse_ws,
                        want_loss=want_loss, stream=stream)
        self.backward(self.dout, stream=stream)
        self.adam(lr=lr, stream=stream)
        return loss

    def state_dict(self):
        return {"dims": self.dims, "step": self.step,
                "layers": [(l.w32.cpu(), l.b32.cpu()) for l in self.layers]}

    def load_state_dict(self, sd):
        for lay, (w, b) in zip(self.layers, sd["layers"]):
            lay.w32.copy_(w)
            lay.b32.copy_(b)
        self.step = sd["step"]
        self.refresh()
