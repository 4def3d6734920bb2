"""Learned warm start for the Newton iterations of ChannelRun (orchestration only).

The guess is the second-order extrapolation x_ex = 2 x^n - x^{n-1} plus a learned
correction: the network maps the residual of the extrapolation, R_ex = R(x_ex),
together with the velocity field the step starts from and the interface band s,
to the correction e = x^{n+1} - x_ex.  Near the solution e ~ J^{-1} R_ex, a linear
map, so R_ex and e are both divided by ||R_ex|| per sample (the network then
learns a fixed, scale-free local approximation of the inverse operator); the
channels are further normalised with training-set statistics.  A network that
has learned nothing returns the extrapolation; the stepper keeps the guess only
if its residual beats the plain one.
The network's correction c is applied with the step length a that minimises the
linearised residual ||R_ex + a (R(x_ex + c) - R_ex)|| (one extra residual
evaluation), so a correction that points the right way is never overshot.

Inputs (8 channels): R_ex / ||R_ex|| (u, v, w, p rows), u, v, w of the previous
state, s.  Target (4): e / ||R_ex||.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import axpby, dot
from . import warmstart as ws
from .stepper import ChannelRun, StepRecord

IN_CH = 8


class LearnedWarmStart:
    def __init__(self, run: ChannelRun, hidden=64, n_hidden=2, seed=0, line_search=True):
        self.run = run
        self.line_search = line_search
        self.last_step = 1.0
        self.N = run.N
        self.dims = run.g.nodes_per_axis
        self.net = ws.WarmStartNet(self.dims, in_ch=IN_CH, hidden=hidden, n_hidden=n_hidden,
                                   out_ch=ws.OUT_CH, seed=seed, device=run.dev)
        self.in_shift = [0.0] * IN_CH
        self.in_scale = [1.0] * IN_CH
        self.out_shift = [0.0] * 4
        self.out_scale = [1.0] * 4
        self.buf32 = torch.empty(self.N * 32, dtype=torch.float32, device=run.dev)
        self.buf_bf = torch.empty(self.N * 32, dtype=torch.int16, device=run.dev)
        self.X: List[torch.Tensor] = []
        self.T: List[torch.Tensor] = []
        self.train_ms = 0.0
        self.losses: List[float] = []

    # ---------------------------------------------------------------- channels
    def _field(self, t, f):
        return t[f * self.N:(f + 1) * self.N]

    def input_sources(self, R_ex, rn_ex, u_prev, s_field, normed=True):
        srcs = []
        for f in range(4):
            srcs.append(([(1.0 / rn_ex, self._field(R_ex, f))], 0.0))
        for f in range(3):
            srcs.append(([(1.0, self._field(u_prev, f))], 0.0))
        srcs.append(([(1.0, s_field)], 0.0))
        out = []
        for c, (terms, cst) in enumerate(srcs):
            sh, sc = (self.in_shift[c], self.in_scale[c]) if normed else (0.0, 1.0)
            out.append((terms, cst, sh, sc))
        return out

    def target_sources(self, rec_next, normed=True):
        out = []
        for f in range(4):
            sc = self.out_scale[f] if normed else 1.0
            terms = [(1.0 / rec_next.rn_ex, self._field(rec_next.x, f)),
                     (-1.0 / rec_next.rn_ex, self._field(rec_next.x_ex, f))]
            out.append((terms, 0.0, 0.0, sc))
        return out

    # ---------------------------------------------------------------- data
    def _samples(self, hist, ks):
        return [hist[k + 1] for k in ks if hist[k + 1].x_ex is not None and hist[k + 1].rn_ex > 0]

    def fit_normalisation(self, hist, ks):
        N = self.N
        sin = np.zeros((IN_CH, 2))
        sout = np.zeros((4, 2))
        recs = self._samples(hist, ks)
        for r in recs:
            ws.pack(N, 32, self.input_sources(r.R_ex, r.rn_ex, r.u_prev, r.s, False), self.buf32)
            sin += np.array(ws.moments(N, 32, self.buf32)[:IN_CH])
            ws.pack(N, 32, self.target_sources(r, False), self.buf32)
            sout += np.array(ws.moments(N, 32, self.buf32)[:4])
        cnt = float(N * len(recs))
        mean = sin[:, 0] / cnt
        rms = np.sqrt(np.maximum(sin[:, 1] / cnt, 0.0))
        std = np.sqrt(np.maximum(sin[:, 1] / cnt - mean ** 2, 0.0))
        shift, scale = np.zeros(IN_CH), np.ones(IN_CH)
        # residual channels: scale only (keeps the map linear); fields: mean and std
        for c in range(IN_CH):
            if c < 4:
                scale[c] = 1.0 / rms[c] if rms[c] > 0 else 1.0
            else:
                shift[c] = mean[c]
                scale[c] = 1.0 / std[c] if std[c] > 1e-12 * max(1.0, abs(mean[c])) else 1.0
        trms = np.sqrt(np.maximum(sout[:, 1] / cnt, 0.0))
        self.in_shift, self.in_scale = list(shift), list(scale)
        self.out_shift = [0.0] * 4
        self.out_scale = list(np.where(trms > 0, 1.0 / trms, 1.0))

    def build_dataset(self, hist, ks):
        N = self.N
        self.X, self.T = [], []
        for r in self._samples(hist, ks):
            ws.pack(N, 32, self.input_sources(r.R_ex, r.rn_ex, r.u_prev, r.s), self.buf32)
            xb = torch.empty(N * 32, dtype=torch.int16, device=self.run.dev)
            ws.to_bf16(self.buf32, xb)
            tt = torch.empty(N * 32, dtype=torch.float32, device=self.run.dev)
            ws.pack(N, 32, self.target_sources(r), tt)
            self.X.append(xb)
            self.T.append(tt)

    def train(self, epochs=20, lr=1e-3, seed=0, log=None):
        rng = np.random.default_rng(seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for ep in range(epochs):
            order = rng.permutation(len(self.X))
            ep_loss = 0.0
            for j, i in enumerate(order):
                lr_ep = lr * 0.5 * (1.0 + math.cos(math.pi * ep / max(epochs, 1)))
                loss = self.net.train_sample(self.X[i], self.T[i], lr=lr_ep, want_loss=True)
                ep_loss += loss
            self.losses.append(ep_loss / len(order))
            if log:
                log(f"epoch {ep + 1}/{epochs}: mean normalised loss {self.losses[-1]:.4e}")
        torch.cuda.synchronize()
        self.train_ms = (time.perf_counter() - t0) * 1e3

    # ---------------------------------------------------------------- inference
    def guess(self, run: ChannelRun, ctx):
        if ctx["x_ex"] is None or not ctx["rn_ex"] > 0:
            return None
        N = self.N
        u_prev = run.history[run.n].x[: 3 * N]
        ws.pack(N, 32, self.input_sources(ctx["R_ex"], ctx["rn_ex"], u_prev, ctx["s"]), self.buf32)
        ws.to_bf16(self.buf32, self.buf_bf)
        out = self.net.forward(self.buf_bf)
        x1 = torch.empty(4 * N, dtype=torch.float64, device=run.dev)
        scale = [sc / ctx["rn_ex"] for sc in self.out_scale]
        ws.unpack(N, 32, out, ctx["x_ex"], [0.0] * 4, scale, x1, mask=run.mask, gD=run.gD)
        if not self.line_search:
            return x1
        # step length along the correction c = x1 - x_ex: near the solution R is affine in x, so
        # R(x_ex + a c) ~ R_ex + a D with D = R(x1) - R_ex, minimised by a = -<R_ex, D> / <D, D>
        run.residual_norm(ctx["P64"], x1, ctx["lamg"])
        D = run.R.clone()
        axpby(-1.0, ctx["R_ex"], 1.0, D)
        dd = dot(D, D)
        if not dd > 0.0:
            return x1
        a = -dot(ctx["R_ex"], D) / dd
        self.last_step = a
        x = ctx["x_ex"].clone()
        axpby(a, x1, 1.0 - a, x)          # x_ex + a (x1 - x_ex); Dirichlet values are kept
        return x



def linear_extrapolation_guess(run: ChannelRun, ctx):
    """The network's backbone alone: 2 x^n - x^{n-1} with the Dirichlet values imposed."""
    return ctx["x_ex"]


def quadratic_extrapolation_guess(run: ChannelRun, ctx):
    """3 x^n - 3 x^{n-1} + x^{n-2} with the new Dirichlet values (a comparison guess)."""
    if run.n < 2:
        return None
    x = torch.empty_like(run.x)
    axpby(3.0, run.history[run.n].x, 0.0, x)
    axpby(-3.0, run.history[run.n - 1].x, 1.0, x)
    axpby(1.0, run.history[run.n - 2].x, 1.0, x)
    out = torch.empty_like(x)
    ws.unpack(run.N, 32, run.zero_out, x, [0, 0, 0, 0], [1, 1, 1, 1], out, mask=run.mask, gD=run.gD)
    return out
