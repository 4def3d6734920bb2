"""Learned warm start for the Newton iterations of ChannelRun (orchestration only).

Sample k (predicting state k+1) uses 19 input channels: u, v, w, p of states
k, k-1, k-2; B^T lambda of state k; B^T kappa g of the new step; the new inflow
value.  The prediction is a correction to the second-order extrapolation
2 x^k - x^{k-1}: the target is x^{k+1} - 2 x^k + x^{k-1} (4 channels), so a
network that has learned nothing returns the extrapolation.  Channels are
normalised with the training set's mean and standard deviation (computed by
the library's moment kernel).  The guess is extrapolation + correction with the
Dirichlet values imposed; the stepper keeps it only if its residual beats the
plain guess.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import axpby
from . import warmstart as ws
from .stepper import ChannelRun, StepRecord


class LearnedWarmStart:
    def __init__(self, run: ChannelRun, hidden=64, n_hidden=8, seed=0):
        self.run = run
        self.N = run.N
        self.dims = run.g.nodes_per_axis
        self.net = ws.WarmStartNet(self.dims, in_ch=ws.IN_CH, hidden=hidden, n_hidden=n_hidden,
                                   out_ch=ws.OUT_CH, seed=seed, device=run.dev)
        self.in_shift = [0.0] * ws.IN_CH
        self.in_scale = [1.0] * ws.IN_CH
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

    def input_sources(self, hist: List[StepRecord], k: int, lamg, inflow, normed=True):
        srcs = []
        for lag in range(3):
            st = hist[max(k - lag, 0)].x
            for f in range(4):
                srcs.append(([(1.0, self._field(st, f))], 0.0))
        for f in range(3):
            srcs.append(([(1.0, self._field(hist[k].btlam, f))], 0.0))
        for f in range(3):
            srcs.append(([(1.0, self._field(lamg, f))], 0.0))
        srcs.append(([], float(inflow)))
        out = []
        for c, (terms, cst) in enumerate(srcs):
            sh, sc = (self.in_shift[c], self.in_scale[c]) if normed else (0.0, 1.0)
            out.append((terms, cst, sh, sc))
        return out

    def target_sources(self, hist, k, normed=True):
        out = []
        prev = hist[max(k - 1, 0)].x
        for f in range(4):
            sh, sc = (self.out_shift[f], self.out_scale[f]) if normed else (0.0, 1.0)
            terms = [(1.0, self._field(hist[k + 1].x, f)), (-2.0, self._field(hist[k].x, f)),
                     (1.0, self._field(prev, f))]
            out.append((terms, 0.0, sh, sc))
        return out

    def extrapolation(self, run: ChannelRun, out: torch.Tensor):
        """out = 2 x^k - x^{k-1} (FP64 [4][N]) for the run's current state k."""
        k = run.n
        hist = run.history
        axpby(2.0, hist[k].x, 0.0, out)
        axpby(-1.0, hist[max(k - 1, 0)].x, 1.0, out)
        return out

    # ---------------------------------------------------------------- data
    def fit_normalisation(self, hist, ks):
        N = self.N
        sin = np.zeros((ws.IN_CH, 2))
        sout = np.zeros((4, 2))
        for k in ks:
            ws.pack(N, 32, self.input_sources(hist, k, hist[k + 1].lamg, hist[k + 1].inflow, False),
                    self.buf32)
            m = ws.moments(N, 32, self.buf32)
            sin += np.array(m[:ws.IN_CH])
            ws.pack(N, 32, self.target_sources(hist, k, False), self.buf32)
            m = ws.moments(N, 32, self.buf32)
            sout += np.array(m[:4])
        cnt = float(N * len(ks))

        def ms(s):
            mean = s[:, 0] / cnt
            var = np.maximum(s[:, 1] / cnt - mean ** 2, 0.0)
            std = np.sqrt(var)
            return mean, np.where(std > 1e-12 * max(1.0, np.abs(mean).max()), std, 1.0)

        mi, si = ms(sin)
        mo, so = ms(sout)
        self.in_shift, self.in_scale = list(mi), list(1.0 / si)
        self.out_shift, self.out_scale = list(mo), list(1.0 / so)

    def build_dataset(self, hist, ks):
        N = self.N
        self.X, self.T = [], []
        for k in ks:
            ws.pack(N, 32, self.input_sources(hist, k, hist[k + 1].lamg, hist[k + 1].inflow), self.buf32)
            xb = torch.empty(N * 32, dtype=torch.int16, device=self.run.dev)
            ws.to_bf16(self.buf32, xb)
            tt = torch.empty(N * 32, dtype=torch.float32, device=self.run.dev)
            ws.pack(N, 32, self.target_sources(hist, k), tt)
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
    def guess(self, run: ChannelRun, lamg, inflow):
        hist = run.history
        k = run.n
        N = self.N
        ws.pack(N, 32, self.input_sources(hist, k, lamg, inflow), self.buf32)
        ws.to_bf16(self.buf32, self.buf_bf)
        out = self.net.forward(self.buf_bf)
        base = self.extrapolation(run, torch.empty(4 * N, dtype=torch.float64, device=run.dev))
        x = torch.empty(4 * N, dtype=torch.float64, device=run.dev)
        ws.unpack(N, 32, out, base, self.out_shift, self.out_scale, x, mask=run.mask, gD=run.gD)
        return x

    def extrapolation_guess(self, run: ChannelRun, lamg, inflow):
        """The network's backbone alone: 2 x^k - x^{k-1} with the Dirichlet values imposed."""
        N = self.N
        base = self.extrapolation(run, torch.empty(4 * N, dtype=torch.float64, device=run.dev))
        x = torch.empty(4 * N, dtype=torch.float64, device=run.dev)
        ws.unpack(N, 32, run.zero_out, base, [0, 0, 0, 0], [1, 1, 1, 1], x, mask=run.mask,
                  gD=run.gD)
        return x
