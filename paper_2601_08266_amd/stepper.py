"""Implicit time stepping of the channel-with-rotating-plates problem (argument
marshalling and orchestration only; every computation runs in libfsi.so).

Per step n -> n+1 (t = (n+1) dt), the order of section 2.4's solution
algorithm with the stand-ins of this library:
  1. the immersed points move (rigid rotation of the plates): locate, sort,
     interface band of s, per-cell DLM blocks, lamg = B^T (kappa g);
  2. the inflow value and the Dirichlet data g_D;
  3. the initial guess: the previous state with the Dirichlet values imposed
     (plain), or a proposed (e.g. learned) guess kept only if its residual is the
     smallest among the plain guess, the extrapolation 2x^n - x^{n-1} and itself;
  4. Newton to ||R|| <= rel_tol ||R(x_plain)|| (the same absolute threshold for
     any guess, so a guess can change the work, never the answer);
  5. the multiplier lambda = kappa (g - B u) of the new state, spread to the
     nodes (B^T lambda), recorded with the state for the learned warm start.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Callable, List, Optional

import numpy as np
import torch

import fsi_workloads as W

from . import (Problem, axpby, dlm_B, dlm_BT, dlm_gram, dlm_locate, make_params, newton_opts,
               newton_solve, norm2, vms_residual)
from . import warmstart as ws


@dataclass
class StepRecord:
    n: int                       # index of the new state (x^{n})
    t: float
    x: torch.Tensor              # [4][N] FP64 state
    btlam: torch.Tensor          # B^T lambda at this state [3][N]
    lamg: torch.Tensor           # B^T kappa g used by this step [3][N]
    inflow: float
    newton_iters: int = 0
    krylov_iters: int = 0
    ms_newton: float = 0.0
    ms_guess: float = 0.0
    res_plain: float = 0.0
    res_guess: float = 0.0
    used_guess: object = False    # True (the proposed guess), "extrapolation" or False (plain)
    res_hist: tuple = ()
    x_ex: Optional[torch.Tensor] = None     # extrapolated guess 2 x^{n-1} - x^{n-2} of this step
    R_ex: Optional[torch.Tensor] = None     # its residual
    rn_ex: float = 0.0
    s: Optional[torch.Tensor] = None        # interface scaling field of this step
    u_prev: Optional[torch.Tensor] = None   # velocity the step started from
    phases_ms: tuple = ()                   # Newton call: (residuals, preconditioner setups, Krylov solves)
    xdot: Optional[torch.Tensor] = None     # rates at this state (generalized-alpha)


class ChannelRun:
    def __init__(self, cfg, device="cuda", inner=torch.float32, eta=1e-3, restart=50,
                 rel_tol=1e-8, period=0.8, amp_deg=20.0, max_krylov=4000, precond="bjacobi",
                 integrator="be", rho_inf=0.5, vel_steps=0, tangent="picard", pc_reuse=False,
                 basis32=False):
        self.cfg = cfg
        self.precond = precond
        self.vel_steps = vel_steps
        self.tangent = tangent
        self.pc_reuse = pc_reuse   # build the preconditioner once per step (at the guess) and reuse it
        self.basis32 = basis32     # FP32 inner solves keep their Krylov basis in FP32
        # time integrator: backward Euler, or generalized-alpha (section 2.4) in stage variables:
        # the stage residual at t_n + alpha_f dt is the backward-Euler-form residual with mass
        # coefficient alpha_m / (gamma dt alpha_f) and source c V_n - (1 - alpha_m/gamma) Vdot_n;
        # velocity and pressure are then advanced through their rates
        if integrator == "be":
            self.coefs = (1.0, 1.0, 1.0)
        elif integrator == "genalpha":
            am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf)
            af = 1.0 / (1.0 + rho_inf)
            self.coefs = (am, af, 0.5 + am - af)
        else:
            raise ValueError(f"unknown integrator {integrator!r}")
        self.integrator = integrator
        self.g = cfg.grid
        self.N = self.g.num_nodes
        self.dev = torch.device(device)
        self.inner, self.eta, self.restart, self.rel_tol = inner, eta, restart, rel_tol
        self.max_krylov = max_krylov
        self.period, self.amp = period, amp_deg
        self.prm = make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
        am, af, gm = self.coefs
        self.c_stage = cfg.c_m if integrator == "be" else am / (gm * cfg.dt * af)
        self.prm_stage = make_params(cfg.nu, self.c_stage, cfg.dt, cfg.C_T, cfg.C_I)
        g = self.g
        mask = W.channel_dirichlet_mask(g)
        self.mask = torch.tensor(W.mask_to_bits(mask).view(np.int32), device=self.dev)
        self.inflow_pattern = torch.tensor(W.channel_inflow_pattern(g).ravel(), dtype=torch.float64,
                                           device=self.dev)
        self.gD = torch.zeros(3 * self.N, dtype=torch.float64, device=self.dev)
        self.f = torch.zeros(3 * self.N, dtype=torch.float64, device=self.dev)
        self.zero_out = torch.zeros(self.N * 32, dtype=torch.float32, device=self.dev)
        self.x = torch.zeros(4 * self.N, dtype=torch.float64, device=self.dev)
        self.xdot = torch.zeros(4 * self.N, dtype=torch.float64, device=self.dev)   # rates (generalized-alpha)
        self.R = torch.empty_like(self.x)
        self.n = 0
        self.record_extrap = False
        self.kappa = None
        self.history: List[StepRecord] = []
        self.newton_ws = None
        self.m = cfg.m_points
        vol = W.plate_volume()
        kap = W.kappa_weights(self.m, vol, cfg.c_m, cfg.alpha)
        self.kappa64 = torch.tensor(kap, dtype=torch.float64, device=self.dev)
        self.kappa32 = torch.tensor(kap, dtype=torch.float32, device=self.dev)
        self.history.append(StepRecord(0, 0.0, self.x.clone(), torch.zeros(3 * self.N, dtype=torch.float64,
                                                                            device=self.dev),
                                       torch.zeros(3 * self.N, dtype=torch.float64, device=self.dev), 0.0))

    def restore(self, k):
        """Go back to the recorded state k (to re-solve the next step another way)."""
        self.x = self.history[k].x.clone()
        if self.history[k].xdot is not None:
            self.xdot = self.history[k].xdot.clone()
        elif k == 0:
            self.xdot.zero_()
        self.n = k

    def checkpoint(self, path):
        """Write the state needed to continue the run (step index, x, the rates and the last
        states the extrapolated guesses use) to an .npz file (plain arrays, no pickles)."""
        keep = self.history[-3:]
        np.savez(path, n=np.int64(self.n), x=self.x.cpu().numpy(), xdot=self.xdot.cpu().numpy(),
                 hist_n=np.array([r.n for r in keep], dtype=np.int64),
                 hist_t=np.array([r.t for r in keep], dtype=np.float64),
                 hist_x=np.stack([r.x.cpu().numpy() for r in keep]),
                 hist_inflow=np.array([r.inflow for r in keep], dtype=np.float64),
                 integrator=np.array(self.integrator), coefs=np.array(self.coefs, dtype=np.float64))

    def resume(self, path):
        """Continue from a checkpoint of the same configuration: the next step is bitwise the
        one the uninterrupted run takes (the library's kernels are deterministic)."""
        with np.load(path, allow_pickle=False) as d:
            if str(d["integrator"]) != self.integrator or not np.array_equal(d["coefs"], np.array(self.coefs)):
                raise ValueError("checkpoint of another time integrator")
            if d["x"].size != 4 * self.N:
                raise ValueError("checkpoint of another grid")
            self.n = int(d["n"])
            self.x = torch.tensor(d["x"], dtype=torch.float64, device=self.dev)
            self.xdot = torch.tensor(d["xdot"], dtype=torch.float64, device=self.dev)
            self.history = []
            for k in range(d["hist_n"].size):
                xk = torch.tensor(d["hist_x"][k], dtype=torch.float64, device=self.dev)
                self.history.append(StepRecord(int(d["hist_n"][k]), float(d["hist_t"][k]), xk, None, None,
                                               float(d["hist_inflow"][k])))
            # history is indexed by step number: pad the steps that were not kept
            first = int(d["hist_n"][0]) if d["hist_n"].size else self.n
            self.history = [None] * first + self.history

    def inflow_value(self, t):
        return W.channel_inflow_value(t, self.period)

    def _points(self, t):
        X, gp = W.rotating_plate_points(self.m, self.cfg.seed_fields, t, period=self.period,
                                        amp_deg=self.amp)
        Xt = torch.tensor(X.ravel(), dtype=torch.float64, device=self.dev)
        gt = torch.tensor(gp.ravel(), dtype=torch.float64, device=self.dev)
        tab64 = dlm_locate(self.g, Xt, dtype=torch.float64, s_max=self.cfg.s_max)
        tab32 = dlm_locate(self.g, Xt, dtype=torch.float32, s_max=self.cfg.s_max)
        gram64 = dlm_gram(self.g, tab64, self.kappa64)
        gram32 = dlm_gram(self.g, tab32, self.kappa32)
        lamg = torch.zeros(3 * self.N, dtype=torch.float64, device=self.dev)
        dlm_BT(self.g, tab64, gt, lamg, kappa=self.kappa64)
        P64 = Problem(self.g, self.prm_stage, self.x, tab64, self.kappa64, s=tab64.s, mask=self.mask,
                      gram=gram64)
        a32 = torch.zeros(3 * self.N, dtype=torch.float32, device=self.dev)
        P32 = Problem(self.g, self.prm_stage, a32, tab32, self.kappa32, s=tab32.s, mask=self.mask,
                      gram=gram32)
        return P64, P32, lamg, gt, tab64

    def residual_norm(self, P64, x, lamg):
        vms_residual(P64, self.f, x, gD=self.gD, lamg=lamg, R=self.R)
        return norm2(self.R)

    def btlam(self, tab64, gt, x):
        """B^T lambda with lambda = kappa (g - B u) (the paper's lambda = -R^s for the stand-in)."""
        Bu = dlm_B(self.g, tab64, x[: 3 * self.N])
        lam = gt.clone()
        axpby(-1.0, Bu, 1.0, lam)
        out = torch.zeros(3 * self.N, dtype=torch.float64, device=self.dev)
        dlm_BT(self.g, tab64, lam, out, kappa=self.kappa64)
        return out

    def step(self, guess_fn: Optional[Callable] = None, inner=None, record=True, precond=None, vel_steps=None,
             tangent=None, pc_reuse=None):
        """Advance one step.  guess_fn(run, ctx) -> FP64 [4][N] guess or None; ctx holds the
        step's FP64 problem, lamg, the inflow value, s and the extrapolated guess with its
        residual (x_ex, R_ex, rn_ex; None before two states exist)."""
        cfg = self.cfg
        n1 = self.n + 1
        t1 = n1 * cfg.dt
        am, af, gm = self.coefs
        be = self.integrator == "be"
        # stage time, solid kinematics and Dirichlet data (t_{n+1} for backward Euler)
        t_s = t1 if be else self.n * cfg.dt + af * cfg.dt
        P64, P32, lamg, gt, tab64 = self._points(t_s)
        inflow = self.inflow_value(t1) if be else \
            (1.0 - af) * self.inflow_value(self.n * cfg.dt) + af * self.inflow_value(t1)
        axpby(inflow, self.inflow_pattern, 0.0, self.gD)
        axpby(self.c_stage, self.x[: 3 * self.N], 0.0, self.f)
        if not be:
            axpby(-(1.0 - am / gm), self.xdot[: 3 * self.N], 1.0, self.f)
        torch.cuda.synchronize()
        t_g0 = time.perf_counter()
        # plain guess: previous state with the new Dirichlet values
        x_plain = torch.empty_like(self.x)
        ws.unpack(self.N, 32, self.zero_out, self.x, [0, 0, 0, 0], [1, 1, 1, 1], x_plain,
                  mask=self.mask, gD=self.gD)
        r_plain = self.residual_norm(P64, x_plain, lamg)
        tol = self.rel_tol * r_plain
        x0, r_guess, used = x_plain, r_plain, False
        # second-order extrapolation 2 x^n - x^{n-1} and its residual (backbone of the learned guess)
        ctx = {"P64": P64, "lamg": lamg, "inflow": inflow, "s": P64.s, "x_ex": None, "R_ex": None,
               "rn_ex": 0.0}
        if self.n >= 1 and (guess_fn is not None or self.record_extrap):
            # linear extrapolation of the state to the stage time: x^n + alpha_f (x^n - x^{n-1})
            x_ex = torch.empty_like(self.x)
            axpby(1.0 + af, self.history[self.n].x, 0.0, x_ex)
            axpby(-af, self.history[self.n - 1].x, 1.0, x_ex)
            ws.unpack(self.N, 32, self.zero_out, x_ex.clone(), [0, 0, 0, 0], [1, 1, 1, 1], x_ex,
                      mask=self.mask, gD=self.gD)
            ctx["rn_ex"] = self.residual_norm(P64, x_ex, lamg)
            ctx["x_ex"], ctx["R_ex"] = x_ex, self.R.clone()
        if guess_fn is not None:
            xg = guess_fn(self, ctx)
            if xg is not None:
                # safeguard: keep the candidate with the smallest residual among the plain guess,
                # the extrapolation (its residual is already known) and the proposed guess
                r_g = r_guess = self.residual_norm(P64, xg, lamg)
                if ctx["x_ex"] is not None and xg is not ctx["x_ex"] and ctx["rn_ex"] < r_plain and \
                        not (math.isfinite(r_g) and r_g <= ctx["rn_ex"]):
                    x0, r_guess, used = ctx["x_ex"], ctx["rn_ex"], "extrapolation"
                elif math.isfinite(r_g) and r_g < r_plain:
                    x0, used = xg, True
        torch.cuda.synchronize()
        ms_guess = (time.perf_counter() - t_g0) * 1e3
        inner = inner if inner is not None else self.inner
        opts = newton_opts(tol_abs=tol, eta=self.eta, restart=self.restart,
                           max_krylov=self.max_krylov, inner=inner,
                           precond=precond if precond is not None else self.precond,
                           vel_steps=vel_steps if vel_steps is not None else self.vel_steps,
                           tangent=tangent if tangent is not None else self.tangent,
                           pc_reuse=pc_reuse if pc_reuse is not None else self.pc_reuse,
                           basis=torch.float32 if self.basis32 and inner == torch.float32 else torch.float64)
        x_new = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = newton_solve(P64, self.f, x_new, opts, P32=P32 if inner == torch.float32 else None,
                              lamg=lamg, gD=self.gD, check=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if rc != 0:
            raise RuntimeError(f"Newton failed at step {n1} (status {rc}, iters {st.newton_iters}, "
                               f"hist {list(st.res_hist[:st.newton_iters + 1])})")
        x_stage = x_new
        if not be:
            # X_{n+1} = X_n + (X_stage - X_n) / alpha_f; Xdot_{n+1} = Xdot_n + (X_{n+1} - X_n - dt Xdot_n) / (gamma dt)
            x_new = self.x.clone()
            axpby(1.0 / af, x_stage, 1.0 - 1.0 / af, x_new)
            xd = self.xdot.clone()
            axpby(1.0 / (gm * cfg.dt), x_new, 1.0 - 1.0 / gm, xd)
            axpby(-1.0 / (gm * cfg.dt), self.x, 1.0, xd)
            self.xdot = xd
        rec = StepRecord(n1, t1, x_new, self.btlam(tab64, gt, x_stage) if record else None, lamg,
                         inflow, st.newton_iters, st.krylov_iters, ms, ms_guess, r_plain, r_guess, used,
                         tuple(st.res_hist[: min(st.newton_iters + 1, 32)]),
                         phases_ms=(round(st.t_residual_ms, 2), round(st.t_setup_ms, 2), round(st.t_krylov_ms, 2)))
        if record and self.record_extrap:
            rec.x_ex, rec.R_ex, rec.rn_ex = ctx["x_ex"], ctx["R_ex"], ctx["rn_ex"]
            rec.s = P64.s.clone()
            rec.u_prev = self.history[self.n].x[: 3 * self.N].clone()
        rec.xdot = self.xdot.clone() if not be else None
        self.x = x_new
        self.n = n1
        if record:
            self.history.append(rec)
        return rec
