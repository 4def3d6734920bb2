"""Time steps of the channel with the hyperelastic solid moving with the fluid.

Host-side orchestration of library calls (every arithmetic step runs in the library's
kernels: locate, the step residual with the solid, Newton, fsi_axpby for the state updates).
Section 2.4: each step solves the monolithic system by Newton; the solid velocity is the
fluid's at the solid nodes (eq. nodal_solid_velo) and the multiplier is eliminated by eq.
nodal_lagrange.  Backward Euler, or generalized-alpha in stage unknowns: the fluid's velocity
and pressure advance through their rates (mass coefficient c = alpha_m / (gamma dt alpha_f),
source c X_n - (1 - alpha_m / gamma) Xdot_n), the solid velocity Vs through its rate and the
displacement U through Vs with the same gamma, so that at the stage U = U_base + gamma dt Vs
and A = c Vs - A_base with U_base = U_n + (alpha_f - gamma) dt Vs_n and
A_base = c Vs_n - (1 - alpha_m / gamma) Vsdot_n.
"""
from __future__ import annotations

import time

import numpy as np
import torch

import fsi_workloads as W

from . import (Problem, Solid, axpby, dlm_gram, dlm_locate, make_params, newton_opts, newton_solid_solve, norm2,
               solid_step_residual)


def ga_coefficients(rho_inf):
    """(alpha_m, alpha_f, gamma) of generalized-alpha for first-order systems."""
    am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf)
    af = 1.0 / (1.0 + rho_inf)
    return am, af, 0.5 + am - af


class SolidChannel:
    """The channel of the configuration `cfg` (Dirichlet: inflow u_x = `inflow` on x = 0, no-slip
    walls) with a solid mesh (X0 [3][M], conn [E][8]) that starts at rest and stress free."""

    def __init__(self, cfg, X0, conn, integrator="be", rho_inf=0.5, precond="schur_tri", vel_steps=8,
                 inner="f32", inflow=1.0, kappa=None, rel_tol=1e-8, max_krylov=6000, gravity=None,
                 basis32=False):
        dev = torch.device("cuda")
        self.cfg, self.g = cfg, cfg.grid
        self.dev = dev
        self.basis32 = basis32   # FP32 inner solves keep their Krylov basis in FP32
        g = self.g
        N = g.num_nodes
        self.N, self.M = N, X0.shape[1]
        self.coefs = (1.0, 1.0, 1.0) if integrator == "be" else ga_coefficients(rho_inf)
        self.precond, self.vel_steps, self.rel_tol, self.max_krylov = precond, vel_steps, rel_tol, max_krylov
        self.inner = torch.float32 if inner == "f32" else torch.float64
        self.X0 = torch.tensor(np.ascontiguousarray(X0).ravel(), dtype=torch.float64, device=dev)
        self.solid = Solid(self.X0, torch.tensor(np.ascontiguousarray(conn).ravel(), dtype=torch.int32, device=dev),
                           **W.SOLID_MATERIAL)
        mask = W.channel_dirichlet_mask(g)
        self.mask_bits = torch.tensor(W.mask_to_bits(mask).view(np.int32), device=dev)
        inflow_nodes = np.arange(N) % g.nodes_per_axis[0] == 0
        gD = np.zeros((3, N))
        gD[0][inflow_nodes & ~(mask[0] & ~inflow_nodes)] = inflow
        self.gD = torch.tensor(gD.ravel(), dtype=torch.float64, device=dev)
        x = np.zeros((4, N))
        x[:3][mask] = gD[mask]
        self.x = torch.tensor(x.ravel(), dtype=torch.float64, device=dev)
        self.xdot = torch.zeros(4 * N, dtype=torch.float64, device=dev)
        self.U = torch.zeros(3 * self.M, dtype=torch.float64, device=dev)
        self.Vs = torch.zeros(3 * self.M, dtype=torch.float64, device=dev)
        self.Vsdot = torch.zeros(3 * self.M, dtype=torch.float64, device=dev)
        if kappa is None:
            mat = W.SOLID_MATERIAL
            kappa = np.full(self.M, cfg.c_m * (mat["rho_s0"] - mat["rho_f"]) * W.plate_volume() / self.M)
        self.kappa = np.asarray(kappa, dtype=np.float64)
        # a body force per unit mass on the solid (eq. solid_weak_form's (rho_s - rho_f)(A - f)):
        # it shifts the acceleration, A - f = c_A V - (A_base + f); the fluid's own weight is
        # balanced by the hydrostatic pressure and left out
        self.body = None
        if gravity is not None:
            self.body = torch.tensor(np.repeat(np.asarray(gravity, dtype=np.float64), self.M), device=dev)
        self.n = 0

    def _t(self, v, dt=torch.float64):
        return torch.tensor(np.ascontiguousarray(v).ravel(), dtype=dt, device=self.dev)

    def step(self):
        cfg, g, N, M = self.cfg, self.g, self.N, self.M
        am, af, gm = self.coefs
        dt = cfg.dt
        c = am / (gm * dt * af)
        r = 1.0 - am / gm
        t0 = time.perf_counter()
        # configuration of t_n
        Xc = self.X0.clone()
        axpby(1.0, self.U, 1.0, Xc)
        prm = make_params(cfg.nu, c, dt, cfg.C_T, cfg.C_I)
        probs = []
        for tdt in ([torch.float64] + ([torch.float32] if self.inner == torch.float32 else [])):
            tab = dlm_locate(g, Xc, dtype=tdt, s_max=cfg.s_max)
            kt = self._t(self.kappa, tdt)
            probs.append(Problem(g, prm, torch.zeros(3 * N, dtype=tdt, device=self.dev), tab, kt, s=tab.s,
                                 mask=self.mask_bits, gram=dlm_gram(g, tab, kt)))
        # fluid source and the solid's affine state at the stage
        f = torch.empty(3 * N, dtype=torch.float64, device=self.dev)
        axpby(c, self.x[:3 * N], 0.0, f)
        axpby(-r, self.xdot[:3 * N], 1.0, f)
        Ub = self.U.clone()
        axpby((af - gm) * dt, self.Vs, 1.0, Ub)
        Ab = torch.empty_like(self.Vs)
        axpby(c, self.Vs, 0.0, Ab)
        axpby(-r, self.Vsdot, 1.0, Ab)
        if self.body is not None:
            axpby(1.0, self.body, 1.0, Ab)
        state = (Ub, Ab, gm * dt, c)
        x_st = self.x.clone()
        R0, _, _ = solid_step_residual(probs[0], self.solid, state, f, x_st, gD=self.gD)
        tol = self.rel_tol * norm2(R0)
        torch.cuda.synchronize()
        t_setup = (time.perf_counter() - t0) * 1e3
        U_st = torch.empty_like(self.U)
        Vs_st = torch.empty_like(self.Vs)
        opts = newton_opts(tol, max_newton=30, inner=self.inner, precond=self.precond, vel_steps=self.vel_steps,
                           max_krylov=self.max_krylov,
                           basis=torch.float32 if self.basis32 and self.inner == torch.float32 else torch.float64)
        t1 = time.perf_counter()
        rc, st = newton_solid_solve(probs[0], self.solid, state, f, x_st, U_st, Vs_st, opts,
                                    P32=probs[1] if self.inner == torch.float32 else None, gD=self.gD, check=False)
        # rate updates: X1 = X + (X_st - X)/af, Xdot1 = Xdot + (X1 - X - dt Xdot)/(gm dt) for the fluid
        # and for the solid velocity, U1 = U + dt Vs + gm dt (Vs1 - Vs)
        for X, Xd, Xs in ((self.x, self.xdot, x_st), (self.Vs, self.Vsdot, Vs_st)):
            X1 = X.clone()
            axpby(1.0 / af, Xs, 1.0 - 1.0 / af, X1)
            axpby(1.0 / (gm * dt), X1, 1.0 - 1.0 / gm, Xd)
            axpby(-1.0 / (gm * dt), X, 1.0, Xd)
            if X is self.Vs:
                axpby((1.0 - gm) * dt, X, 1.0, self.U)
                axpby(gm * dt, X1, 1.0, self.U)
            X.copy_(X1)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3
        self.n += 1
        return {"step": self.n, "status": rc, "newton": st.newton_iters, "krylov": st.krylov_iters,
                "ms_newton": round(ms, 1), "ms_locate_setup": round(t_setup, 1),
                "ms_residuals": round(st.t_residual_ms, 1), "ms_setups": round(st.t_setup_ms, 1),
                "ms_krylov": round(st.t_krylov_ms, 1), "n_occupied_cells": probs[0].tables.n_occ,
                "tol": tol, "stage_x": x_st}
