"""Generalized-alpha time stepping of the fluid system (test infrastructure only).

Section 2.4 integrates in time with the implicit, second-order generalized-alpha
method (the variant that keeps the pressure second order) and solves, per step,
Newton corrections for the velocity and pressure rates.  The paper prints no
formulas for it; this module takes the following reading:

* parameters from the spectral radius rho_inf at infinity (first-order systems):
  alpha_m = (3 - rho_inf) / (2 (1 + rho_inf)), alpha_f = 1 / (1 + rho_inf),
  gamma = 1/2 + alpha_m - alpha_f;
* both fields, velocity V and pressure P, are advanced through their rates:
  X_{n+1} = X_n + dt Xdot_n + gamma dt (Xdot_{n+1} - Xdot_n);
* the residual is evaluated at the stage: X_{n+alpha_f} = X_n + alpha_f (X_{n+1} - X_n)
  for V and P, Vdot_{n+alpha_m} = Vdot_n + alpha_m (Vdot_{n+1} - Vdot_n), the solid
  kinematics and the Dirichlet data at t_n + alpha_f dt.

Eliminating the rates, Vdot_{n+alpha_m} = c V_{n+alpha_f} - (c V_n - (1 - alpha_m/gamma) Vdot_n)
with c = alpha_m / (gamma dt alpha_f).  The stage residual in the unknowns
(V_{n+alpha_f}, P_{n+alpha_f}) is therefore the backward-Euler-form residual
(oracle.newton.residual) with mass coefficient c_m = c and nodal source
c V_n - (1 - alpha_m/gamma) Vdot_n, and Newton in the stage unknowns takes the same
iterates as Newton in the rates (the two Jacobians differ by the factor
alpha_f gamma dt).  The stabilisation keeps its own dt (the tau_m bracket), so
the semi-discrete system does not change with the time step.
(alpha_m, alpha_f, gamma) = (1, 1, 1) is backward Euler.
"""
from __future__ import annotations

import numpy as np

from . import newton


def coefficients(rho_inf):
    am = 0.5 * (3.0 - rho_inf) / (1.0 + rho_inf)
    af = 1.0 / (1.0 + rho_inf)
    return am, af, 0.5 + am - af


def stage_mass(coefs, dt):
    am, af, gm = coefs
    return am / (gm * dt * af)


def stage_source(coefs, dt, v_n, vdot_n):
    """Nodal source of the stage residual: c V_n - (1 - alpha_m/gamma) Vdot_n ([3][N])."""
    am, af, gm = coefs
    c = stage_mass(coefs, dt)
    return c * np.asarray(v_n) - (1.0 - am / gm) * np.asarray(vdot_n)


def update(coefs, dt, x_n, xdot_n, x_stage):
    """(X_{n+1}, Xdot_{n+1}) from the converged stage values (all [4][N])."""
    am, af, gm = coefs
    x_n = np.asarray(x_n)
    xdot_n = np.asarray(xdot_n)
    x1 = x_n + (np.asarray(x_stage) - x_n) / af
    xdot1 = xdot_n + (x1 - x_n - dt * xdot_n) / (gm * dt)
    return x1, xdot1


def step(grid, prm, coefs, dt, x_n, xdot_n, cell, xi, kappa, g_stage, s=None, mask=None,
         gD_stage=None, x0=None, tol_abs=None, rel=1e-8, max_newton=20):
    """One step: Newton (dense) on the stage residual from x0 (default: x_n with the stage
    Dirichlet values), then the rate updates.  prm: the operator parameters [nu, c_m, dt_tau,
    C_T, C_I]; its c_m is replaced by the stage mass coefficient.  Returns
    (x_{n+1}, xdot_{n+1}, x_stage, info)."""
    N = grid.num_nodes
    x_n = np.asarray(x_n, dtype=np.float64).reshape(4, N)
    xdot_n = np.asarray(xdot_n, dtype=np.float64).reshape(4, N)
    c = stage_mass(coefs, dt)
    p2 = np.array(prm, dtype=np.float64).copy()
    p2[1] = c
    body = -(1.0 - coefs[0] / coefs[2]) * xdot_n[:3]
    if x0 is None:
        x0 = x_n.copy()
        if mask is not None:
            m = np.asarray(mask, dtype=bool).reshape(3, N)
            x0[:3][m] = np.asarray(gD_stage).reshape(3, N)[m]
    xs, info = newton.solve_step(grid, p2, x0, x_n[:3], cell, xi, kappa, g_stage, s=s, mask=mask,
                                 gD=gD_stage, tol_abs=tol_abs, rel=rel, max_newton=max_newton,
                                 body=body)
    x1, xdot1 = update(coefs, dt, x_n, xdot_n, xs)
    return x1, xdot1, xs, info
