"""Nonlinear residual of one implicit step and Newton's method (test infrastructure only).

Section 2.4: each step solves the coupled nonlinear system with Newton's
method, each iteration solving the reduced block system.  Readings used here
(the paper's integrator is generalized-alpha; this reference uses backward
Euler, c_m = 1/dt):

  R(x) = A(a = u, tau(u)) x - F(u) + [B^T kappa (B u - g); 0]
  F(u) = Galerkin + SUPG + PSPG weighting of c_m u_old + f (f = 0 here)
  Dirichlet rows: R_D = u_D - g_D
  Newton matrix J(u_k) = A(a = u_k, tau(u_k)) + B^T kappa B (Picard / Oseen),
  Dirichlet rows identity, columns zero.
  Multiplier reported afterwards: lambda_B = kappa_B (g_B - (B u)_B), the
  paper's lambda = -R^s (eq. nodal_lagrange) for the stand-in solid residual.
  Full Newton tangent (tangent="full"): the derivative of R itself, including
  the reactive convection (du.grad)u, the linearised SUPG test function
  (du.grad)w and the derivatives of tau_m and tau_c, from the element tangents
  of vms_ref.c written out term by term; the DLM part is linear, so it keeps
  B^T kappa B; Dirichlet rows are the identity and Dirichlet columns zero.
"""
from __future__ import annotations

import numpy as np

from . import dlm, jacobian, krylov, vms


def residual(grid, prm, x, u_old, cell, xi, kappa, g, s=None, mask=None, gD=None,
             body=None, visc_strong=True):
    N = grid.num_nodes
    x = np.asarray(x, dtype=np.float64).reshape(4, N)
    c_m = float(prm[1])
    f = c_m * np.asarray(u_old, dtype=np.float64).reshape(3, N)
    if body is not None:
        f = f + np.asarray(body).reshape(3, N)
    R = vms.residual_fluid(grid, prm, x, f, s=s, visc_strong=visc_strong)
    Bu = dlm.apply_B(grid, cell, xi, x[:3])
    R[:3] += dlm.apply_BT(grid, cell, xi, Bu - np.asarray(g).reshape(3, -1), kappa)
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        gd = np.zeros((3, N)) if gD is None else np.asarray(gD).reshape(3, N)
        R[:3][m] = x[:3][m] - gd[m]
    return R


def multiplier(grid, x, cell, xi, kappa, g):
    N = grid.num_nodes
    Bu = dlm.apply_B(grid, cell, xi, np.asarray(x).reshape(4, N)[:3])
    return np.asarray(kappa)[None, :] * (np.asarray(g).reshape(3, -1) - Bu)


def tangent_apply(grid, prm, x, v, u_old, cell, xi, kappa, s=None, mask=None, body=None,
                  visc_strong=True):
    """Full Newton tangent of residual() at x times v ([4][N]; see the header)."""
    N = grid.num_nodes
    x = np.asarray(x, dtype=np.float64).reshape(4, N)
    v = np.asarray(v, dtype=np.float64).reshape(4, N)
    c_m = float(prm[1])
    f = c_m * np.asarray(u_old, dtype=np.float64).reshape(3, N)
    if body is not None:
        f = f + np.asarray(body).reshape(3, N)
    y = vms.tangent_apply(grid, prm, x, f, v, s=s, mask=mask, visc_strong=visc_strong)
    vm = v[:3].copy()
    m = None
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        vm[m] = 0.0
    dl = dlm.apply_BT(grid, cell, xi, dlm.apply_B(grid, cell, xi, vm), kappa)
    if m is not None:
        dl[m] = 0.0
    y[:3] += dl
    return y


def tangent_dense(grid, prm, x, u_old, cell, xi, kappa, s=None, mask=None, body=None,
                  visc_strong=True):
    """Dense full tangent (4N x 4N) by columns of tangent_apply (small grids only)."""
    n = 4 * grid.num_nodes
    J = np.empty((n, n))
    for j in range(n):
        e_j = np.zeros(n)
        e_j[j] = 1.0
        J[:, j] = tangent_apply(grid, prm, x, e_j, u_old, cell, xi, kappa, s, mask, body,
                                visc_strong).ravel()
    return J


def solve_step(grid, prm, x0, u_old, cell, xi, kappa, g, s=None, mask=None, gD=None,
               tol_abs=None, rel=1e-8, max_newton=20, linear="dense", eta=1e-3,
               visc_strong=True, restart=50, body=None, tangent="picard"):
    """Newton from x0 until ||R||_2 <= tol_abs (default rel * ||R(x0)||_2); body: an optional
    nodal source added to c_m u_old."""
    N = grid.num_nodes
    x = np.asarray(x0, dtype=np.float64).reshape(4, N).copy()
    hist = []
    lin_iters = []
    R = residual(grid, prm, x, u_old, cell, xi, kappa, g, s, mask, gD, body=body, visc_strong=visc_strong)
    r0 = np.linalg.norm(R)
    if tol_abs is None:
        tol_abs = rel * r0
    hist.append(r0)
    for _ in range(max_newton):
        if hist[-1] <= tol_abs:
            break
        a = x[:3].copy()
        if tangent == "full":
            J = tangent_dense(grid, prm, x, u_old, cell, xi, kappa, s, mask, body, visc_strong)
            dx = np.linalg.solve(J, -R.ravel())
            lin_iters.append(0)
        elif linear == "dense":
            J = jacobian.dense(grid, prm, a, cell, xi, kappa, s=s, mask=mask, visc_strong=visc_strong)
            dx = np.linalg.solve(J, -R.ravel())
            lin_iters.append(0)
        else:
            blocks = jacobian.diag_blocks(grid, prm, a, cell, xi, kappa, s=s, mask=mask,
                                          visc_strong=visc_strong)

            def mv(v):
                return jacobian.apply(grid, prm, a, v, cell, xi, kappa, s=s, mask=mask,
                                      visc_strong=visc_strong).ravel()

            def pc(v):
                return jacobian.block_jacobi_apply(blocks, v).ravel()

            b = -R.ravel()
            lin_tol = max(eta, 0.5 * tol_abs / max(np.linalg.norm(b), 1e-300))
            dx, info = krylov.fgmres(mv, b, precond=pc, restart=restart, rtol=lin_tol,
                                     max_iters=2000)
            lin_iters.append(info["iters"])
        x = x + dx.reshape(4, N)
        R = residual(grid, prm, x, u_old, cell, xi, kappa, g, s, mask, gD, body=body, visc_strong=visc_strong)
        hist.append(np.linalg.norm(R))
    return x, {"history": hist, "tol_abs": tol_abs, "linear_iters": lin_iters,
               "converged": hist[-1] <= tol_abs}
