"""Reduced block system of section 2.4 with the per-point solid stand-in (test infrastructure).

The paper eliminates the multiplier with its nodal definition (eq.
nodal_lagrange) and the solid velocity with eq. nodal_solid_velo, leaving a
fluid-sized 2x2 block system whose momentum-momentum block is
dR^{f,m}/dV + C^lambda dR^s/dU (C^lambda)^T.  The solid tangent is replaced
here by a per-point diagonal stand-in kappa_B I, so with B = (C^lambda)^T:

    J = A_VMS + [[B^T diag(kappa) B, 0], [0, 0]]

Dirichlet velocity DOFs: their columns are zero and their rows the identity
(the guess carries the prescribed values, so corrections there vanish).
"""
from __future__ import annotations

import numpy as np

from . import dlm, vms


def apply(grid, prm, a, x, cell, xi, kappa, s=None, mask=None, visc_strong=True):
    """J x ([4][N]) by the oracle's own element matrices and point-by-point DLM."""
    N = grid.num_nodes
    x = np.asarray(x, dtype=np.float64).reshape(4, N)
    xm = x.copy()
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        xm[:3][m] = 0.0
    y = vms.apply(grid, prm, a, xm, s=s, mask=None, visc_strong=visc_strong)
    Bu = dlm.apply_B(grid, cell, xi, xm[:3])
    y[:3] += dlm.apply_BT(grid, cell, xi, Bu, kappa)
    if mask is not None:
        y[:3][m] = x[:3][m]
    return y


def dense(grid, prm, a, cell, xi, kappa, s=None, mask=None, visc_strong=True):
    """Dense J (small grids only), same DOF order as the [4][N] vectors."""
    N = grid.num_nodes
    A = vms.assemble_dense(grid, prm, a, s=s, visc_strong=visc_strong)
    Bs = dlm.dense_B(grid, cell, xi)
    D = Bs.T @ (np.asarray(kappa)[:, None] * Bs)
    for f in range(3):
        A[f * N:(f + 1) * N, f * N:(f + 1) * N] += D
    if mask is not None:
        m = np.concatenate([np.asarray(mask, dtype=bool).reshape(-1), np.zeros(N, dtype=bool)])
        A[:, m] = 0.0
        A[m, :] = 0.0
        A[m, m] = 1.0
    return A


def diag_blocks(grid, prm, a, cell, xi, kappa, s=None, mask=None, visc_strong=True):
    """Nodal 4x4 diagonal blocks of J ([N][4][4]); Dirichlet rows/cols -> identity."""
    blocks = vms.diag_blocks(grid, prm, a, s=s, mask=None, visc_strong=visc_strong)
    d = dlm.dlm_diag(grid, cell, xi, kappa)
    for f in range(3):
        blocks[:, f, f] += d
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, -1)
        for f in range(3):
            sel = m[f]
            blocks[sel, f, :] = 0.0
            blocks[sel, :, f] = 0.0
            blocks[sel, f, f] = 1.0
    return blocks


def block_jacobi_apply(blocks, v):
    """z = P^{-1} v with P the nodal 4x4 blocks (solved per node in FP64)."""
    N = blocks.shape[0]
    v = np.asarray(v, dtype=np.float64).reshape(4, N)
    z = np.linalg.solve(blocks, v.T[:, :, None])[:, :, 0]
    return z.T.copy()
