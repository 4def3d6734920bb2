"""Textbook flexible GMRES (test infrastructure only).

Section 2.4 solves the reduced block system iteratively with block
preconditioners; the Krylov method itself is not printed, so this is Saad's
flexible GMRES with right preconditioning, restart m, modified Gram-Schmidt
and Givens rotations, in FP64.  Each restart cycle begins from the explicitly
computed residual b - J x; convergence is ||b - J x||_2 <= rtol ||b||_2 with
the explicit residual.
"""
from __future__ import annotations

import numpy as np


def fgmres(matvec, b, x0=None, precond=None, restart=50, rtol=1e-10, max_iters=1000):
    """Returns (x, info) with info = {'iters', 'cycles', 'res0', 'res', 'history'}."""
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    M = precond if precond is not None else (lambda v: v)
    bnorm = np.linalg.norm(b)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    info = {"iters": 0, "cycles": 0, "res0": beta, "res": beta, "history": [beta]}
    target = rtol * bnorm
    if beta <= target:
        return x, info
    while info["iters"] < max_iters:
        m = min(restart, max_iters - info["iters"])
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k_used = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            k_used = j + 1
            if abs(g[j + 1]) <= target or H[j, j] == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + Z[:k_used].T @ y
        info["cycles"] += 1
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        info["history"].append(beta)
        info["res"] = beta
        if beta <= target:
            break
    return x, info
