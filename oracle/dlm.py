"""FP64 reference of the DLM coupling (test infrastructure only).

Section 2.3: with delta-function multiplier basis functions at the solid
points, the constraint becomes nodal interpolation of the fluid velocity at
each solid point, (B u)_B = sum_A N_A(phi(X_B)) u_A (eq. nodal_solid_velo),
and the force spreading operator is C^lambda_AB = N_A(phi(X_B)) I
(eq. fsi_constraint_matrix), i.e. (B^T lambda)_A = sum_B N_A(X_B) lambda_B.
Appendix A's per-point steps are: find the containing element and the
parametric position xi of each point, then evaluate the fluid shape functions
of that element at xi.

Reading of the cell rule (points on faces or outside are not specified):
breakpoints b_k = x0 + k h (FP64 as written); a point belongs to cell i if
b_i <= X <= b_{i+1}; among several such cells the largest index is taken, and
a coordinate outside [b_0, b_n] marks the point as outside (cell -1).
xi_d = (X_d - (x0_d + i_d h_d)) / h_d.
"""
from __future__ import annotations

import numpy as np


def _axis_break(x0, h, k):
    return x0 + np.asarray(k, dtype=np.float64) * h


def locate_bruteforce(grid, X):
    """Every point against every cell; O(M E).  Returns (cell[M] int64, xi[3][M])."""
    X = np.asarray(X, dtype=np.float64).reshape(3, -1)
    M = X.shape[1]
    nx, ny, nz = grid.n
    cell = np.full(M, -1, dtype=np.int64)
    idx = np.full((3, M), -1, dtype=np.int64)
    for b in range(M):
        best = None
        for cz in range(nz):
            for cy in range(ny):
                for cx in range(nx):
                    ok = True
                    for d, c in enumerate((cx, cy, cz)):
                        lo = grid.x0[d] + float(c) * grid.h[d]
                        hi = grid.x0[d] + float(c + 1) * grid.h[d]
                        if not (lo <= X[d, b] <= hi):
                            ok = False
                            break
                    if ok:
                        cand = (cx, cy, cz)
                        if best is None:
                            best = list(cand)
                        else:
                            best = [max(best[d], cand[d]) for d in range(3)]
        if best is not None:
            idx[:, b] = best
            cell[b] = best[0] + nx * (best[1] + ny * best[2])
    xi = np.zeros((3, M))
    for d in range(3):
        inside = cell >= 0
        lo = grid.x0[d] + idx[d, inside].astype(np.float64) * grid.h[d]
        xi[d, inside] = (X[d, inside] - lo) / grid.h[d]
    return cell, xi


def locate(grid, X):
    """Same rule as locate_bruteforce, per axis by searching the breakpoints. O(M log n)."""
    X = np.asarray(X, dtype=np.float64).reshape(3, -1)
    M = X.shape[1]
    idx = np.zeros((3, M), dtype=np.int64)
    inside = np.ones(M, dtype=bool)
    for d in range(3):
        n = grid.n[d]
        b = _axis_break(grid.x0[d], grid.h[d], np.arange(n + 1))
        # largest k with b_k <= X, then clamp to the last cell
        k = np.searchsorted(b, X[d], side="right") - 1
        inside &= (X[d] >= b[0]) & (X[d] <= b[n])
        idx[d] = np.clip(k, 0, n - 1)
    cell = np.where(inside, idx[0] + grid.n[0] * (idx[1] + grid.n[1] * idx[2]), -1)
    xi = np.zeros((3, M))
    for d in range(3):
        lo = grid.x0[d] + idx[d].astype(np.float64) * grid.h[d]
        xi[d] = np.where(inside, (X[d] - lo) / grid.h[d], 0.0)
    return cell.astype(np.int64), xi


def sort_by_cell(grid, cell):
    """Stable order of the points by cell, outside points last.

    Returns (perm, occ_cell, occ_start): perm lists point indices, occupied
    cells ascending, occ_start[k]..occ_start[k+1] the range of perm in cell k.
    """
    cell = np.asarray(cell, dtype=np.int64)
    E = grid.num_cells
    key = np.where(cell >= 0, cell, E)
    perm = np.argsort(key, kind="stable")
    inside = cell[perm] >= 0
    sorted_cells = cell[perm][inside]
    occ_cell, first = np.unique(sorted_cells, return_index=True)
    occ_start = np.append(first, sorted_cells.size)
    return perm.astype(np.int64), occ_cell.astype(np.int64), occ_start.astype(np.int64)


def s_field(grid, cell, s_max):
    """Interface scaling s (section 2.1): s_max on every node of a cell holding a solid point, else 1."""
    N = grid.num_nodes
    s = np.ones(N)
    p = grid.order
    q = p + 1
    Nx, Ny, _ = grid.nodes_per_axis
    occ = np.unique(np.asarray(cell)[np.asarray(cell) >= 0])
    cx = occ % grid.n[0]
    cy = (occ // grid.n[0]) % grid.n[1]
    cz = occ // (grid.n[0] * grid.n[1])
    for az in range(q):
        for ay in range(q):
            for ax in range(q):
                s[(p * cx + ax) + Nx * ((p * cy + ay) + Ny * (p * cz + az))] = s_max
    return s


def _lagrange1d(p, t):
    t = np.asarray(t, dtype=np.float64)
    if p == 1:
        return np.stack([1.0 - t, t])
    return np.stack([2.0 * (t - 0.5) * (t - 1.0), -4.0 * t * (t - 1.0), 2.0 * t * (t - 0.5)])


def point_shapes(grid, cell, xi):
    """Shape values N_A(xi_B) and node ids of the containing cell: ([nen][M], [nen][M])."""
    p = grid.order
    q = p + 1
    cell = np.asarray(cell, dtype=np.int64)
    Nx, Ny, _ = grid.nodes_per_axis
    inside = cell >= 0
    c = np.where(inside, cell, 0)
    cx = c % grid.n[0]
    cy = (c // grid.n[0]) % grid.n[1]
    cz = c // (grid.n[0] * grid.n[1])
    Lx, Ly, Lz = (_lagrange1d(p, xi[d]) for d in range(3))
    vals, ids = [], []
    for az in range(q):
        for ay in range(q):
            for ax in range(q):
                vals.append(np.where(inside, Lx[ax] * Ly[ay] * Lz[az], 0.0))
                ids.append((p * cx + ax) + Nx * ((p * cy + ay) + Ny * (p * cz + az)))
    return np.stack(vals), np.stack(ids)


def apply_B(grid, cell, xi, u):
    """(B u)_B = sum_A N_A(xi_B) u_A for each of the 3 components ([3][N] -> [3][M])."""
    vals, ids = point_shapes(grid, cell, xi)
    u = np.asarray(u, dtype=np.float64).reshape(3, -1)
    out = np.zeros((3, vals.shape[1]))
    for A in range(vals.shape[0]):
        out += vals[A] * u[:, ids[A]]
    return out


def apply_BT(grid, cell, xi, lam, kappa=None):
    """(B^T (kappa lam))_A = sum_B N_A(xi_B) kappa_B lam_B ([3][M] -> [3][N])."""
    vals, ids = point_shapes(grid, cell, xi)
    lam = np.asarray(lam, dtype=np.float64).reshape(3, -1)
    if kappa is not None:
        lam = lam * np.asarray(kappa, dtype=np.float64)[None, :]
    out = np.zeros((3, grid.num_nodes))
    for A in range(vals.shape[0]):
        for d in range(3):
            np.add.at(out[d], ids[A], vals[A] * lam[d])
    return out


def dense_B(grid, cell, xi):
    """Scalar interpolation matrix Bs (M x N); the 3-component B is kron(I3, Bs)."""
    vals, ids = point_shapes(grid, cell, xi)
    M = vals.shape[1]
    Bs = np.zeros((M, grid.num_nodes))
    for A in range(vals.shape[0]):
        np.add.at(Bs, (np.arange(M), ids[A]), vals[A])
    return Bs


def dlm_diag(grid, cell, xi, kappa):
    """Diagonal of B^T diag(kappa) B per node: sum_B kappa_B N_A(xi_B)^2 ([N])."""
    vals, ids = point_shapes(grid, cell, xi)
    out = np.zeros(grid.num_nodes)
    for A in range(vals.shape[0]):
        np.add.at(out, ids[A], np.asarray(kappa) * vals[A] ** 2)
    return out
