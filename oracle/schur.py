"""Block preconditioner from the 2x2 sub-matrices of the reduced system (test infrastructure only).

Section 2.4 solves the reduced fluid-sized block system

    J = [[F, G], [D, C]]      (velocity rows first, then pressure rows)

with Krylov iterations preconditioned by block preconditioners built from its
sub-matrices (the paper names the family, not a member).  The member written
here is the block factorisation's upper factor

    P = [[F_hat, G], [0, S_hat]]          (right preconditioning)

or its block diagonal, with

* F_hat: the nodal 3x3 velocity blocks of J (the velocity part of the nodal
  4x4 diagonal blocks), inverted per node, optionally followed by k
  minimal-residual steps on F preconditioned by them (velocity_solve);
* S_hat ~ S = C - D F^{-1} G: because D = -G^T for the Galerkin terms, C is
  tau_m times a pressure Laplacian (PSPG) and F ~ c_m M + the DLM block, S acts
  like the variable-coefficient Laplacian  -div(alpha grad p)  with
  alpha = tau_m + 1 / (c_m + DLM density).  S_hat is that Laplacian with
  trilinear elements on the node lattice (spacing h/p per axis), and S_hat^{-1}
  is replaced by one geometric-multigrid V-cycle.

Definitions (the GPU path computes the same quantities its own way):

* lattice: nodes of the grid (p n_d + 1 per axis), lattice cells of sides
  l_d = h_d / p, volume v = l_0 l_1 l_2;
* node weight  beta_A = 1 / (c_m + max(d_A, 0) / v_A)  with
  d_A = (B^T kappa)_A = sum_B kappa_B N_A(xi_B) (the DLM row sums) and
  v_A = (number of lattice cells holding A) v / 8 (the lumped lattice volume);
* lattice-cell coefficient  alpha_c = tau_m(c) + mean of beta over c's corners,
  tau_m(c) from the stabilisation-parameter equation of section 2.1 with the
  corner means of a and s (s = 1 when absent), G = diag(1/h_d^2) of the grid's
  own cells;
* Dirichlet set of the Laplacian: lattice nodes on the domain boundary whose
  three velocity DOFs are not all prescribed (traction-free boundaries fix the
  pressure level), i.e. every boundary node when there is no velocity mask;
  node 0 alone when that set is empty (an enclosed flow);
* level 0 operator K_0 = sum_c alpha_c k(l), k the trilinear stiffness of a box,
  rows and columns of the Dirichlet set removed;
* coarse levels: lattice cells merged 2x2x2 while every axis has an even count
  and the level holds more than 64 nodes; alpha of a coarse cell = mean of its
  8 children; coarse node (I,J,K) = fine node (2I,2J,2K), Dirichlet when that
  fine node is; K_{l+1} rediscretised the same way;
* prolongation P_l: trilinear interpolation between non-Dirichlet nodes (rows of
  fine Dirichlet nodes and columns of coarse Dirichlet nodes are zero);
  restriction R_l = P_l^T;
* smoother: Jacobi with weight 8/9 on the non-Dirichlet nodes;
* V-cycle(l, b): coarsest level -> exact solve; else
  x = w D^-1 b;  x += w D^-1 (b - K x);  x += P V(l+1, R (b - K x));
  x += w D^-1 (b - K x) twice;
  Dirichlet nodes of level 0 finally get x_A = b_A / (K_0)_AA with the assembled
  diagonal (coarse Dirichlet nodes carry zero corrections).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dlm

OMEGA = 8.0 / 9.0
COARSE_MAX_NODES = 64
DIRECT_MAX_NODES = 1000

# 1D trilinear building blocks on the unit interval: int N_a' N_b' and int N_a N_b
_K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


def box_stiffness(l):
    """8x8 trilinear stiffness int grad N_a . grad N_b of a box with sides l (local a = a0 + 2 a1 + 4 a2)."""
    v = l[0] * l[1] * l[2]
    k = np.zeros((8, 8))
    for a in range(8):
        ad = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
        for b in range(8):
            bd = (b & 1, (b >> 1) & 1, (b >> 2) & 1)
            s = 0.0
            for d in range(3):
                t = _K1[ad[d], bd[d]] / (l[d] * l[d])
                for e in range(3):
                    if e != d:
                        t *= _M1[ad[e], bd[e]]
                s += t
            k[a, b] = v * s
    return k


class Level:
    def __init__(self, ncell, l, alpha, dset):
        self.ncell = tuple(int(c) for c in ncell)
        self.nn = tuple(c + 1 for c in self.ncell)
        self.l = tuple(float(v) for v in l)
        self.alpha = alpha            # [nz-1][ny-1][nx-1] flattened, x fastest
        self.dset = dset              # bool [N]
        self.K = None
        self.diag = None
        self.P = None                 # to this level from the next coarser one


def _corner_ids(nn):
    nx, ny, nz = nn
    cz, cy, cx = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
    ids = []
    for a in range(8):
        ids.append((cx + (a & 1)) + nx * ((cy + ((a >> 1) & 1)) + ny * (cz + ((a >> 2) & 1))))
    return np.stack(ids)          # [8][cells]


def assemble(lev):
    """K of a level (scipy CSR) with Dirichlet rows/cols removed, and its assembled diagonal."""
    nn = lev.nn
    N = nn[0] * nn[1] * nn[2]
    k = box_stiffness(lev.l)
    ids = _corner_ids(nn)
    rows = np.repeat(ids, 8, axis=0)                   # [64][cells]: a-major
    cols = np.tile(ids, (8, 1))
    vals = k.reshape(64, 1) * lev.alpha.reshape(1, -1)
    K = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N)).tocsr()
    diag = K.diagonal().copy()
    keep = (~lev.dset).astype(np.float64)
    Dk = sp.diags(keep)
    K = (Dk @ K @ Dk).tocsr()
    lev.K, lev.diag = K, diag
    return K, diag


def _prolongation(coarse, fine):
    """Trilinear interpolation coarse -> fine between non-Dirichlet nodes (sparse, fine x coarse)."""
    nf = fine.nn
    nc = coarse.nn
    Nf = nf[0] * nf[1] * nf[2]
    Nc = nc[0] * nc[1] * nc[2]
    kz, jy, ix = np.meshgrid(np.arange(nf[2]), np.arange(nf[1]), np.arange(nf[0]), indexing="ij")
    ix, jy, kz = ix.ravel(), jy.ravel(), kz.ravel()
    fid = ix + nf[0] * (jy + nf[1] * kz)
    rows, cols, vals = [], [], []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                # fine index i: coarse i//2 (weight 1 if even else 1/2) and i//2 + 1 for odd i
                wx = np.where(ix % 2 == 0, 1.0 - dx, 0.5)
                wy = np.where(jy % 2 == 0, 1.0 - dy, 0.5)
                wz = np.where(kz % 2 == 0, 1.0 - dz, 0.5)
                w = wx * wy * wz
                cx = ix // 2 + dx
                cy = jy // 2 + dy
                cz = kz // 2 + dz
                ok = (w > 0) & (cx < nc[0]) & (cy < nc[1]) & (cz < nc[2])
                cid = cx + nc[0] * (cy + nc[1] * cz)
                rows.append(fid[ok])
                cols.append(cid[ok])
                vals.append(w[ok])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nf, Nc)).tocsr()
    Rf = sp.diags((~fine.dset).astype(np.float64))
    Cc = sp.diags((~coarse.dset).astype(np.float64))
    return (Rf @ P @ Cc).tocsr()


def dirichlet_set(nn, mask=None):
    """Pressure-Laplacian Dirichlet nodes: boundary nodes whose velocity is not fully prescribed."""
    nx, ny, nz = nn
    kz, jy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    bnd = ((ix == 0) | (ix == nx - 1) | (jy == 0) | (jy == ny - 1) | (kz == 0) | (kz == nz - 1)).ravel()
    if mask is None:
        return bnd
    m = np.asarray(mask, dtype=bool).reshape(3, -1)
    return bnd & ~(m[0] & m[1] & m[2])


def dlm_row_sums(grid, cell, xi, kappa):
    """d_A = sum_B kappa_B N_A(xi_B): B^T applied to kappa (the DLM block's row sums)."""
    if cell is None or len(cell) == 0:
        return np.zeros(grid.num_nodes)
    M = len(cell)
    return dlm.apply_BT(grid, cell, xi, np.ones((3, M)), kappa)[0]


def node_beta(grid, prm, d):
    """beta_A = 1 / (c_m + max(d_A, 0) / v_A) on the node lattice."""
    c_m = float(prm[1])
    nn = grid.nodes_per_axis
    p = grid.order
    l = [grid.h[k] / p for k in range(3)]
    v = l[0] * l[1] * l[2]
    cnt = np.ones(nn[::-1])
    # lattice cells holding a node: 2 per axis inside, 1 on the boundary
    for axis, n in zip((2, 1, 0), nn):
        w = np.full(n, 2.0)
        w[0] = w[-1] = 1.0
        shape = [1, 1, 1]
        shape[axis] = n
        cnt = cnt * w.reshape(shape)
    vA = cnt.ravel() * v / 8.0
    return 1.0 / (c_m + np.maximum(np.asarray(d, dtype=np.float64), 0.0) / vA)


def cell_alpha(grid, prm, a, s, beta):
    """alpha_c = tau_m(c) + mean corner beta per lattice cell (flat, x fastest)."""
    nu, c_m, dt, C_T, C_I = (float(v) for v in prm)
    nn = grid.nodes_per_axis
    N = grid.num_nodes
    a = np.asarray(a, dtype=np.float64).reshape(3, N)
    ids = _corner_ids(nn)
    am = a[:, ids].mean(axis=1)                        # [3][cells]
    sm = np.ones(ids.shape[1]) if s is None else np.asarray(s, dtype=np.float64)[ids].mean(axis=0)
    h = grid.h
    aga = sum(am[d] ** 2 / h[d] ** 2 for d in range(3))
    gg = sum(1.0 / h[d] ** 4 for d in range(3))
    tau_m = 1.0 / np.sqrt(sm * (C_T / dt ** 2 + aga + C_I * nu * nu * gg))
    return tau_m + np.asarray(beta)[ids].mean(axis=0)


def level_shapes(ncell):
    """Lattice-cell counts of the levels: halve while every axis is even and the level has more
    than COARSE_MAX_NODES nodes."""
    shapes = [tuple(int(c) for c in ncell)]
    while all(c % 2 == 0 for c in shapes[-1]) and \
            (shapes[-1][0] + 1) * (shapes[-1][1] + 1) * (shapes[-1][2] + 1) > COARSE_MAX_NODES:
        shapes.append(tuple(c // 2 for c in shapes[-1]))
    return shapes


def coarsen(lev):
    """The next coarser level of lev (alpha averaged over 2x2x2 children, Dirichlet by injection)."""
    nc = tuple(c // 2 for c in lev.ncell)
    al = lev.alpha.reshape(lev.ncell[2], lev.ncell[1], lev.ncell[0])
    ac = 0.125 * (al[0::2, 0::2, 0::2] + al[0::2, 0::2, 1::2] + al[0::2, 1::2, 0::2] + al[0::2, 1::2, 1::2]
                  + al[1::2, 0::2, 0::2] + al[1::2, 0::2, 1::2] + al[1::2, 1::2, 0::2] + al[1::2, 1::2, 1::2])
    ds = lev.dset.reshape(lev.nn[2], lev.nn[1], lev.nn[0])[0::2, 0::2, 0::2].ravel()
    return Level(nc, [2.0 * v for v in lev.l], ac.ravel(), ds)


def finish_hierarchy(levels):
    """Operators and prolongations of a list of levels (finest first)."""
    if levels[-1].nn[0] * levels[-1].nn[1] * levels[-1].nn[2] > DIRECT_MAX_NODES:
        raise ValueError("lattice cannot be coarsened to a directly solvable size")
    for L in levels:
        assemble(L)
    for i in range(1, len(levels)):
        levels[i - 1].P = _prolongation(levels[i], levels[i - 1])
    return levels


def build_hierarchy(grid, prm, a, s=None, mask=None, cell=None, xi=None, kappa=None):
    """Levels of the pressure multigrid (finest first); the last one is solved directly."""
    p = grid.order
    nn = grid.nodes_per_axis
    d = dlm_row_sums(grid, cell, xi, kappa)
    beta = node_beta(grid, prm, d)
    alpha = cell_alpha(grid, prm, a, s, beta)
    dset = dirichlet_set(nn, mask)
    if not dset.any():
        dset[0] = True            # enclosed flow: pin the level of the Laplacian at node 0
    lev = Level([p * c for c in grid.n], [grid.h[k] / p for k in range(3)], alpha, dset)
    levels = [lev]
    for _ in level_shapes(lev.ncell)[1:]:
        levels.append(coarsen(levels[-1]))
    finish_hierarchy(levels)
    return levels


def vcycle(levels, b, i=0):
    """One V(2,2) cycle for K_i x = b on the non-Dirichlet nodes (Dirichlet entries of x: 0)."""
    lev = levels[i]
    keep = ~lev.dset
    if i == len(levels) - 1:
        x = np.zeros_like(b)
        idx = np.flatnonzero(keep)
        if idx.size:
            Kc = lev.K[idx][:, idx].toarray()
            x[idx] = np.linalg.solve(Kc, b[idx])
        return x
    winv = np.where(keep, OMEGA / np.where(lev.diag != 0.0, lev.diag, 1.0), 0.0)
    x = winv * b
    x = x + winv * (b - lev.K @ x)
    r = np.where(keep, b - lev.K @ x, 0.0)
    xc = vcycle(levels, lev.P.T @ r, i + 1)
    x = x + lev.P @ xc
    for _ in range(2):
        x = x + winv * (b - lev.K @ x)
    return x


def schur_solve(levels, b):
    """S_hat^{-1} b approximated by one V-cycle, Dirichlet nodes by their diagonal."""
    b = np.asarray(b, dtype=np.float64)
    lev = levels[0]
    bk = np.where(lev.dset, 0.0, b)
    x = vcycle(levels, bk, 0)
    return np.where(lev.dset, b / lev.diag, x)


def velocity_inverses(blocks):
    """Inverses of the nodal 3x3 velocity blocks ([N][3][3]) of the 4x4 diagonal blocks."""
    return np.linalg.inv(np.asarray(blocks, dtype=np.float64)[:, :3, :3])


def velocity_solve(finv, t, vel_steps=0, jac=None):
    """F_hat^{-1} t for the velocity block ([3][N]).  vel_steps = 0: the nodal block inverses;
    k > 0: k minimal-residual steps on F (the velocity rows of J [u; 0]) preconditioned by them:
    r = t, z = 0; each step p = blocks^{-1} r, q = F p, alpha = (q.r)/(q.q), z += alpha p,
    r -= alpha q."""
    N = finv.shape[0]
    t = np.asarray(t, dtype=np.float64).reshape(3, N)
    if vel_steps == 0:
        return np.einsum("nij,jn->in", finv, t)
    z = np.zeros((3, N))
    r = t.copy()
    for _ in range(vel_steps):
        p = np.einsum("nij,jn->in", finv, r)
        xp = np.zeros((4, N))
        xp[:3] = p
        q = np.asarray(jac(xp)).reshape(4, N)[:3]
        qq = float(np.sum(q * q))
        alpha = float(np.sum(q * r)) / qq if qq > 0.0 else 0.0
        z += alpha * p
        r -= alpha * q
    return z


def precond_apply(levels, finv, v, mode="diag", jac=None, vel_steps=0):
    """z = P^{-1} v ([4][N]); mode 'diag' (block diagonal) or 'tri' (upper block triangular, needs
    jac(x) = J x for the velocity rows of J [0; z_p]); vel_steps: minimal-residual steps of the
    velocity solve (velocity_solve, also needs jac)."""
    N = finv.shape[0]
    v = np.asarray(v, dtype=np.float64).reshape(4, N)
    z = np.zeros((4, N))
    z[3] = schur_solve(levels, v[3])
    t = v[:3].copy()
    if mode == "tri":
        xp = np.zeros((4, N))
        xp[3] = z[3]
        t -= np.asarray(jac(xp)).reshape(4, N)[:3]
    elif mode != "diag":
        raise ValueError(mode)
    z[:3] = velocity_solve(finv, t, vel_steps, jac)
    return z
