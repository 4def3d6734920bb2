"""FP64 reference of the VMS-stabilised Oseen operator (test infrastructure only).

Thin ctypes wrapper around ``vms_ref.c``.  The operator is the Galerkin weak
form of section 2.1 (eq. fluid_weak_form, per unit density, Oseen-linearised
about a nodal advection field a, mass coefficient c_m = 1/dt) plus the
residual-based SUPG / PSPG / LSIC terms with tau_m, tau_c, G from the
stabilisation-parameter equations of section 2.1.  See the C file's header
for the full statement.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

MASS, CONV, VISC, PDIV, CONT, SUPG, PSPG, LSIC = 1, 2, 4, 8, 16, 32, 64, 128
ALL = 255
# test functions of the source load (Galerkin, SUPG, PSPG)
SRC_GAL, SRC_SUPG, SRC_PSPG = 1, 2, 4
SRC_ALL = 7

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or any(
                os.path.getmtime(path) < os.path.getmtime(s) for s in _build.SOURCES):
            _build.build(force=True)
        _lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int
        _lib.oracle_element_matrix.argtypes = [I, P, P, I, I, P, P, ctypes.c_uint, P]
        _lib.oracle_source_matrix.argtypes = [I, P, P, I, P, P, ctypes.c_uint, P]
        _lib.oracle_element_tangent.argtypes = [I, P, P, I, I, P, P, P, P]
        _lib.oracle_vms_tangent_apply.argtypes = [P, I, P, P, I, P, P, P, P, P, P]
        _lib.oracle_vms_step_rows.argtypes = [P, I, P, P, I, P, P, P, P, P, I, P, ctypes.c_int64, P]
        _lib.oracle_vms_apply.argtypes = [P, I, P, P, I, P, P, P, P, P]
        _lib.oracle_vms_rows.argtypes = [P, I, P, P, I, P, P, P, P, P, ctypes.c_int64, P]
        _lib.oracle_vms_diag_blocks.argtypes = [P, I, P, P, I, P, P, P, P]
        _lib.oracle_vms_residual.argtypes = [P, I, P, P, I, P, P, P, P]
        for f in (_lib.oracle_element_matrix, _lib.oracle_source_matrix, _lib.oracle_vms_apply,
                  _lib.oracle_vms_rows, _lib.oracle_vms_diag_blocks, _lib.oracle_vms_residual,
                  _lib.oracle_element_tangent, _lib.oracle_vms_tangent_apply,
                  _lib.oracle_vms_step_rows):
            f.restype = ctypes.c_int
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def params_array(nu, c_m, dt, C_T=4.0, C_I=36.0):
    return np.array([nu, c_m, dt, C_T, C_I], dtype=np.float64)


def _mask_bytes(mask):
    return None if mask is None else np.ascontiguousarray(np.asarray(mask, dtype=bool).reshape(-1)).view(np.uint8)


def element_matrix(p, h, prm, a_e, s_e=None, terms=ALL, visc_strong=True, nq=0):
    """Dense (4 nen)^2 element matrix; rows = test DOFs (f*nen + A), cols = trial DOFs."""
    nen = (p + 1) ** 3
    K = np.zeros((4 * nen, 4 * nen))
    h = _f64(h); prm = _f64(prm); a_e = _f64(a_e); s_e = _f64(s_e)
    rc = lib().oracle_element_matrix(p, _p(h), _p(prm), int(bool(visc_strong)), nq, _p(a_e),
                                     _p(s_e), terms, _p(K))
    if rc:
        raise ValueError(f"oracle_element_matrix failed ({rc})")
    return K


def source_matrix(p, h, prm, a_e, s_e=None, nq=0, terms=SRC_ALL):
    """Load matrix of a nodal source: rows = test DOFs, cols = [3][nen] source values."""
    nen = (p + 1) ** 3
    L = np.zeros((4 * nen, 3 * nen))
    h = _f64(h); prm = _f64(prm); a_e = _f64(a_e); s_e = _f64(s_e)
    rc = lib().oracle_source_matrix(p, _p(h), _p(prm), nq, _p(a_e), _p(s_e), terms, _p(L))
    if rc:
        raise ValueError(f"oracle_source_matrix failed ({rc})")
    return L


def element_tangent(p, h, prm, x_e, f_e, s_e=None, visc_strong=True, nq=0):
    """Dense (4 nen)^2 full Newton tangent of the element residual K(a=u) x - L(a=u) f at the
    element state x_e ([4][nen]) with nodal source f_e ([3][nen])."""
    nen = (p + 1) ** 3
    T = np.zeros((4 * nen, 4 * nen))
    h = _f64(h); prm = _f64(prm); x_e = _f64(x_e); f_e = _f64(f_e); s_e = _f64(s_e)
    rc = lib().oracle_element_tangent(p, _p(h), _p(prm), int(bool(visc_strong)), nq, _p(x_e), _p(f_e),
                                      _p(s_e), _p(T))
    if rc:
        raise ValueError(f"oracle_element_tangent failed ({rc})")
    return T


def _grid_args(grid):
    n = np.array(grid.n, dtype=np.int32)
    h = np.array(grid.h, dtype=np.float64)
    return n, h


def apply(grid, prm, a, x, s=None, mask=None, visc_strong=True):
    """y = A x on the whole grid ([4][N] in and out)."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    a = _f64(a).reshape(3, N); x = _f64(x).reshape(4, N); s = _f64(s)
    prm = _f64(prm)
    m = _mask_bytes(mask)
    y = np.zeros((4, N))
    rc = lib().oracle_vms_apply(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)), _p(a),
                                _p(s), _p(m), _p(x), _p(y))
    if rc:
        raise ValueError(f"oracle_vms_apply failed ({rc})")
    return y


def apply_rows(grid, prm, a, x, rows, s=None, mask=None, visc_strong=True):
    """Entries y[rows] of y = A x (rows are flat indices f*N + node)."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    a = _f64(a).reshape(3, N); x = _f64(x).reshape(4, N); s = _f64(s)
    prm = _f64(prm)
    m = _mask_bytes(mask)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    rc = lib().oracle_vms_rows(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)), _p(a),
                               _p(s), _p(m), _p(x), _p(rows), rows.size, _p(out))
    if rc:
        raise ValueError(f"oracle_vms_rows failed ({rc})")
    return out


def diag_blocks(grid, prm, a, s=None, mask=None, visc_strong=True):
    """Nodal 4x4 diagonal blocks of A, [N][4][4]; Dirichlet velocity rows/cols -> identity."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    a = _f64(a).reshape(3, N); s = _f64(s); prm = _f64(prm)
    m = _mask_bytes(mask)
    out = np.zeros((N, 4, 4))
    rc = lib().oracle_vms_diag_blocks(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)),
                                      _p(a), _p(s), _p(m), _p(out))
    if rc:
        raise ValueError(f"oracle_vms_diag_blocks failed ({rc})")
    return out


def residual_fluid(grid, prm, x, f, s=None, visc_strong=True):
    """sum_e K_e(a=u) x_e - L_e(a=u) f_e : the fluid part of the step residual ([4][N])."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    x = _f64(x).reshape(4, N); f = _f64(f).reshape(3, N); s = _f64(s); prm = _f64(prm)
    R = np.zeros((4, N))
    rc = lib().oracle_vms_residual(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)),
                                   _p(s), _p(x), _p(f), _p(R))
    if rc:
        raise ValueError(f"oracle_vms_residual failed ({rc})")
    return R


def tangent_apply(grid, prm, x, f, v, s=None, mask=None, visc_strong=True):
    """Fluid part of the full Newton tangent at state x (source f) times v ([4][N]); Dirichlet
    columns of v zeroed, Dirichlet rows return v."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    x = _f64(x).reshape(4, N); f = _f64(f).reshape(3, N); v = _f64(v).reshape(4, N)
    s = _f64(s); prm = _f64(prm)
    m = _mask_bytes(mask)
    y = np.zeros((4, N))
    rc = lib().oracle_vms_tangent_apply(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)),
                                        _p(s), _p(m), _p(x), _p(f), _p(v), _p(y))
    if rc:
        raise ValueError(f"oracle_vms_tangent_apply failed ({rc})")
    return y


def step_rows(grid, prm, x, f, rows, s=None, mask=None, v=None, visc_strong=True):
    """Rows (flat f*N + node) of residual_fluid (v is None) or of tangent_apply (v given)."""
    n, h = _grid_args(grid)
    N = grid.num_nodes
    x = _f64(x).reshape(4, N); f = _f64(f).reshape(3, N); s = _f64(s); prm = _f64(prm)
    vv = None if v is None else _f64(v).reshape(4, N)
    m = _mask_bytes(mask)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(rows.size)
    rc = lib().oracle_vms_step_rows(_p(n), grid.order, _p(h), _p(prm), int(bool(visc_strong)), _p(s),
                                    _p(m), _p(x), _p(f), _p(vv), 1 if v is None else 2, _p(rows),
                                    rows.size, _p(out))
    if rc:
        raise ValueError(f"oracle_vms_step_rows failed ({rc})")
    return out


def cell_node_ids(grid, cx, cy, cz):
    p = grid.order
    q = p + 1
    Nx, Ny, _ = grid.nodes_per_axis
    ids = np.zeros(q ** 3, dtype=np.int64)
    for az in range(q):
        for ay in range(q):
            for ax in range(q):
                ids[ax + q * (ay + q * az)] = (p * cx + ax) + Nx * ((p * cy + ay) + Ny * (p * cz + az))
    return ids


def assemble_dense(grid, prm, a, s=None, terms=ALL, visc_strong=True):
    """Dense global matrix (4N x 4N, field-major DOFs) - small grids only."""
    N = grid.num_nodes
    p = grid.order
    nen = (p + 1) ** 3
    a = _f64(a).reshape(3, N)
    A = np.zeros((4 * N, 4 * N))
    for cz in range(grid.n[2]):
        for cy in range(grid.n[1]):
            for cx in range(grid.n[0]):
                ids = cell_node_ids(grid, cx, cy, cz)
                a_e = a[:, ids].reshape(-1)
                s_e = None if s is None else np.asarray(s)[ids]
                K = element_matrix(p, grid.h, prm, a_e, s_e, terms, visc_strong)
                dofs = np.concatenate([f * N + ids for f in range(4)])
                A[np.ix_(dofs, dofs)] += K
    return A
