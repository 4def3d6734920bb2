"""MI355X (gfx950) library for the Jacobian hot path of the immersed FD/DLM FSI
method of arXiv 2601.08266 - Python binding.

The binding only marshals arguments: every step of the path runs in the HIP
kernels of libfsi.so behind the C ABI of include/fsi.h.  PyTorch tensors
supply device memory and the current stream.  Names follow the C ABI
(fsi_vms_apply -> vms_apply, ...).  There is no CPU fallback: if the library
is missing, importing a function that needs it raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _lib as L
from ._lib import (FSI_F32, FSI_F64, FsiError, FsiGrid, FsiNewtonOpts, FsiNewtonStats, FsiProblem,
                   FsiSolveOpts, FsiSolveStats, FsiVmsParams)

__all__ = [
    "FSI_F64", "FSI_F32", "FsiError", "make_grid", "make_params", "version",
    "vms_apply_workspace", "vms_apply", "PointTables", "dlm_locate", "dlm_B", "dlm_BT", "dlm_B_located", "dlm_permute",
    "Problem", "jacobian_apply", "jacobian_apply_block", "BLOCK_F", "BLOCK_G", "jacobian_workspace", "dlm_gram", "profile_enable",
    "profile_read", "vms_residual", "bjacobi_setup", "bjacobi_apply", "fgmres_solve",
    "schur_size", "schur_info", "schur_setup", "schur_apply", "PRECONDS", "tangent_apply",
    "newton_solve", "solve_opts", "newton_opts", "Solid", "solid_apply", "jacobian_solid_workspace",
    "jacobian_solid_apply", "solid_residual", "solid_step_residual", "solid_be_state", "newton_solid_solve",
]

_TORCH_OF = {FSI_F64: torch.float64, FSI_F32: torch.float32}


def version() -> str:
    return L.lib().fsi_version().decode()


def dtype_code(t: torch.dtype) -> int:
    if t == torch.float64:
        return FSI_F64
    if t == torch.float32:
        return FSI_F32
    raise TypeError(f"unsupported dtype {t}")


def make_grid(n, order=1, x0=(0.0, 0.0, 0.0), h=None) -> FsiGrid:
    """Grid struct from cell counts, order, origin and cell size (default 1/n)."""
    if h is None:
        h = tuple(1.0 / float(v) for v in n)
    g = FsiGrid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.x0[d] = float(x0[d])
        g.h[d] = float(h[d])
    g.order = int(order)
    return g


def grid_from(obj) -> FsiGrid:
    if isinstance(obj, FsiGrid):
        return obj
    return make_grid(obj.n, obj.order, obj.x0, obj.h)


def make_params(nu, c_m, dt, C_T=4.0, C_I=36.0, visc_strong=True) -> FsiVmsParams:
    p = FsiVmsParams()
    p.nu, p.c_m, p.dt, p.C_T, p.C_I = float(nu), float(c_m), float(dt), float(C_T), float(C_I)
    p.visc_strong = 1 if visc_strong else 0
    return p


def num_nodes(g: FsiGrid) -> int:
    return (g.order * g.n[0] + 1) * (g.order * g.n[1] + 1) * (g.order * g.n[2] + 1)


def num_cells(g: FsiGrid) -> int:
    return g.n[0] * g.n[1] * g.n[2]


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype=None, numel=None):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def _workspace(nbytes: int, device, ws: Optional[torch.Tensor]):
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small")
        return ws
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


# --------------------------------------------------------------------------- VMS
def vms_apply_workspace(grid, dtype: torch.dtype) -> int:
    g = grid_from(grid)
    return int(L.lib().fsi_vms_apply_workspace(ctypes.byref(g), dtype_code(dtype)))


def vms_apply(grid, prm: FsiVmsParams, a: torch.Tensor, x: torch.Tensor,
              s: Optional[torch.Tensor] = None, mask: Optional[torch.Tensor] = None,
              y: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """y = A(a, s) x (fsi_vms_apply)."""
    g = grid_from(grid)
    N = num_nodes(g)
    dt = x.dtype
    _need(x, "x", dt, 4 * N)
    _need(a, "a", dt, 3 * N)
    if s is not None:
        _need(s, "s", dt, N)
    if mask is not None:
        _need(mask, "mask", torch.int32)
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", dt, 4 * N)
    nbytes = vms_apply_workspace(g, dt)
    ws = _workspace(nbytes, x.device, ws)
    L.check("fsi_vms_apply", L.lib().fsi_vms_apply(
        ctypes.byref(g), ctypes.byref(prm), dtype_code(dt), _ptr(a), _ptr(s), _ptr(mask), _ptr(x),
        _ptr(y), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return y


# --------------------------------------------------------------------------- DLM
@dataclass
class PointTables:
    """Output of fsi_dlm_locate (device tensors) plus the two host counts."""

    m: int
    cell: torch.Tensor
    xi: torch.Tensor
    perm: torch.Tensor
    occ_cell: torch.Tensor
    occ_start: torch.Tensor
    occ_index: torch.Tensor
    n_occ: int
    n_outside: int
    s: Optional[torch.Tensor] = None


def dlm_locate(grid, X: torch.Tensor, dtype: torch.dtype = torch.float64,
               s_max: Optional[float] = None, ws: Optional[torch.Tensor] = None,
               stream=None) -> PointTables:
    """Cell, parametric position, cell-sorted order and occupied-cell CSR (fsi_dlm_locate)."""
    g = grid_from(grid)
    _need(X, "X", torch.float64)
    if X.numel() % 3:
        raise ValueError("X must be [3][M]")
    m = X.numel() // 3
    dev = X.device
    E = num_cells(g)
    cell = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    xi = torch.empty(3 * max(m, 1), dtype=dtype, device=dev)
    perm = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    occ_cell = torch.empty(E, dtype=torch.int32, device=dev)
    occ_start = torch.zeros(E + 1, dtype=torch.int32, device=dev)
    occ_index = torch.empty(E, dtype=torch.int32, device=dev)
    s = torch.empty(num_nodes(g), dtype=dtype, device=dev) if s_max is not None else None
    nbytes = int(L.lib().fsi_dlm_locate_workspace(ctypes.byref(g), m))
    ws = _workspace(nbytes, dev, ws)
    n_occ = ctypes.c_int64(0)
    n_out = ctypes.c_int64(0)
    L.check("fsi_dlm_locate", L.lib().fsi_dlm_locate(
        ctypes.byref(g), m, _ptr(X), dtype_code(dtype), _ptr(cell), _ptr(xi), _ptr(perm),
        _ptr(occ_cell), _ptr(occ_start), _ptr(occ_index), _ptr(s),
        float(s_max if s_max is not None else 1.0), ctypes.byref(n_occ), ctypes.byref(n_out),
        _ptr(ws), ws.numel(), _stream(stream)))
    return PointTables(m, cell[:m], xi[:3 * m], perm[:m], occ_cell, occ_start, occ_index,
                       int(n_occ.value), int(n_out.value), s)


def dlm_B(grid, tables: PointTables, u: torch.Tensor, Bu: Optional[torch.Tensor] = None,
          stream=None) -> torch.Tensor:
    """(B u)_B = sum_A N_A(xi_B) u_A (fsi_dlm_B).  u: [3][N] (or the first 3N of a [4][N])."""
    g = grid_from(grid)
    N = num_nodes(g)
    dt = tables.xi.dtype
    _need(u, "u", dt)
    if u.numel() < 3 * N:
        raise ValueError("u must hold at least 3N values")
    m = tables.m
    if Bu is None:
        Bu = torch.empty(3 * max(m, 1), dtype=dt, device=u.device)
    L.check("fsi_dlm_B", L.lib().fsi_dlm_B(
        ctypes.byref(g), dtype_code(dt), m, _ptr(tables.cell), _ptr(tables.xi), _ptr(u), _ptr(Bu),
        _stream(stream)))
    return Bu[:3 * m]


def dlm_BT(grid, tables: PointTables, lam: torch.Tensor, y: torch.Tensor,
           kappa: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
           stream=None, xi_loc: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y += B^T (kappa * lam) (fsi_dlm_BT); y: [3][N] (or a [4][N] whose first 3N are used).
    With xi_loc (the tables' xi in located order, dlm_permute), lam and kappa are taken in
    located order too and read without indirection (perm = NULL)."""
    g = grid_from(grid)
    dt = tables.xi.dtype
    _need(lam, "lam", dt, 3 * tables.m)
    _need(y, "y", dt)
    if kappa is not None:
        _need(kappa, "kappa", dt, tables.m)
    if xi_loc is not None:
        _need(xi_loc, "xi_loc", dt, 3 * tables.m)
    nbytes = int(L.lib().fsi_dlm_BT_workspace(ctypes.byref(g), tables.n_occ, dtype_code(dt)))
    ws = _workspace(nbytes, y.device, ws)
    xi, perm = (tables.xi, tables.perm) if xi_loc is None else (xi_loc, None)
    L.check("fsi_dlm_BT", L.lib().fsi_dlm_BT(
        ctypes.byref(g), dtype_code(dt), tables.m, _ptr(tables.cell), _ptr(xi),
        _ptr(perm), _ptr(tables.occ_cell), _ptr(tables.occ_start), _ptr(tables.occ_index),
        tables.n_occ, _ptr(lam), _ptr(kappa), _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


def dlm_permute(tables: PointTables, src: torch.Tensor, nf: int, to_point: bool = False,
                dst: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """nf fields of the M points ([nf][M]) into located order (dst[f][j] = src[f][perm[j]]) or,
    with to_point, back (fsi_dlm_permute)."""
    m = tables.m
    _need(src, "src", src.dtype, nf * m)
    if dst is None:
        dst = torch.empty(max(nf * m, 1), dtype=src.dtype, device=src.device)
    L.check("fsi_dlm_permute", L.lib().fsi_dlm_permute(
        dtype_code(src.dtype), m, nf, _ptr(tables.perm), 1 if to_point else 0, _ptr(src), _ptr(dst),
        _stream(stream)))
    return dst[:nf * m]


def dlm_B_located(grid, tables: PointTables, xi_loc: torch.Tensor, u: torch.Tensor,
                  Bu_loc: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """B u with xi_loc and the result in located order (fsi_dlm_B_located)."""
    g = grid_from(grid)
    N = num_nodes(g)
    dt = tables.xi.dtype
    _need(u, "u", dt)
    _need(xi_loc, "xi_loc", dt, 3 * tables.m)
    if u.numel() < 3 * N:
        raise ValueError("u must hold at least 3N values")
    m = tables.m
    if Bu_loc is None:
        Bu_loc = torch.empty(3 * max(m, 1), dtype=dt, device=u.device)
    L.check("fsi_dlm_B_located", L.lib().fsi_dlm_B_located(
        ctypes.byref(g), dtype_code(dt), m, _ptr(tables.occ_cell), _ptr(tables.occ_start), tables.n_occ,
        _ptr(xi_loc), _ptr(u), _ptr(Bu_loc), _stream(stream)))
    return Bu_loc[:3 * m]


def dlm_gram(grid, tables: PointTables, kappa: Optional[torch.Tensor] = None,
             out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Per occupied cell, the block sum_B kappa_B N_A(xi_B) N_C(xi_B) (fsi_dlm_gram)."""
    g = grid_from(grid)
    dt = tables.xi.dtype
    nen = (g.order + 1) ** 3
    if kappa is not None:
        _need(kappa, "kappa", dt, tables.m)
    if out is None:
        out = torch.empty(max(tables.n_occ, 1) * nen * nen, dtype=dt, device=tables.xi.device)
    L.check("fsi_dlm_gram", L.lib().fsi_dlm_gram(
        ctypes.byref(g), dtype_code(dt), tables.m, _ptr(tables.xi), _ptr(tables.perm),
        _ptr(tables.occ_start), tables.n_occ, _ptr(kappa), _ptr(out), _stream(stream)))
    return out


# --------------------------------------------------------------------------- Jacobian
class Problem:
    """fsi_problem: everything J = A_VMS + B^T diag(kappa) B needs, in one precision."""

    def __init__(self, grid, prm: FsiVmsParams, a: torch.Tensor, tables: Optional[PointTables],
                 kappa: Optional[torch.Tensor], s: Optional[torch.Tensor] = None,
                 mask: Optional[torch.Tensor] = None, gram: Optional[torch.Tensor] = None,
                 solid: Optional["Solid"] = None, solid_U: Optional[torch.Tensor] = None,
                 solid_coefs=(0.0, 0.0, 0.0)):
        """With `solid` (and its displacement `solid_U`, coefficients (c_M, c_K, c_V)) every
        apply uses the solid block B^T K_s B; kappa / gram then only feed the preconditioners."""
        g = grid_from(grid)
        dt = a.dtype
        self.grid, self.prm, self.dtype = g, prm, dt
        self.a, self.s, self.mask, self.tables, self.kappa = a, s, mask, tables, kappa
        self.gram = gram
        st = FsiProblem()
        st.grid = g
        st.prm = prm
        st.dtype = dtype_code(dt)
        st.a = a.data_ptr()
        st.s = s.data_ptr() if s is not None else None
        st.dir_mask = mask.data_ptr() if mask is not None else None
        if tables is not None and tables.m > 0:
            if tables.xi.dtype != dt or (kappa is not None and kappa.dtype != dt):
                raise TypeError("point tables and kappa must match the problem precision")
            st.m = tables.m
            st.cell = tables.cell.data_ptr()
            st.xi = tables.xi.data_ptr()
            st.perm = tables.perm.data_ptr()
            st.occ_cell = tables.occ_cell.data_ptr()
            st.occ_start = tables.occ_start.data_ptr()
            st.occ_index = tables.occ_index.data_ptr()
            st.n_occ = tables.n_occ
            st.kappa = kappa.data_ptr() if kappa is not None else None
            st.dlm_gram = gram.data_ptr() if gram is not None else None
        self.solid, self.solid_U = solid, solid_U
        if solid is not None:
            _need(solid_U, "solid_U", torch.float64, 3 * solid.m)
            st.solid = ctypes.addressof(solid.struct)
            st.solid_U = solid_U.data_ptr()
            st.solid_cM, st.solid_cK, st.solid_cV = (float(c) for c in solid_coefs)
        self.struct = st
        self.N = num_nodes(g)

    def workspace_bytes(self) -> int:
        return int(L.lib().fsi_jacobian_workspace(ctypes.byref(self.struct)))

    def bind(self, x: torch.Tensor, y: torch.Tensor, ws: torch.Tensor, stream=None):
        """A zero-argument callable running y = J x with pre-marshalled arguments
        (for tight loops where per-call Python checks would dominate)."""
        _need(x, "x", self.dtype, 4 * self.N)
        _need(y, "y", self.dtype, 4 * self.N)
        if ws.numel() * ws.element_size() < self.workspace_bytes():
            raise ValueError("workspace too small")
        f = L.lib().fsi_jacobian_apply
        args = (ctypes.byref(self.struct), _ptr(x), _ptr(y), _ptr(ws),
                ws.numel() * ws.element_size(), _stream(stream))

        def run():
            rc = f(*args)
            if rc:
                L.check("fsi_jacobian_apply", rc)
        return run


def jacobian_workspace(problem: Problem) -> int:
    return problem.workspace_bytes()


def jacobian_apply(problem: Problem, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = J x (fsi_jacobian_apply)."""
    _need(x, "x", problem.dtype, 4 * problem.N)
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", problem.dtype, 4 * problem.N)
    ws = _workspace(problem.workspace_bytes(), x.device, ws)
    L.check("fsi_jacobian_apply", L.lib().fsi_jacobian_apply(
        ctypes.byref(problem.struct), _ptr(x), _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


BLOCK_F, BLOCK_G = 1, 2


def jacobian_apply_block(problem: Problem, block: int, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Velocity rows of J on one input block (fsi_jacobian_apply_block): block BLOCK_F gives
    y_u = [J (x_u, 0)]_u, BLOCK_G gives y_u = [J (0, x_p)]_u; y's pressure part is not written."""
    _need(x, "x", problem.dtype, 4 * problem.N)
    if y is None:
        y = torch.zeros_like(x)
    _need(y, "y", problem.dtype, 4 * problem.N)
    ws = _workspace(problem.workspace_bytes(), x.device, ws)
    L.check("fsi_jacobian_apply_block", L.lib().fsi_jacobian_apply_block(
        ctypes.byref(problem.struct), int(block), _ptr(x), _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


# --------------------------------------------------------------------------- solid block
class Solid:
    """fsi_solid: a trilinear-hex solid mesh whose nodes are the DLM points, with the
    neo-Hookean material of eq. inc_neoHk; the node -> element-corner table is built by
    fsi_solid_setup (which validates the connectivity)."""

    def __init__(self, X0: torch.Tensor, conn: torch.Tensor, C0: float, kappa_s: float, rho_s0: float,
                 rho_f: float, mu_f: float, stream=None):
        _need(X0, "X0", torch.float64)
        _need(conn, "conn", torch.int32)
        m = X0.numel() // 3
        ne = conn.numel() // 8
        if X0.numel() != 3 * m or conn.numel() != 8 * ne:
            raise ValueError("X0 must be [3][M] and conn [n_elem][8]")
        self.X0, self.conn, self.m, self.n_elem = X0, conn, m, ne
        self.node_start = torch.empty(m + 1, dtype=torch.int32, device=X0.device)
        self.node_slot = torch.empty(max(8 * ne, 1), dtype=torch.int32, device=X0.device)
        L.check("fsi_solid_setup", L.lib().fsi_solid_setup(
            m, ne, _ptr(conn), _ptr(self.node_start), _ptr(self.node_slot), _stream(stream)))
        st = L.FsiSolid()
        st.n_nodes, st.n_elem = m, ne
        st.X0, st.conn = X0.data_ptr(), conn.data_ptr()
        st.node_start, st.node_slot = self.node_start.data_ptr(), self.node_slot.data_ptr()
        st.C0, st.kappa_s, st.rho_s0, st.rho_f, st.mu_f = C0, kappa_s, rho_s0, rho_f, mu_f
        self.struct = st


def solid_apply(solid: Solid, U: torch.Tensor, v: torch.Tensor, cM: float, cK: float, cV: float,
                y: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """y = (c_M M + c_K K(U) - c_V K_v(U)) v at the solid nodes (fsi_solid_apply)."""
    dt = v.dtype
    _need(U, "U", torch.float64, 3 * solid.m)
    _need(v, "v", dt, 3 * solid.m)
    if y is None:
        y = torch.empty_like(v)
    _need(y, "y", dt, 3 * solid.m)
    ws = _workspace(int(L.lib().fsi_solid_workspace(solid.n_elem, dtype_code(dt))), v.device, ws)
    L.check("fsi_solid_apply", L.lib().fsi_solid_apply(
        ctypes.byref(solid.struct), dtype_code(dt), _ptr(U), cM, cK, cV, _ptr(v), _ptr(y), _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream)))
    return y


def jacobian_solid_workspace(problem: Problem, solid: Solid) -> int:
    return int(L.lib().fsi_jacobian_solid_workspace(ctypes.byref(problem.struct), ctypes.byref(solid.struct)))


def jacobian_solid_apply(problem: Problem, solid: Solid, U: torch.Tensor, x: torch.Tensor, cM: float,
                         cK: float, cV: float, y: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """y = J x with the solid block B^T K_s B in place of the point stand-in
    (fsi_jacobian_solid_apply); the problem's points are the solid's nodes."""
    _need(x, "x", problem.dtype, 4 * problem.N)
    _need(U, "U", torch.float64, 3 * solid.m)
    if y is None:
        y = torch.empty_like(x)
    _need(y, "y", problem.dtype, 4 * problem.N)
    ws = _workspace(jacobian_solid_workspace(problem, solid), x.device, ws)
    L.check("fsi_jacobian_solid_apply", L.lib().fsi_jacobian_solid_apply(
        ctypes.byref(problem.struct), ctypes.byref(solid.struct), _ptr(U), cM, cK, cV, _ptr(x), _ptr(y),
        _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return y


# --------------------------------------------------------------------------- solvers
def vms_residual(problem: Problem, f: torch.Tensor, x: torch.Tensor, gD=None, lamg=None,
                 R: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """Nonlinear step residual (fsi_vms_residual); problem.a is ignored (a = u)."""
    N = problem.N
    _need(x, "x", problem.dtype, 4 * N)
    _need(f, "f", problem.dtype, 3 * N)
    if gD is not None:
        _need(gD, "gD", problem.dtype, 3 * N)
    if lamg is not None:
        _need(lamg, "lamg", problem.dtype, 3 * N)
    if R is None:
        R = torch.empty_like(x)
    ws = _workspace(problem.workspace_bytes(), x.device, ws)
    L.check("fsi_vms_residual", L.lib().fsi_vms_residual(
        ctypes.byref(problem.struct), _ptr(f), _ptr(lamg), _ptr(gD), _ptr(x), _ptr(R), _ptr(ws),
        ws.numel(), _stream(stream)))
    return R


def bjacobi_setup(problem: Problem, want32: bool = True, want_blocks: bool = False, stream=None):
    """Inverse nodal 4x4 blocks of J (fsi_bjacobi_setup): returns (pinv64, pinv32, blocks, n_sing)."""
    if problem.dtype != torch.float64:
        raise TypeError("block-Jacobi setup takes the FP64 problem")
    N = problem.N
    dev = problem.a.device
    pinv64 = torch.empty(16 * N, dtype=torch.float64, device=dev)
    pinv32 = torch.empty(16 * N, dtype=torch.float32, device=dev) if want32 else None
    blocks = torch.empty(16 * N, dtype=torch.float64, device=dev) if want_blocks else None
    nbytes = int(L.lib().fsi_bjacobi_workspace(ctypes.byref(problem.grid)))
    ws = _workspace(nbytes, dev, None)
    nsing = ctypes.c_int64(0)
    L.check("fsi_bjacobi_setup", L.lib().fsi_bjacobi_setup(
        ctypes.byref(problem.struct), _ptr(pinv64), _ptr(pinv32), _ptr(blocks), ctypes.byref(nsing),
        _ptr(ws), ws.numel(), _stream(stream)))
    return pinv64, pinv32, blocks, int(nsing.value)


def bjacobi_apply(grid, pinv: torch.Tensor, v: torch.Tensor, z: Optional[torch.Tensor] = None,
                  stream=None):
    g = grid_from(grid)
    _need(v, "v", pinv.dtype, 4 * num_nodes(g))
    if z is None:
        z = torch.empty_like(v)
    L.check("fsi_bjacobi_apply", L.lib().fsi_bjacobi_apply(
        ctypes.byref(g), dtype_code(pinv.dtype), _ptr(pinv), _ptr(v), _ptr(z), _stream(stream)))
    return z


PRECONDS = {"bjacobi": L.FSI_PC_BJACOBI, "schur_diag": L.FSI_PC_SCHUR_DIAG, "schur_tri": L.FSI_PC_SCHUR_TRI}


def _precond_code(precond) -> int:
    return PRECONDS[precond] if isinstance(precond, str) else int(precond)


def schur_size(grid) -> int:
    """Bytes of the Schur-complement preconditioner object (fsi_schur_size); 0 if unsupported."""
    return int(L.lib().fsi_schur_size(ctypes.byref(grid_from(grid))))


def schur_info(grid):
    """(levels, [(cells x, y, z) per level], [byte offset of each level's FP64 alpha])."""
    g = grid_from(grid)
    n = ctypes.c_int32(0)
    cells = (ctypes.c_int32 * 48)()
    offs = (ctypes.c_int64 * 16)()
    L.check("fsi_schur_info", L.lib().fsi_schur_info(ctypes.byref(g), ctypes.byref(n), cells, offs))
    k = int(n.value)
    return k, [tuple(cells[3 * i:3 * i + 3]) for i in range(k)], [int(offs[i]) for i in range(k)]


def schur_setup(problem: Problem, blocks: torch.Tensor, pc: Optional[torch.Tensor] = None, stream=None):
    """Schur-complement block preconditioner of J (fsi_schur_setup) from the raw nodal blocks of
    bjacobi_setup(want_blocks=True); returns the object (a uint8 device tensor)."""
    if problem.dtype != torch.float64:
        raise TypeError("the Schur preconditioner setup takes the FP64 problem")
    _need(blocks, "blocks", torch.float64, 16 * problem.N)
    nbytes = schur_size(problem.grid)
    if nbytes == 0:
        raise ValueError("Schur preconditioner unsupported: " + L.lib().fsi_last_error().decode())
    pc = _workspace(nbytes, blocks.device, pc)
    L.check("fsi_schur_setup", L.lib().fsi_schur_setup(
        ctypes.byref(problem.struct), _ptr(blocks), _ptr(pc), pc.numel(), _stream(stream)))
    return pc


def schur_apply(problem: Problem, precond, pc: torch.Tensor, v: torch.Tensor,
                z: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None,
                vel_steps: int = 0):
    """z = P^{-1} v (fsi_schur_apply) in the problem's precision."""
    _need(v, "v", problem.dtype, 4 * problem.N)
    if z is None:
        z = torch.empty_like(v)
    ws = _workspace(problem.workspace_bytes(), v.device, ws)
    L.check("fsi_schur_apply", L.lib().fsi_schur_apply(
        ctypes.byref(problem.struct), _precond_code(precond), int(vel_steps), _ptr(pc), _ptr(v), _ptr(z), _ptr(ws),
        ws.numel(), _stream(stream)))
    return z


def _attach_host_ring(o, restart, pinned):
    """Give the options a pinned host ring for the Arnoldi coefficients (the library keeps no
    host memory of its own); the tensor lives as long as the options object."""
    n = int(restart) * (int(restart) + 2)
    if pinned and torch.cuda.is_available():
        ring = torch.empty(n, dtype=torch.float64, pin_memory=True)
        o._host_ring = ring
        o.host_ring, o.host_ring_len = ring.data_ptr(), n
    else:
        o.host_ring, o.host_ring_len = None, 0


def solve_opts(restart=50, max_iters=2000, rtol=1e-10, inner=torch.float32,
               inner_reduction=1e-5, precond="bjacobi", vel_steps=0, pinned=True,
               basis=torch.float64) -> FsiSolveOpts:
    """basis: storage of the Krylov basis (torch.float32 only with inner=torch.float32 and
    restart <= 52; the Gram-Schmidt arithmetic stays FP64)."""
    o = FsiSolveOpts()
    o.basis = dtype_code(basis)
    o.restart, o.max_iters, o.rtol = int(restart), int(max_iters), float(rtol)
    o.inner = dtype_code(inner)
    o.inner_reduction = float(inner_reduction)
    o.precond = _precond_code(precond)
    o.vel_steps = int(vel_steps)
    _attach_host_ring(o, restart, pinned)
    return o


def fgmres_solve(J64: Problem, b: torch.Tensor, x: torch.Tensor, opts: FsiSolveOpts,
                 J32: Optional[Problem] = None, pinv: Optional[torch.Tensor] = None,
                 ws: Optional[torch.Tensor] = None, stream=None, check: bool = True):
    """Mixed-precision FGMRES (fsi_fgmres_solve); x is updated in place. Returns (status, stats)."""
    _need(b, "b", torch.float64, 4 * J64.N)
    _need(x, "x", torch.float64, 4 * J64.N)
    p32 = ctypes.byref(J32.struct) if J32 is not None else None
    nbytes = int(L.lib().fsi_fgmres_workspace(ctypes.byref(J64.struct), p32, ctypes.byref(opts)))
    if nbytes == 0:
        raise ValueError("invalid FGMRES arguments: " + L.lib().fsi_last_error().decode())
    ws = _workspace(nbytes, x.device, ws)
    st = FsiSolveStats()
    rc = L.lib().fsi_fgmres_solve(ctypes.byref(J64.struct), p32, _ptr(pinv), _ptr(b), _ptr(x),
                                  ctypes.byref(opts), ctypes.byref(st), _ptr(ws), ws.numel(),
                                  _stream(stream))
    if check:
        L.check("fsi_fgmres_solve", rc)
    return rc, st


def newton_opts(tol_abs, max_newton=20, eta=1e-3, restart=50, max_krylov=2000,
                inner=torch.float32, inner_reduction=1e-5, precond="bjacobi", vel_steps=0,
                tangent="picard", pinned=True, pc_reuse=False, basis=torch.float64) -> FsiNewtonOpts:
    o = FsiNewtonOpts()
    o.basis = dtype_code(basis)
    o.max_newton, o.tol_abs, o.eta = int(max_newton), float(tol_abs), float(eta)
    o.restart, o.max_krylov = int(restart), int(max_krylov)
    o.inner = dtype_code(inner)
    o.inner_reduction = float(inner_reduction)
    o.precond = _precond_code(precond)
    o.vel_steps = int(vel_steps)
    o.tangent = {"picard": 0, "full": 1}[tangent] if isinstance(tangent, str) else int(tangent)
    o.pc_reuse = 1 if pc_reuse else 0
    _attach_host_ring(o, restart, pinned)
    return o


def tangent_apply(P: Problem, x: torch.Tensor, f: torch.Tensor, v: torch.Tensor,
                  y: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """Full Newton tangent of the step residual at state x (source f) times v (fsi_tangent_apply),
    all in the problem's precision."""
    dt = P.dtype
    _need(x, "x", dt, 4 * P.N)
    _need(f, "f", dt, 3 * P.N)
    _need(v, "v", dt, 4 * P.N)
    if y is None:
        y = torch.empty_like(v)
    nbytes = int(L.lib().fsi_tangent_workspace(ctypes.byref(P.struct)))
    if nbytes == 0:
        raise ValueError("invalid tangent arguments: " + L.lib().fsi_last_error().decode())
    ws = _workspace(nbytes, x.device, ws)
    L.check("fsi_tangent_apply", L.lib().fsi_tangent_apply(
        ctypes.byref(P.struct), _ptr(x), _ptr(f), _ptr(v), _ptr(y), _ptr(ws), ws.numel(), _stream(stream)))
    return y


def newton_solve(P64: Problem, f: torch.Tensor, x: torch.Tensor, opts: FsiNewtonOpts,
                 P32: Optional[Problem] = None, lamg=None, gD=None,
                 ws: Optional[torch.Tensor] = None, stream=None, check: bool = True):
    """One implicit step by Newton (fsi_newton_solve); x updated in place. Returns (status, stats)."""
    _need(x, "x", torch.float64, 4 * P64.N)
    _need(f, "f", torch.float64, 3 * P64.N)
    p32 = ctypes.byref(P32.struct) if P32 is not None else None
    nbytes = int(L.lib().fsi_newton_workspace(ctypes.byref(P64.struct), p32, ctypes.byref(opts)))
    if nbytes == 0:
        raise ValueError("invalid Newton arguments: " + L.lib().fsi_last_error().decode())
    ws = _workspace(nbytes, x.device, ws)
    st = FsiNewtonStats()
    rc = L.lib().fsi_newton_solve(ctypes.byref(P64.struct), p32, _ptr(f), _ptr(lamg), _ptr(gD),
                                  _ptr(x), ctypes.byref(opts), ctypes.byref(st), _ptr(ws),
                                  ws.numel(), _stream(stream))
    if check:
        L.check("fsi_newton_solve", rc)
    return rc, st


def solid_residual(solid: "Solid", U: torch.Tensor, V: torch.Tensor, A: torch.Tensor,
                   R: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None):
    """R^s = M_rho(U) A + f_int(U) - K_v(U) V at the solid nodes (fsi_solid_residual, FP64)."""
    for t, n in ((U, "U"), (V, "V"), (A, "A")):
        _need(t, n, torch.float64, 3 * solid.m)
    if R is None:
        R = torch.empty_like(U)
    _need(R, "R", torch.float64, 3 * solid.m)
    ws = _workspace(int(L.lib().fsi_solid_workspace(solid.n_elem, FSI_F64)), U.device, ws)
    L.check("fsi_solid_residual", L.lib().fsi_solid_residual(
        ctypes.byref(solid.struct), _ptr(U), _ptr(V), _ptr(A), _ptr(R), _ptr(ws), ws.numel(), _stream(stream)))
    return R


def solid_step_residual(problem: Problem, solid: "Solid", state, f: torch.Tensor, x: torch.Tensor, gD=None,
                        R=None, U=None, V=None, ws=None, stream=None):
    """Step residual with the solid (fsi_solid_step_residual); state = (U_base, A_base, cU, cA).
    Returns (R, U, V)."""
    Ub, Ab, cU, cA = state
    N, M = problem.N, solid.m
    _need(x, "x", torch.float64, 4 * N)
    _need(f, "f", torch.float64, 3 * N)
    R = torch.empty_like(x) if R is None else R
    U = torch.empty_like(Ub) if U is None else U
    V = torch.empty_like(Ub) if V is None else V
    for t, n in ((Ub, "U_base"), (Ab, "A_base"), (U, "U"), (V, "V")):
        _need(t, n, torch.float64, 3 * M)
    ws = _workspace(int(L.lib().fsi_solid_step_workspace(ctypes.byref(problem.struct), ctypes.byref(solid.struct))),
                    x.device, ws)
    L.check("fsi_solid_step_residual", L.lib().fsi_solid_step_residual(
        ctypes.byref(problem.struct), ctypes.byref(solid.struct), _ptr(Ub), _ptr(Ab), float(cU), float(cA),
        _ptr(f), _ptr(gD), _ptr(x), _ptr(R), _ptr(U), _ptr(V), _ptr(ws), ws.numel(), _stream(stream)))
    return R, U, V


def solid_be_state(U_n: torch.Tensor, V_n: torch.Tensor, dt: float):
    """(U_base, A_base, cU, cA) of a backward-Euler step: (U_n, V_n / dt, dt, 1 / dt)."""
    Ab = torch.empty_like(V_n)
    axpby(1.0 / dt, V_n, 0.0, Ab)
    return U_n, Ab, dt, 1.0 / dt


def newton_solid_solve(P64: Problem, solid: "Solid", state, f: torch.Tensor, x: torch.Tensor, U: torch.Tensor,
                       V: torch.Tensor, opts: FsiNewtonOpts, P32: Optional[Problem] = None, gD=None,
                       ws: Optional[torch.Tensor] = None, stream=None, check: bool = True):
    """One time step with the solid (fsi_newton_solid_solve); state = (U_base, A_base, cU, cA);
    x, U, V updated in place.  Returns (status, stats)."""
    Ub, Ab, cU, cA = state
    _need(x, "x", torch.float64, 4 * P64.N)
    _need(f, "f", torch.float64, 3 * P64.N)
    p32 = ctypes.byref(P32.struct) if P32 is not None else None
    nbytes = int(L.lib().fsi_newton_solid_workspace(ctypes.byref(P64.struct), p32, ctypes.byref(solid.struct),
                                                     ctypes.byref(opts)))
    if nbytes == 0:
        raise ValueError("invalid Newton arguments: " + L.lib().fsi_last_error().decode())
    ws = _workspace(nbytes, x.device, ws)
    st = FsiNewtonStats()
    rc = L.lib().fsi_newton_solid_solve(ctypes.byref(P64.struct), p32, ctypes.byref(solid.struct), _ptr(Ub),
                                        _ptr(Ab), float(cU), float(cA), _ptr(f), _ptr(gD), _ptr(x), _ptr(U), _ptr(V),
                                        ctypes.byref(opts), ctypes.byref(st), _ptr(ws), ws.numel(),
                                        _stream(stream))
    if check:
        L.check("fsi_newton_solid_solve", rc)
    return rc, st


# --------------------------------------------------------------------------- BLAS-1
_DOT_WS = {}


def axpby(alpha: float, x: torch.Tensor, beta: float, y: torch.Tensor, stream=None):
    """y = alpha x + beta y on FP64 device vectors (fsi_axpby)."""
    _need(x, "x", torch.float64)
    _need(y, "y", torch.float64, x.numel())
    L.check("fsi_axpby", L.lib().fsi_axpby(x.numel(), float(alpha), _ptr(x), float(beta), _ptr(y),
                                            _stream(stream)))
    return y


def dot(x: torch.Tensor, y: torch.Tensor, stream=None) -> float:
    """x . y (fsi_dot, deterministic; synchronises)."""
    _need(x, "x", torch.float64)
    _need(y, "y", torch.float64, x.numel())
    dev = x.device
    if dev not in _DOT_WS:
        _DOT_WS[dev] = torch.empty(int(L.lib().fsi_dot_workspace()), dtype=torch.uint8, device=dev)
    ws = _DOT_WS[dev]
    out = ctypes.c_double(0.0)
    L.check("fsi_dot", L.lib().fsi_dot(x.numel(), _ptr(x), _ptr(y), ctypes.byref(out), _ptr(ws),
                                        ws.numel(), _stream(stream)))
    return float(out.value)


def norm2(x: torch.Tensor, stream=None) -> float:
    return dot(x, x, stream) ** 0.5


# --------------------------------------------------------------------------- timing
def profile_enable(on: bool = True) -> None:
    """Start (and reset) or stop per-kernel hipEvent timing inside the library."""
    L.check("fsi_profile_enable", L.lib().fsi_profile_enable(1 if on else 0))


def profile_read(kernel: str):
    """(total milliseconds, launches) recorded for `kernel` since profile_enable(True)."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    L.check("fsi_profile_read", L.lib().fsi_profile_read(kernel.encode(), ctypes.byref(ms),
                                                         ctypes.byref(n)))
    return float(ms.value), int(n.value)
