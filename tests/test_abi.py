"""The C-ABI library loads on the CPU host and exports every entry point that
include/fsi.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsi.h")
LIB = os.path.join(ROOT, "paper_2601_08266_amd", "libfsi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(fsi_[A-Za-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_core_entry_points():
    names = declared_functions()
    for core in ["fsi_vms_apply", "fsi_dlm_locate", "fsi_dlm_B", "fsi_dlm_BT",
                 "fsi_jacobian_apply"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libfsi.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"


def test_binding_signatures_cover_the_header():
    import paper_2601_08266_amd._lib as L
    assert set(declared_functions()) <= set(L.SIGNATURES)


def test_status_strings_and_argument_errors_without_gpu():
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    assert lib.fsi_status_string(0) == b"ok"
    assert b"gfx950" in lib.fsi_version()
    # invalid grids are rejected before any device work
    g = L.FsiGrid()
    g.order = 3
    assert lib.fsi_vms_apply_workspace(ctypes.byref(g), 0) == 0
    p = L.FsiVmsParams()
    rc = lib.fsi_vms_apply(ctypes.byref(g), ctypes.byref(p), 0, None, None, None, None, None,
                           None, 0, None)
    assert rc == L.FSI_ERR_ARG
    assert b"order" in lib.fsi_last_error()


@pytest.mark.parametrize("n,order", [((192, 192, 192), 1), ((96, 96, 96), 2), ((64, 64, 64), 1),
                                     ((8, 8, 8), 1), ((10, 12, 14), 1), ((5, 6, 7), 2), ((3, 3, 3), 1)])
def test_schur_levels_follow_the_coarsening_rule(n, order):
    # host-only: the library's multigrid levels equal the oracle's rule (no device work)
    import paper_2601_08266_amd as fsi
    from oracle import schur
    k, cells, offs = fsi.schur_info(fsi.make_grid(n, order))
    want = schur.level_shapes(tuple(order * c for c in n))
    assert k == len(want) and cells == want
    assert offs == sorted(offs) and fsi.schur_size(fsi.make_grid(n, order)) > offs[-1]


def test_schur_rejects_lattices_without_a_small_coarse_level():
    import paper_2601_08266_amd as fsi
    assert fsi.schur_size(fsi.make_grid((13, 13, 13), 1)) == 0
    assert b"coarsened" in fsi._lib.lib().fsi_last_error()


def test_solid_entry_points_reject_bad_arguments_without_gpu():
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    assert lib.fsi_solid_setup(-1, 0, None, None, None, None) == L.FSI_ERR_ARG
    assert lib.fsi_solid_setup(8, 1, None, None, None, None) == L.FSI_ERR_ARG
    assert lib.fsi_solid_workspace(10, 0) >= 10 * 24 * 8
    s = L.FsiSolid()
    s.n_nodes, s.n_elem = 8, 1          # tables missing
    rc = lib.fsi_solid_apply(ctypes.byref(s), 0, None, 1.0, 1.0, 1.0, None, None, None, 0, None)
    assert rc == L.FSI_ERR_ARG
    s.n_nodes, s.n_elem = 0, 0
    s.C0 = float("nan")
    rc = lib.fsi_solid_apply(ctypes.byref(s), 0, None, 1.0, 1.0, 1.0, None, None, None, 0, None)
    assert rc == L.FSI_ERR_ARG and b"finite" in lib.fsi_last_error()


def test_block_products_reject_bad_arguments_without_gpu():
    # host-only checks of fsi_jacobian_apply_block: a block id other than F (1) or G (2), and a Q2
    # grid, are rejected before any device work (the pointers below are never dereferenced)
    import paper_2601_08266_amd as fsi
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    p = L.FsiProblem()
    p.grid = fsi.make_grid((8, 8, 8), 1)
    p.prm = fsi.make_params(0.01, 1000.0, 1e-3, 4.0, 36.0)
    p.dtype = L.FSI_F64
    p.a = 16
    x, y = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    assert lib.fsi_jacobian_apply_block(ctypes.byref(p), 3, x, y, None, 0, None) == L.FSI_ERR_ARG
    assert b"FSI_BLOCK_F" in lib.fsi_last_error()
    assert lib.fsi_jacobian_apply_block(ctypes.byref(p), fsi.BLOCK_G, x, x, None, 0, None) == L.FSI_ERR_ARG
    p.grid = fsi.make_grid((4, 4, 4), 2)
    assert lib.fsi_jacobian_apply_block(ctypes.byref(p), fsi.BLOCK_F, x, y, None, 0, None) == L.FSI_ERR_UNSUPPORTED
    assert b"Q1" in lib.fsi_last_error()


def test_fp32_krylov_basis_options_without_gpu():
    # host-only: the FP32 Krylov basis needs the FP32 inner precision and restart <= 52, and it
    # shrinks the FGMRES workspace by the basis' half (the pointers are never dereferenced)
    import torch

    import paper_2601_08266_amd as fsi
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    probs = []
    for dt in (L.FSI_F64, L.FSI_F32):
        p = L.FsiProblem()
        p.grid = fsi.make_grid((8, 8, 8), 1)
        p.prm = fsi.make_params(0.01, 1000.0, 1e-3, 4.0, 36.0)
        p.dtype = dt
        p.a = 16
        probs.append(p)
    p64, p32 = (ctypes.byref(p) for p in probs)
    n = 4 * 9 ** 3
    o = fsi.solve_opts(restart=50, inner=torch.float32, pinned=False)
    w64 = lib.fsi_fgmres_workspace(p64, p32, ctypes.byref(o))
    o.basis = L.FSI_F32
    w32 = lib.fsi_fgmres_workspace(p64, p32, ctypes.byref(o))
    assert w64 > 0 and w32 > 0
    assert abs((w64 - w32) - 51 * n * 4) <= 512
    o.restart = 53
    assert lib.fsi_fgmres_workspace(p64, p32, ctypes.byref(o)) == 0
    assert b"restart" in lib.fsi_last_error()
    o.restart, o.inner = 50, L.FSI_F64
    assert lib.fsi_fgmres_workspace(p64, None, ctypes.byref(o)) == 0
    assert b"inner" in lib.fsi_last_error()
    o.inner, o.basis = L.FSI_F32, 7
    assert lib.fsi_fgmres_workspace(p64, p32, ctypes.byref(o)) == 0
    no = fsi.newton_opts(tol_abs=1e-8, restart=60, inner=torch.float32, basis=torch.float32, pinned=False)
    assert lib.fsi_newton_workspace(p64, p32, ctypes.byref(no)) == 0
    no.restart = 50
    assert lib.fsi_newton_workspace(p64, p32, ctypes.byref(no)) > 0
