"""GPU parity of the hyperelastic solid block (section 2.4's C^lambda dR^s/dU (C^lambda)^T
with the solid weak form of section 2.2 and the neo-Hookean energy of eq. inc_neoHk)
against oracle/solid.py: the solid apply alone on small plate meshes (every row, each
term separately and combined, FP64 and FP32), on the full 200k-node mesh by sampled rows
and by symmetry, and the reduced-system Jacobian with the solid block
(fsi_jacobian_solid_apply) against the oracle's composition of the VMS operator, B, the
solid block and B^T, with and without Dirichlet rows.
"""
import dataclasses

import numpy as np
import pytest

import fsi_workloads as W
from oracle import dlm as odlm
from oracle import solid as osolid
from oracle import vms as ovms

from helpers import field_rel_err, rows_rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
MAT = W.SOLID_MATERIAL
# backward Euler in velocity form at dt = 1e-3: (1/dt, dt, 1)
COEFS = {"all": (1.0e3, 1.0e-3, 1.0), "mass": (1.0e3, 0.0, 0.0), "stiff": (0.0, 1.0e-3, 0.0),
         "visc": (0.0, 0.0, 1.0)}


def _t(arr, dtype="f64"):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return torch.tensor(np.ascontiguousarray(arr).ravel(), dtype=tdt, device="cuda")


def _solid(X, conn):
    import paper_2601_08266_amd as fsi
    import torch
    return fsi.Solid(_t(X), torch.tensor(conn.ravel(), dtype=torch.int32, device="cuda"), **MAT)


def _mesh(n_t, n_f, seed=1001):
    X, conn = W.plate_solid_mesh(n_t, n_f)
    U = W.solid_displacement(X, seed)
    return X, conn, U


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("terms", ["all", "mass", "stiff", "visc"])
@pytest.mark.parametrize("size", [(3, 4), (6, 8), (12, 16)])
def test_solid_apply_matches_oracle(size, terms, dtype):
    import paper_2601_08266_amd as fsi
    if size == (12, 16) and terms != "all":
        pytest.skip("the separate terms are covered on the smaller meshes")
    X, conn, U = _mesh(*size)
    M = X.shape[1]
    npdt = np.float64 if dtype == "f64" else np.float32
    v = W.random_vector(3 * M, 2001).astype(npdt).astype(np.float64).reshape(3, M)
    cM, cK, cV = COEFS[terms]
    print(f"solid {size} {terms} {dtype}: {M} nodes, {conn.shape[0]} elements", flush=True)
    y = fsi.solid_apply(_solid(X, conn), _t(U), _t(v, dtype), cM, cK, cV).cpu().numpy()
    ref = osolid.apply(X, conn, U, v, MAT, cM, cK, cV)
    err = field_rel_err(y, ref, 3)
    print(f"  rel err {err:.3e}")
    assert err <= TOL[dtype]


def test_solid_apply_full_mesh_rows_symmetry_and_repeat():
    """The 200k-node plate mesh of the 64^3 workload: sampled rows against the oracle,
    <K v, w> = <v, K w>, and bitwise-equal repeats."""
    import paper_2601_08266_amd as fsi
    import torch
    n_t, n_f = W.solid_mesh_size(W.CONFIGS["c2"].m_points)
    X, conn, U = _mesh(n_t, n_f)
    M = X.shape[1]
    print(f"solid full mesh: {M} nodes, {conn.shape[0]} elements", flush=True)
    S = _solid(X, conn)
    cM, cK, cV = COEFS["all"]
    v = W.random_vector(3 * M, 2002).reshape(3, M)
    w = W.random_vector(3 * M, 2003).reshape(3, M)
    Ut = _t(U)
    y = fsi.solid_apply(S, Ut, _t(v), cM, cK, cV)
    y2 = fsi.solid_apply(S, Ut, _t(v), cM, cK, cV)
    assert torch.equal(y, y2)
    z = fsi.solid_apply(S, Ut, _t(w), cM, cK, cV)
    y = y.cpu().numpy().reshape(3, M)
    z = z.cpu().numpy().reshape(3, M)
    rows = np.random.default_rng(4).choice(M, 60, replace=False)
    ref = osolid.apply_rows(X, conn, U, v, MAT, cM, cK, cV, rows)
    err = rows_rel_err(y[:, rows], ref)
    a, b = np.sum(y * w), np.sum(v * z)
    sym = abs(a - b) / (np.linalg.norm(y) * np.linalg.norm(w))
    print(f"  sampled rows {err:.3e}, symmetry {sym:.3e}")
    assert err <= TOL["f64"]
    assert sym <= 1e-13


def _jacobian_solid_case(n, size, dtype, mask_on):
    import paper_2601_08266_amd as fsi
    import torch
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((n, n, n), 1))
    g = cfg.grid
    N = g.num_nodes
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    X0, conn, U = _mesh(*size)
    Xc = X0 + U
    tab = fsi.dlm_locate(g, _t(Xc), dtype=tdt, s_max=cfg.s_max)
    a = W.advection_field(g, cfg.seed_fields).astype(npdt).astype(np.float64)
    x = W.random_vector(4 * N, cfg.seed_vectors).astype(npdt).astype(np.float64)
    cell, xi = odlm.locate(g, Xc)
    s = odlm.s_field(g, cell, cfg.s_max)
    mask = W.channel_dirichlet_mask(g) if mask_on else None
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device="cuda") if mask_on else None
    prob = fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), _t(a, dtype), tab,
                       None, s=tab.s, mask=mt)
    cM, cK, cV = COEFS["all"]
    y = fsi.jacobian_solid_apply(prob, _solid(X0, conn), _t(U), _t(x, dtype), cM, cK, cV).cpu().numpy()
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    ref = osolid.jacobian_apply(g, prm_o, a, x, cell, xi.astype(npdt).astype(np.float64), X0, conn, U, MAT,
                                cM, cK, cV, s=s, mask=mask)
    return y, ref, tab.n_occ


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("mask_on", [False, True])
@pytest.mark.parametrize("n,size", [(8, (6, 8)), (16, (12, 16))])
def test_jacobian_with_solid_block_matches_oracle(n, size, dtype, mask_on):
    print(f"J+solid {n}^3 mesh {size} {dtype} mask={mask_on}", flush=True)
    y, ref, n_occ = _jacobian_solid_case(n, size, dtype, mask_on)
    assert n_occ > 0
    err = field_rel_err(y, ref, 4)
    print(f"  rel err {err:.3e} ({n_occ} occupied cells)")
    assert err <= TOL[dtype]


def test_setup_rejects_connectivity_out_of_range():
    import paper_2601_08266_amd as fsi
    X, conn = W.plate_solid_mesh(3, 4)
    bad = conn.copy()
    bad[5, 3] = X.shape[1]
    with pytest.raises(fsi.FsiError, match="connectivity"):
        _solid(X, bad)


def _solid_problem(n, size, dtype, mask_on):
    """Problem whose applies carry the solid block; kappa = the solid's lumped inertia
    c_M (rho_s0 - rho_f) V / M per point (with its per-cell blocks) feeds the preconditioners."""
    import paper_2601_08266_amd as fsi
    import torch
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((n, n, n), 1))
    g = cfg.grid
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X0, conn, U = _mesh(*size)
    M = X0.shape[1]
    cM, cK, cV = COEFS["all"]
    tab = fsi.dlm_locate(g, _t(X0 + U), dtype=tdt, s_max=cfg.s_max)
    kappa = np.full(M, cM * (MAT["rho_s0"] - MAT["rho_f"]) * W.plate_volume() / M)
    kt = _t(kappa, dtype)
    a = W.advection_field(g, cfg.seed_fields)
    mask = W.channel_dirichlet_mask(g) if mask_on else None
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device="cuda") if mask_on else None
    S = _solid(X0, conn)
    Ut = _t(U)
    prob = fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), _t(a, dtype), tab, kt,
                       s=tab.s, mask=mt, gram=fsi.dlm_gram(g, tab, kt), solid=S, solid_U=Ut,
                       solid_coefs=(cM, cK, cV))
    return dict(cfg=cfg, g=g, prob=prob, S=S, Ut=Ut, X0=X0, conn=conn, U=U, a=a, mask=mask, tab=tab)


def test_problem_with_solid_applies_the_solid_block():
    import paper_2601_08266_amd as fsi
    import torch
    c = _solid_problem(8, (6, 8), "f64", True)
    N = c["g"].num_nodes
    x = _t(W.random_vector(4 * N, 7))
    y1 = fsi.jacobian_apply(c["prob"], x)
    y2 = fsi.jacobian_solid_apply(c["prob"], c["S"], c["Ut"], x, *COEFS["all"])
    assert torch.equal(y1, y2)
    with pytest.raises(fsi.FsiError, match="solid"):
        fsi.vms_residual(c["prob"], torch.zeros(3 * N, dtype=torch.float64, device="cuda"), x,
                         gD=torch.zeros(3 * N, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("inner,precond", [("f64", "bjacobi"), ("f32", "bjacobi"), ("f32", "schur_tri")])
def test_fgmres_with_solid_block_matches_dense_solve(inner, precond):
    """FGMRES on J = A + B^T K_s B (8^3 channel, 288-node plate mesh) against LAPACK on the
    oracle's dense matrix."""
    import paper_2601_08266_amd as fsi
    import torch
    c64 = _solid_problem(8, (6, 8), "f64", True)
    c32 = _solid_problem(8, (6, 8), "f32", True) if inner == "f32" else None
    g, cfg = c64["g"], c64["cfg"]
    N = g.num_nodes
    cell, xi = odlm.locate(g, c64["X0"] + c64["U"])
    s = odlm.s_field(g, cell, cfg.s_max)
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    J = osolid.jacobian_dense(g, prm_o, c64["a"], cell, xi, c64["X0"], c64["conn"], c64["U"], MAT,
                              *COEFS["all"], s=s, mask=c64["mask"])
    b = W.smooth_fourier_field(g, cfg.seed_vectors).ravel()
    b[:3 * N][c64["mask"].ravel()] = 0.0
    x_ref = np.linalg.solve(J, b)
    tdt = torch.float64 if inner == "f64" else torch.float32
    pinv64, pinv32, blocks, _ = fsi.bjacobi_setup(c64["prob"], want_blocks=True)
    pc = pinv32 if inner == "f32" else pinv64
    if precond != "bjacobi":
        pc = fsi.schur_setup(c64["prob"], blocks)
    opts = fsi.solve_opts(restart=50, max_iters=4000, rtol=1e-10, inner=tdt, precond=precond)
    x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    rc, st = fsi.fgmres_solve(c64["prob"], _t(b), x, opts, J32=c32["prob"] if c32 else None, pinv=pc)
    xs = x.cpu().numpy()
    res = np.linalg.norm(b - J @ xs) / np.linalg.norm(b)
    err = np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref)
    print(f"fgmres+solid inner={inner} {precond}: {st.iters} it, oracle residual {res:.3e}, x err {err:.3e}")
    assert res <= 1.5e-10
    assert err <= 1e-6
