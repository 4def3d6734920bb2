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

from helpers import field_rel_err

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


# each term alone on the two small meshes, all terms together on the three sizes
SOLID_CASES = [(size, terms, dtype) for dtype in ("f64", "f32")
               for size in ((3, 4), (6, 8)) for terms in ("all", "mass", "stiff", "visc")] + \
              [((12, 16), "all", dtype) for dtype in ("f64", "f32")]


@pytest.mark.parametrize("size,terms,dtype", SOLID_CASES)
def test_solid_apply_matches_oracle(size, terms, dtype):
    import paper_2601_08266_amd as fsi
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
    err = field_rel_err(y[:, rows], ref, 3)
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


# ---- the solid's residual and one coupled time step ----

def test_solid_residual_matches_oracle():
    import paper_2601_08266_amd as fsi
    for size in ((6, 8), (12, 16)):
        X0, conn, U = _mesh(*size)
        M = X0.shape[1]
        rng = np.random.default_rng(11)
        V = 0.1 * rng.standard_normal((3, M))
        A = 10.0 * rng.standard_normal((3, M))
        print(f"solid residual {size}", flush=True)
        R = fsi.solid_residual(_solid(X0, conn), _t(U), _t(V), _t(A)).cpu().numpy()
        ref = osolid.residual(X0, conn, U, V, A, MAT)
        err = field_rel_err(R, ref, 3)
        print(f"  rel err {err:.3e}")
        assert err <= TOL["f64"]


def _channel_solid(n=8, size=(6, 8), seed=3):
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((n, n, n), 1))
    g = cfg.grid
    N = g.num_nodes
    X0, conn, U_n = _mesh(*size)
    M = X0.shape[1]
    rng = np.random.default_rng(seed)
    V_n = 0.05 * rng.standard_normal((3, M))
    mask = W.channel_dirichlet_mask(g)
    nx = g.nodes_per_axis[0]
    gD = np.zeros((3, N))
    gD[0][(np.arange(N) % nx == 0) & mask[0]] = 1.0
    gD[:, ~mask[0]] = 0.0
    u_old = 0.1 * W.smooth_fourier_field(g, cfg.seed_vectors)[:3]
    x0 = np.concatenate([u_old, np.zeros((1, N))])
    x0[:3][mask] = gD[mask]
    return cfg, g, X0, conn, U_n, V_n, mask, gD, u_old, x0


def _gpu_problems(cfg, g, X0, conn, U_n, mask, inner):
    """FP64 (and FP32) problems on the solid's nodes located at the step's configuration, with the
    lumped-inertia kappa for the preconditioners."""
    import paper_2601_08266_amd as fsi
    import torch
    M = X0.shape[1]
    kappa = np.full(M, cfg.c_m * (MAT["rho_s0"] - MAT["rho_f"]) * W.plate_volume() / M)
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device="cuda")
    out = []
    for dt in ([torch.float64] + ([torch.float32] if inner == "f32" else [])):
        tab = fsi.dlm_locate(g, _t(X0 + U_n), dtype=dt, s_max=cfg.s_max)
        kt = _t(kappa, "f64" if dt == torch.float64 else "f32")
        a = torch.zeros(3 * g.num_nodes, dtype=dt, device="cuda")
        out.append(fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), a, tab, kt,
                               s=tab.s, mask=mt, gram=fsi.dlm_gram(g, tab, kt)))
    return out


def test_step_residual_matches_oracle():
    import paper_2601_08266_amd as fsi
    cfg, g, X0, conn, U_n, V_n, mask, gD, u_old, x0 = _channel_solid()
    N = g.num_nodes
    rng = np.random.default_rng(5)
    x = x0 + 0.1 * rng.standard_normal((4, N))
    x[:3][mask] = gD[mask] + 0.01
    f = cfg.c_m * u_old
    (P64,) = _gpu_problems(cfg, g, X0, conn, U_n, mask, "f64")
    R, U, V = fsi.solid_step_residual(P64, _solid(X0, conn), (_t(U_n), _t(V_n / cfg.dt), cfg.dt, 1.0 / cfg.dt),
                                      _t(f), _t(x), gD=_t(gD))
    cell, xi = odlm.locate(g, X0 + U_n)
    s = odlm.s_field(g, cell, cfg.s_max)
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    be = osolid.be_state(U_n, V_n, cfg.dt)
    ref = osolid.step_residual(g, prm_o, x, f, cell, xi, X0, conn, be, MAT, s=s, mask=mask, gD=gD)
    Vr, Ur, _ = osolid.step_state(g, cell, xi, x, *be)
    err = field_rel_err(R.cpu().numpy(), ref, 4)
    eu = field_rel_err(U.cpu().numpy(), Ur, 3)
    ev = field_rel_err(V.cpu().numpy(), Vr, 3)
    print(f"step residual rel err {err:.3e}, U {eu:.3e}, V {ev:.3e}")
    assert err <= TOL["f64"] and eu <= TOL["f64"] and ev <= TOL["f64"]


@pytest.mark.parametrize("inner,precond,vel_steps", [("f64", "schur_tri", 4), ("f32", "schur_tri", 4),
                                                     ("f32", "bjacobi", 0)])
def test_newton_with_solid_matches_oracle(inner, precond, vel_steps):
    """Two backward-Euler steps of the 8^3 channel with the 288-node elastic plates, the solid
    moving with the fluid: the library's Newton (FGMRES inner solves) against the oracle's Newton
    with dense solves, both to 1e-8 of the same initial residual per step.  The library's state
    must solve the oracle's step equations (the oracle's residual evaluated at it, from the
    library's own step-start state) to that tolerance; the two states agree to the accuracy the
    tolerance allows on this stiff system (1e-5)."""
    import paper_2601_08266_amd as fsi
    import torch
    cfg, g, X0, conn, U_n, V_n, mask, gD, u_old, x0 = _channel_solid()
    N = g.num_nodes
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    S = _solid(X0, conn)
    x_gpu = _t(x0)
    Ug, Vg = _t(U_n), _t(V_n)
    x_ref, U_ref, V_ref = x0.copy(), U_n.copy(), V_n.copy()
    for step in range(2):
        # oracle step (the configuration of step n locates the points)
        cell, xi = odlm.locate(g, X0 + U_ref)
        s = odlm.s_field(g, cell, cfg.s_max)
        f_ref = cfg.c_m * x_ref[:3]
        be = osolid.be_state(U_ref, V_ref, cfg.dt)
        R0 = osolid.step_residual(g, prm_o, x_ref, f_ref, cell, xi, X0, conn, be, MAT, s=s, mask=mask, gD=gD)
        tol = 1e-8 * np.linalg.norm(R0)
        x_ref, U_ref, V_ref, info = osolid.newton_step(g, prm_o, x_ref, f_ref, cell, xi, X0, conn, be, MAT, s=s,
                                                       mask=mask, gD=gD, tol_abs=tol)
        assert info["converged"]
        # library step from its own state
        x_prev = x_gpu.cpu().numpy().reshape(4, N).copy()
        Un_g, Vn_g = Ug.clone(), Vg.clone()
        Un_np, Vn_np = Un_g.cpu().numpy().reshape(3, -1), Vn_g.cpu().numpy().reshape(3, -1)
        probs = _gpu_problems(cfg, g, X0, conn, Un_np, mask, inner)
        f_g = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        fsi.axpby(cfg.c_m, x_gpu[:3 * N], 0.0, f_g)
        opts = fsi.newton_opts(tol, max_newton=30, inner=torch.float64 if inner == "f64" else torch.float32,
                               precond=precond, vel_steps=vel_steps, max_krylov=4000)
        rc, st = fsi.newton_solid_solve(probs[0], S, fsi.solid_be_state(Un_g, Vn_g, cfg.dt), f_g, x_gpu, Ug, Vg,
                                        opts, P32=probs[1] if inner == "f32" else None, gD=_t(gD))
        xg = x_gpu.cpu().numpy().reshape(4, N)
        cg, xig = odlm.locate(g, X0 + Un_np)
        be_g = osolid.be_state(Un_np, Vn_np, cfg.dt)
        Rg = osolid.step_residual(g, prm_o, xg, cfg.c_m * x_prev[:3], cg, xig, X0, conn, be_g, MAT,
                                  s=odlm.s_field(g, cg, cfg.s_max), mask=mask, gD=gD)
        Vo, Uo, _ = osolid.step_state(g, cg, xig, xg, *be_g)
        ex = np.linalg.norm(xg - x_ref) / np.linalg.norm(x_ref)
        eu = np.linalg.norm(Ug.cpu().numpy() - U_ref.ravel()) / np.linalg.norm(U_ref)
        print(f"step {step} {inner} {precond}: {st.newton_iters} Newton / {st.krylov_iters} Krylov, "
              f"oracle {len(info['history']) - 1} Newton; oracle residual at the library's state "
              f"{np.linalg.norm(Rg):.3e} (tol {tol:.3e}); x rel diff {ex:.3e}, U rel diff {eu:.3e}", flush=True)
        assert np.linalg.norm(Rg) <= 1.05 * tol
        assert field_rel_err(Ug.cpu().numpy(), Uo, 3) <= TOL["f64"]
        assert field_rel_err(Vg.cpu().numpy(), Vo, 3) <= TOL["f64"]
        assert ex <= 1e-5 and eu <= 1e-7


def test_jacobian_with_solid_block_sampled_full_size():
    """The benchmark's configuration (64^3 Q1, the plates meshed by 98,787 hexahedra, FP64, no
    Dirichlet rows): sampled rows of J x with the solid block.  VMS rows from the oracle's
    per-row recomputation; the solid term at a fluid node A is sum_B N_A(X_B) (K_s B x)_B over the
    solid nodes B in the cells around A, with K_s B x from the oracle's rows of the solid block."""
    import paper_2601_08266_amd as fsi
    import torch
    cfg = W.CONFIGS["c2"]
    g = cfg.grid
    N = g.num_nodes
    n_t, n_f = W.solid_mesh_size(cfg.m_points)
    X0, conn, U = _mesh(n_t, n_f)
    Xc = X0 + U
    print(f"J+solid full size: {X0.shape[1]} solid nodes, {conn.shape[0]} elements", flush=True)
    tab = fsi.dlm_locate(g, _t(Xc), dtype=torch.float64, s_max=cfg.s_max)
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    prob = fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), _t(a), tab, None, s=tab.s)
    cM, cK, cV = cfg.c_m, cfg.dt, 1.0
    y = fsi.jacobian_solid_apply(prob, _solid(X0, conn), _t(U), _t(x), cM, cK, cV).cpu().numpy()
    cell, xi = odlm.locate(g, Xc)
    s = odlm.s_field(g, cell, cfg.s_max)
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    vals, ids = odlm.point_shapes(g, cell, xi)
    rng = np.random.default_rng(9)
    # two fluid nodes of occupied cells (their rows carry the solid term) and random rows
    occ_nodes = np.unique(ids[:, cell >= 0])
    near = rng.choice(occ_nodes, 2, replace=False)
    nodes_all = np.concatenate([near, rng.choice(N, 200, replace=False)])
    rows = np.concatenate([f * N + nodes_all for f in range(4)])
    ref = ovms.apply_rows(g, prm_o, a, x, rows, s=s)
    us = odlm.apply_B(g, cell, xi, x.reshape(4, N)[:3])
    pts = np.nonzero(np.isin(ids, nodes_all).any(axis=0) & (cell >= 0))[0]
    ksu = osolid.apply_rows(X0, conn, U, us, MAT, cM, cK, cV, pts)
    solid_term = np.zeros((3, nodes_all.size))
    pos = {int(n): i for i, n in enumerate(nodes_all)}
    for j, b in enumerate(pts):
        for c in range(ids.shape[0]):
            i = pos.get(int(ids[c, b]))
            if i is not None:
                solid_term[:, i] += vals[c, b] * ksu[:, j]
    ref = ref.reshape(4, -1)
    ref[:3] += solid_term
    got = y.reshape(4, N)[:, nodes_all]
    err = field_rel_err(got, ref, 4)
    err_near = field_rel_err(got[:, :2], ref[:, :2], 4)
    print(f"  sampled rows {err:.3e}, rows with the solid term {err_near:.3e} ({pts.size} solid nodes)")
    assert np.abs(solid_term[:, :2]).max() > 0
    assert err <= TOL["f64"] and err_near <= TOL["f64"]


def test_solid_degenerate_cases():
    """Edge cases of the solid block: a mesh with nodes and no elements (K_s = 0), a single
    element, and plates sticking out of the fluid grid (solid nodes outside every cell: B gives
    them zero velocity and B^T drops their forces, but they still couple to the nodes inside)."""
    import paper_2601_08266_amd as fsi
    import torch
    X0, conn, U = _mesh(6, 8)
    M = X0.shape[1]
    v = W.random_vector(3 * M, 21).reshape(3, M)
    cM, cK, cV = COEFS["all"]
    # no elements
    S0 = fsi.Solid(_t(X0), torch.zeros(0, dtype=torch.int32, device="cuda"), **MAT)
    y0 = fsi.solid_apply(S0, _t(U), _t(v), cM, cK, cV)
    assert torch.count_nonzero(y0).item() == 0
    # one element
    y1 = fsi.solid_apply(_solid(X0, conn[:1]), _t(U), _t(v), cM, cK, cV).cpu().numpy().reshape(3, M)
    ref1 = osolid.apply(X0, conn[:1], U, v, MAT, cM, cK, cV)
    assert np.linalg.norm(y1 - ref1) <= 1e-12 * np.linalg.norm(ref1)
    assert np.count_nonzero(np.abs(ref1).sum(axis=0)) == 8
    # plates shifted by 0.3 in x: part of the solid lies outside [0, 1]^3
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((8, 8, 8), 1))
    g = cfg.grid
    N = g.num_nodes
    Xs = X0 + np.array([[0.3], [0.0], [0.0]])
    Xc = Xs + U
    tab = fsi.dlm_locate(g, _t(Xc), dtype=torch.float64, s_max=cfg.s_max)
    assert 0 < tab.n_outside < M
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    prob = fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), _t(a), tab, None, s=tab.s)
    y = fsi.jacobian_solid_apply(prob, _solid(Xs, conn), _t(U), _t(x), cM, cK, cV).cpu().numpy()
    cell, xi = odlm.locate(g, Xc)
    s = odlm.s_field(g, cell, cfg.s_max)
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    ref = osolid.jacobian_apply(g, prm_o, a, x, cell, xi, Xs, conn, U, MAT, cM, cK, cV, s=s)
    err = field_rel_err(y, ref, 4)
    print(f"solid partly outside ({tab.n_outside} of {M} nodes outside): rel err {err:.3e}")
    assert err <= TOL["f64"]


@pytest.mark.parametrize("integrator", ["be", "genalpha"])
def test_solid_channel_steps_match_oracle(integrator):
    """Two coupled steps of the 8^3 channel with the elastic plates through the library's stepper
    (solid_stepper.SolidChannel: locate, step residual, Newton, rate updates by fsi_axpby) against
    the oracle's steps (oracle/solid.genalpha_step, dense Newton), backward Euler and
    generalized-alpha with rho_inf = 0.5.  At every step the library's stage state solves the
    oracle's stage equations (built from the library's own step-start state) to the step's
    tolerance, and the states agree to what that tolerance allows on this stiff system."""
    from paper_2601_08266_amd.solid_stepper import SolidChannel, ga_coefficients
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((8, 8, 8), 1))
    g = cfg.grid
    N = g.num_nodes
    X0, conn = W.plate_solid_mesh(6, 8)
    M = X0.shape[1]
    run = SolidChannel(cfg, X0, conn, integrator=integrator, rho_inf=0.5, precond="schur_tri", vel_steps=4)
    coefs = (1.0, 1.0, 1.0) if integrator == "be" else ga_coefficients(0.5)
    am, af, gm = coefs
    dt = cfg.dt
    c = am / (gm * dt * af)
    prm_stage = ovms.params_array(cfg.nu, c, dt, cfg.C_T, cfg.C_I)
    mask = W.channel_dirichlet_mask(g)
    gD = run.gD.cpu().numpy().reshape(3, N)
    ref = dict(x=run.x.cpu().numpy().reshape(4, N), xd=np.zeros((4, N)), Vs=np.zeros((3, M)), Vsd=np.zeros((3, M)),
               U=np.zeros((3, M)))
    for step in range(2):
        start = dict(x=run.x.cpu().numpy().reshape(4, N), xd=run.xdot.cpu().numpy().reshape(4, N),
                     Vs=run.Vs.cpu().numpy().reshape(3, M), Vsd=run.Vsdot.cpu().numpy().reshape(3, M),
                     U=run.U.cpu().numpy().reshape(3, M))
        rec = run.step()
        assert rec["status"] == 0
        # the oracle's stage equations at the library's stage state
        cg, xig = odlm.locate(g, X0 + start["U"])
        sg = odlm.s_field(g, cg, cfg.s_max)
        f = c * start["x"][:3] - (1.0 - am / gm) * start["xd"][:3]
        state = (start["U"] + (af - gm) * dt * start["Vs"], c * start["Vs"] - (1.0 - am / gm) * start["Vsd"], gm * dt, c)
        Rg = osolid.step_residual(g, prm_stage, rec["stage_x"].cpu().numpy().reshape(4, N), f, cg, xig, X0, conn, state,
                                  MAT, s=sg, mask=mask, gD=gD)
        # the oracle's own step from its own state
        co, xio = odlm.locate(g, X0 + ref["U"])
        so = odlm.s_field(g, co, cfg.s_max)
        x1, xd1, Vs1, Vsd1, U1, _, info = osolid.genalpha_step(g, prm_stage, coefs, dt, ref["x"], ref["xd"], ref["Vs"],
                                                               ref["Vsd"], ref["U"], co, xio, X0, conn, MAT, s=so,
                                                               mask=mask, gD_stage=gD, tol_abs=rec["tol"])
        assert info["converged"]
        ref = dict(x=x1, xd=xd1, Vs=Vs1, Vsd=Vsd1, U=U1)
        ex = np.linalg.norm(run.x.cpu().numpy() - x1.ravel()) / np.linalg.norm(x1)
        eu = np.linalg.norm(run.U.cpu().numpy() - U1.ravel()) / np.linalg.norm(U1)
        print(f"{integrator} step {step}: {rec['newton']} Newton / {rec['krylov']} Krylov; oracle residual at the "
              f"library's stage {np.linalg.norm(Rg):.3e} (tol {rec['tol']:.3e}); x rel diff {ex:.3e}, "
              f"U rel diff {eu:.3e}", flush=True)
        assert np.linalg.norm(Rg) <= 1.05 * rec["tol"]
        assert ex <= 1e-5 and eu <= 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_jacobian_with_solid_block_q2(dtype):
    """The solid block through a Q2-Q2 fluid grid (4^3 cells of order 2): the same B / B^T with
    quadratic shape functions, against the oracle's composition, with Dirichlet rows."""
    import paper_2601_08266_amd as fsi
    import torch
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((4, 4, 4), 2))
    g = cfg.grid
    N = g.num_nodes
    tdt = torch.float64 if dtype == "f64" else torch.float32
    npdt = np.float64 if dtype == "f64" else np.float32
    X0, conn, U = _mesh(6, 8)
    Xc = X0 + U
    tab = fsi.dlm_locate(g, _t(Xc), dtype=tdt, s_max=cfg.s_max)
    a = W.advection_field(g, cfg.seed_fields).astype(npdt).astype(np.float64)
    x = W.random_vector(4 * N, cfg.seed_vectors).astype(npdt).astype(np.float64)
    mask = W.channel_dirichlet_mask(g)
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device="cuda")
    prob = fsi.Problem(g, fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I), _t(a, dtype), tab, None,
                       s=tab.s, mask=mt)
    cM, cK, cV = COEFS["all"]
    y = fsi.jacobian_solid_apply(prob, _solid(X0, conn), _t(U), _t(x, dtype), cM, cK, cV).cpu().numpy()
    cell, xi = odlm.locate(g, Xc)
    s = odlm.s_field(g, cell, cfg.s_max)
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    ref = osolid.jacobian_apply(g, prm_o, a, x, cell, xi.astype(npdt).astype(np.float64), X0, conn, U, MAT, cM, cK,
                                cV, s=s, mask=mask)
    err = field_rel_err(y, ref, 4)
    print(f"J+solid Q2 {dtype}: rel err {err:.3e} ({tab.n_occ} occupied cells)")
    assert tab.n_occ > 0 and err <= TOL[dtype]


def test_solid_channel_with_gravity_matches_oracle():
    """Plates released from rest under a body force (no inflow): two generalized-alpha steps of
    the library's stepper against the oracle's steps with the same body force."""
    from paper_2601_08266_amd.solid_stepper import SolidChannel, ga_coefficients
    cfg = dataclasses.replace(W.CONFIGS["c2"], grid=W.Grid((8, 8, 8), 1))
    g = cfg.grid
    N = g.num_nodes
    X0, conn = W.plate_solid_mesh(6, 8)
    M = X0.shape[1]
    grav = (0.0, 0.0, -9.81)
    run = SolidChannel(cfg, X0, conn, integrator="genalpha", rho_inf=0.5, precond="schur_tri", vel_steps=4,
                       inflow=0.0, gravity=grav)
    coefs = ga_coefficients(0.5)
    am, af, gm = coefs
    dt = cfg.dt
    prm_stage = ovms.params_array(cfg.nu, am / (gm * dt * af), dt, cfg.C_T, cfg.C_I)
    mask = W.channel_dirichlet_mask(g)
    gD = np.zeros((3, N))
    ref = dict(x=np.zeros((4, N)), xd=np.zeros((4, N)), Vs=np.zeros((3, M)), Vsd=np.zeros((3, M)), U=np.zeros((3, M)))
    for step in range(2):
        rec = run.step()
        assert rec["status"] == 0
        co, xio = odlm.locate(g, X0 + ref["U"])
        x1, xd1, Vs1, Vsd1, U1, _, info = osolid.genalpha_step(
            g, prm_stage, coefs, dt, ref["x"], ref["xd"], ref["Vs"], ref["Vsd"], ref["U"], co, xio, X0, conn, MAT,
            s=odlm.s_field(g, co, cfg.s_max), mask=mask, gD_stage=gD, tol_abs=rec["tol"], body=np.array(grav))
        assert info["converged"]
        ref = dict(x=x1, xd=xd1, Vs=Vs1, Vsd=Vsd1, U=U1)
        ev = np.linalg.norm(run.Vs.cpu().numpy() - Vs1.ravel()) / np.linalg.norm(Vs1)
        ex = np.linalg.norm(run.x.cpu().numpy() - x1.ravel()) / np.linalg.norm(x1)
        print(f"gravity step {step}: {rec['newton']} Newton / {rec['krylov']} Krylov; solid velocity z mean "
              f"{run.Vs.cpu().numpy().reshape(3, M)[2].mean():.3e} (oracle {Vs1[2].mean():.3e}); "
              f"x rel diff {ex:.3e}, Vs rel diff {ev:.3e}", flush=True)
        assert Vs1[2].mean() < 0.0          # the plates start to fall
        assert ex <= 1e-5 and ev <= 1e-5
