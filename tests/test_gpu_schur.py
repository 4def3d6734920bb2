"""GPU parity of the Schur-complement block preconditioner (section 2.4: block
preconditioners built from the sub-matrices of the reduced 2x2 system).

Oracle: oracle/schur.py (coefficients per multigrid level, the V-cycle, the
block-diagonal and block-triangular applies), with the nodal blocks from
jacobian.diag_blocks and the triangular form's J (0, z_p) from jacobian.apply.
Then FGMRES and Newton with this preconditioner against dense LU / dense Newton.
"""
import numpy as np
import pytest

import fsi_workloads as W
from oracle import jacobian as ojac
from oracle import newton as onewton
from oracle import schur as oschur

from helpers import field_rel_err
from test_gpu_solve import _t, build, newton_case

pytestmark = pytest.mark.gpu


def _cavity_mask(g):
    """Every boundary node's velocity prescribed: no node fixes the pressure level."""
    nx, ny, nz = g.nodes_per_axis
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    node = ((i == 0) | (i == nx - 1) | (j == 0) | (j == ny - 1) | (k == 0) | (k == nz - 1)).ravel()
    return np.stack([node, node, node])


def _case(name):
    cfg = W.CONFIGS["c1"]
    rng = np.random.default_rng(11)
    if name == "c1":
        return build(cfg, W.advection_field(cfg.grid, cfg.seed_fields))
    if name == "c2":
        c2 = W.CONFIGS["c2"]
        return build(c2, W.advection_field(c2.grid, c2.seed_fields))
    grids = {"ragged": W.Grid((10, 12, 14), 1), "q2": W.Grid((6, 6, 6), 2), "three": W.Grid((16, 16, 16), 1),
             "single": W.Grid((3, 3, 3), 1), "cavity": W.Grid((8, 8, 8), 1)}
    g = grids[name]
    X = rng.uniform(0.15, 0.85, (3, 3000))
    kappa = rng.uniform(1.0, 50.0, 3000)
    P = build(cfg, W.advection_field(g, cfg.seed_fields), grid=g, X=X, kappa=kappa,
              mask_on=name not in ("single",))
    if name == "cavity":
        import torch
        m = _cavity_mask(g)
        mt = torch.tensor(W.mask_to_bits(m).view(np.int32), device="cuda")
        for J in (P["J64"], P["J32"]):
            J.mask = mt
            J.struct.dir_mask = mt.data_ptr()
        P["mask"] = m
    return P


def _oracle(P):
    g = P["g"]
    blocks = ojac.diag_blocks(g, P["prm_o"], P["a"], P["cell"], P["xi"], P["kappa"], s=P["s"], mask=P["mask"])
    lv = oschur.build_hierarchy(g, P["prm_o"], P["a"], s=P["s"], mask=P["mask"], cell=P["cell"], xi=P["xi"],
                                kappa=P["kappa"])
    return lv, oschur.velocity_inverses(blocks)


CASES = ["c1", "ragged", "q2", "three", "single", "cavity", "c2"]


@pytest.mark.parametrize("name", CASES)
def test_schur_levels_and_applies_match_oracle(name):
    import torch
    import paper_2601_08266_amd as fsi
    P = _case(name)
    g = P["g"]
    N = g.num_nodes
    print(f"schur {name}: grid {g.n} order {g.order}", flush=True)
    lv, finv = _oracle(P)
    _, _, blocks, nsing = fsi.bjacobi_setup(P["J64"], want32=False, want_blocks=True)
    assert nsing == 0
    pc = fsi.schur_setup(P["J64"], blocks)
    k, cells, offs = fsi.schur_info(g)
    assert k == len(lv) and cells == [L.ncell for L in lv]
    for L, off in zip(lv, offs):
        got = pc[off:off + 8 * L.alpha.size].view(torch.float64).cpu().numpy()
        err = np.linalg.norm(got - L.alpha) / np.linalg.norm(L.alpha)
        assert err <= 1e-13, (L.ncell, err)
    v = np.random.default_rng(5).standard_normal(4 * N)
    v32 = v.astype(np.float32).astype(np.float64)

    def jac(x):
        return ojac.apply(g, P["prm_o"], P["a"], x, P["cell"], P["xi"], P["kappa"], s=P["s"], mask=P["mask"])

    modes = ["schur_diag", "schur_tri"] if name != "c2" else ["schur_diag"]
    for mode in modes:
        form = "diag" if mode == "schur_diag" else "tri"
        ref = oschur.precond_apply(lv, finv, v, form, jac=jac)
        z = fsi.schur_apply(P["J64"], mode, pc, _t(v)).cpu().numpy()
        e64 = field_rel_err(z, ref, 4)
        ref32 = oschur.precond_apply(lv, finv, v32, form, jac=jac)
        z32 = fsi.schur_apply(P["J32"], mode, pc, _t(v32, "f32")).cpu().numpy()
        e32 = field_rel_err(z32, ref32, 4)
        print(f"  {mode}: FP64 {e64:.3e}  FP32 {e32:.3e}", flush=True)
        assert e64 <= 1e-12
        assert e32 <= 1e-5


@pytest.mark.parametrize("mode,inner", [("schur_diag", "f64"), ("schur_tri", "f64"), ("schur_tri", "f32"),
                                        ("schur_tri", "f32b")])
def test_fgmres_with_schur_c1_matches_dense_lu(mode, inner):
    """inner f32b: FP32 inner precision with the Krylov basis stored in FP32 (the preconditioner
    then reads FP32 basis vectors)."""
    import torch
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    P = build(cfg, W.advection_field(cfg.grid, cfg.seed_fields))
    g = P["g"]
    N = g.num_nodes
    b = W.smooth_fourier_field(g, cfg.seed_vectors).ravel()
    b[:3 * N][P["mask"].ravel()] = 0.0
    J = ojac.dense(g, P["prm_o"], P["a"], P["cell"], P["xi"], P["kappa"], s=P["s"], mask=P["mask"])
    x_ref = np.linalg.solve(J, b)
    _, _, blocks, _ = fsi.bjacobi_setup(P["J64"], want32=False, want_blocks=True)
    pc = fsi.schur_setup(P["J64"], blocks)
    x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    tdt = torch.float64 if inner == "f64" else torch.float32
    opts = fsi.solve_opts(restart=50, max_iters=3000, rtol=1e-10, inner=tdt, precond=mode,
                          basis=torch.float32 if inner == "f32b" else torch.float64)
    rc, st = fsi.fgmres_solve(P["J64"], _t(b), x, opts, J32=P["J32"] if inner != "f64" else None, pinv=pc)
    xs = x.cpu().numpy()
    res = np.linalg.norm(b - J @ xs) / np.linalg.norm(b)
    err = np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref)
    print(f"fgmres c1 {mode} inner={inner}: iters {st.iters} cycles {st.cycles} residual {res:.3e} "
          f"x err {err:.3e}")
    assert res <= 1.5e-10
    assert err <= 1e-6


@pytest.mark.parametrize("mode,pc_reuse,basis", [("schur_diag", False, "f64"), ("schur_tri", False, "f64"),
                                                 ("schur_tri", True, "f64"), ("bjacobi", True, "f64"),
                                                 ("schur_tri", True, "f32"), ("bjacobi", False, "f32")])
def test_newton_with_schur_c1_matches_dense_newton(mode, pc_reuse, basis):
    """Newton with the Schur (or block-Jacobi) preconditioner rebuilt at every iterate, or built at
    the first iterate and reused (pc_reuse), with the Krylov basis of the FP32 inner solves in
    FP64 or FP32: the same converged state as the oracle's dense Newton, within the common
    residual tolerance."""
    import torch
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    X, g_pts, kappa, u_old, mask, gD, x0 = newton_case(cfg)
    g = cfg.grid
    N = g.num_nodes
    P = build(cfg, u_old, X=X, kappa=kappa)
    kappa = P["kappa"]
    R0 = onewton.residual(g, P["prm_o"], x0, u_old, P["cell"], P["xi"], kappa, g_pts, s=P["s"],
                          mask=mask, gD=gD)
    tol = 1e-8 * np.linalg.norm(R0)
    x_ref, info = onewton.solve_step(g, P["prm_o"], x0, u_old, P["cell"], P["xi"], kappa, g_pts,
                                     s=P["s"], mask=mask, gD=gD, tol_abs=tol, linear="dense")
    assert info["converged"]
    lamg = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    fsi.dlm_BT(g, P["J64"].tables, _t(g_pts), lamg, kappa=_t(kappa))
    x = _t(x0)
    opts = fsi.newton_opts(tol_abs=tol, inner=torch.float32, precond=mode, pc_reuse=pc_reuse,
                           basis=torch.float32 if basis == "f32" else torch.float64)
    rc, st = fsi.newton_solve(P["J64"], _t(cfg.c_m * u_old), x, opts, P32=P["J32"], lamg=lamg, gD=_t(gD))
    xs = x.cpu().numpy()
    R = onewton.residual(g, P["prm_o"], xs, u_old, P["cell"], P["xi"], kappa, g_pts, s=P["s"],
                         mask=mask, gD=gD)
    print(f"newton c1 {mode} reuse={pc_reuse} basis={basis}: {st.newton_iters} Newton / {st.krylov_iters} Krylov, {st.t_total_ms:.1f} ms, "
          f"oracle ||R|| {np.linalg.norm(R):.3e} (tol {tol:.3e})")
    assert np.linalg.norm(R) <= tol * 1.01
    assert np.linalg.norm(xs - x_ref.ravel()) <= 1e-6 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("name", ["c5", "c3"])
def test_schur_full_size_properties(name):
    """Full-size workloads (192^3 Q1 + 2M points; 96^3 Q2 + 500k points), where the oracle
    cannot run whole V-cycles: level-0 alpha at sampled lattice cells against the oracle's
    formula, coarse alpha = mean of the 8 children, linearity of P^{-1}, and symmetry of the
    pressure V(2,2) cycle (Jacobi smoothing, R = P^T, exact coarse solve) in FP64 and FP32."""
    import torch
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS[name]
    print(f"schur full size {name}", flush=True)
    P = build(cfg, W.advection_field(cfg.grid, cfg.seed_fields))
    g = P["g"]
    N = g.num_nodes
    _, _, blocks, nsing = fsi.bjacobi_setup(P["J64"], want32=False, want_blocks=True)
    assert nsing == 0
    pc = fsi.schur_setup(P["J64"], blocks)
    del blocks
    k, cells, offs = fsi.schur_info(g)
    alphas = [pc[off:off + 8 * c[0] * c[1] * c[2]].view(torch.float64) for off, c in zip(offs, cells)]
    # sampled level-0 cells against the oracle's definition
    rng = np.random.default_rng(7)
    nc0 = cells[0]
    sel = rng.choice(nc0[0] * nc0[1] * nc0[2], 4000, replace=False)
    d = oschur.dlm_row_sums(g, P["cell"], P["xi"], P["kappa"])
    beta = oschur.node_beta(g, P["prm_o"], d)
    nn = g.nodes_per_axis
    cx, cy, cz = sel % nc0[0], (sel // nc0[0]) % nc0[1], sel // (nc0[0] * nc0[1])
    ids = np.stack([(cx + (o & 1)) + nn[0] * ((cy + ((o >> 1) & 1)) + nn[1] * (cz + (o >> 2))) for o in range(8)])
    nu, c_m, dt, C_T, C_I = P["prm_o"]
    a = P["a"].reshape(3, N)
    am = a[:, ids].mean(axis=1)
    sm = P["s"][ids].mean(axis=0)
    h = g.h
    tau = 1.0 / np.sqrt(sm * (C_T / dt ** 2 + sum(am[q] ** 2 / h[q] ** 2 for q in range(3))
                              + C_I * nu * nu * sum(1.0 / h[q] ** 4 for q in range(3))))
    ref = tau + beta[ids].mean(axis=0)
    got = alphas[0][torch.tensor(sel, device="cuda")].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  level-0 alpha at 4000 cells: {err:.3e}", flush=True)
    assert err <= 1e-13
    for l in range(1, k):
        f = alphas[l - 1].view(cells[l - 1][2], cells[l - 1][1], cells[l - 1][0])
        mean = 0.125 * sum(f[dz::2, dy::2, dx::2] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1))
        e = (mean.reshape(-1) - alphas[l]).abs().max().item() / alphas[l].abs().max().item()
        assert e <= 1e-15, (l, e)
    # linearity and symmetry
    for dt_, J, tol_lin, tol_sym in ((torch.float64, P["J64"], 1e-13, 1e-11), (torch.float32, P["J32"], 2e-6, 1e-4)):
        gen = torch.Generator(device="cuda").manual_seed(3)
        u = torch.randn(4 * N, dtype=dt_, device="cuda", generator=gen)
        w = torch.randn(4 * N, dtype=dt_, device="cuda", generator=gen)
        zu = fsi.schur_apply(J, "schur_diag", pc, u)
        zw = fsi.schur_apply(J, "schur_diag", pc, w)
        zc = fsi.schur_apply(J, "schur_diag", pc, 2.0 * u - 3.0 * w)
        lin = ((zc - (2.0 * zu - 3.0 * zw)).norm() / zc.norm()).item()
        up, wp, zup, zwp = u[3 * N:].double(), w[3 * N:].double(), zu[3 * N:].double(), zw[3 * N:].double()
        a1, a2 = torch.dot(zup, wp).item(), torch.dot(up, zwp).item()
        sym = abs(a1 - a2) / max(abs(a1), abs(a2))
        print(f"  {dt_}: linearity {lin:.3e}, pressure V-cycle symmetry {sym:.3e}", flush=True)
        assert lin <= tol_lin
        assert sym <= tol_sym


@pytest.mark.parametrize("name", ["c1", "ragged", "q2", "c2"])
def test_schur_velocity_steps_match_oracle(name):
    """Minimal-residual steps on the velocity block (the step lengths on the device) against
    oracle/schur.velocity_solve: block-diagonal and block-triangular forms, 1 and 3 steps."""
    import torch
    import paper_2601_08266_amd as fsi
    P = _case(name)
    g = P["g"]
    N = g.num_nodes
    print(f"schur velocity steps {name}", flush=True)
    lv, finv = _oracle(P)
    _, _, blocks, _ = fsi.bjacobi_setup(P["J64"], want32=False, want_blocks=True)
    pc = fsi.schur_setup(P["J64"], blocks)
    v = np.random.default_rng(6).standard_normal(4 * N)
    v32 = v.astype(np.float32).astype(np.float64)

    def jac(x):
        return ojac.apply(g, P["prm_o"], P["a"], x, P["cell"], P["xi"], P["kappa"], s=P["s"], mask=P["mask"])

    # FP32 bar of the triangular form: its velocity rows apply the discrete gradient to the FP32
    # pressure solve, whose rounding-level error e_p is rough (cell-scale), while the pressure
    # itself is smooth; the gradient amplifies the former relative to the latter by up to about
    # the cells per unit length n.  So the bar is max(1e-5, 2 n e_p), e_p the pressure field's
    # FP32 error measured here (block-diagonal form, same input).
    e_p = None
    for mode, form in (("schur_diag", "diag"), ("schur_tri", "tri")):
        for k in (1, 3):
            ref = oschur.precond_apply(lv, finv, v, form, jac=jac, vel_steps=k)
            z = fsi.schur_apply(P["J64"], mode, pc, _t(v), vel_steps=k).cpu().numpy()
            e64 = field_rel_err(z, ref, 4)
            ref32 = oschur.precond_apply(lv, finv, v32, form, jac=jac, vel_steps=k)
            z32 = fsi.schur_apply(P["J32"], mode, pc, _t(v32, "f32"), vel_steps=k).cpu().numpy()
            e32 = field_rel_err(z32, ref32, 4)
            if form == "diag":
                zp, rp = z32.reshape(4, N)[3], ref32.reshape(4, N)[3]
                e_p = max(e_p or 0.0, np.linalg.norm(zp - rp) / np.linalg.norm(rp))
                bar32 = 1e-5
            else:
                bar32 = max(1e-5, 2 * max(g.n) * e_p)
            print(f"  {mode} k={k}: FP64 {e64:.3e}  FP32 {e32:.3e} (bar {bar32:.2e})", flush=True)
            assert e64 <= 1e-12
            assert e32 <= bar32


@pytest.mark.parametrize("inner", ["f64", "f32"])
def test_fgmres_with_schur_velocity_steps_c1(inner):
    import torch
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    P = build(cfg, W.advection_field(cfg.grid, cfg.seed_fields))
    g = P["g"]
    N = g.num_nodes
    b = W.smooth_fourier_field(g, cfg.seed_vectors).ravel()
    b[:3 * N][P["mask"].ravel()] = 0.0
    J = ojac.dense(g, P["prm_o"], P["a"], P["cell"], P["xi"], P["kappa"], s=P["s"], mask=P["mask"])
    x_ref = np.linalg.solve(J, b)
    _, _, blocks, _ = fsi.bjacobi_setup(P["J64"], want32=False, want_blocks=True)
    pc = fsi.schur_setup(P["J64"], blocks)
    its = {}
    for k in (0, 2):
        x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
        tdt = torch.float64 if inner == "f64" else torch.float32
        opts = fsi.solve_opts(restart=50, max_iters=3000, rtol=1e-10, inner=tdt, precond="schur_tri", vel_steps=k)
        rc, st = fsi.fgmres_solve(P["J64"], _t(b), x, opts, J32=P["J32"] if inner == "f32" else None, pinv=pc)
        xs = x.cpu().numpy()
        res = np.linalg.norm(b - J @ xs) / np.linalg.norm(b)
        err = np.linalg.norm(xs - x_ref) / np.linalg.norm(x_ref)
        its[k] = st.iters
        print(f"fgmres c1 schur_tri vel_steps={k} inner={inner}: iters {st.iters} residual {res:.3e} x err {err:.3e}")
        assert res <= 1.5e-10
        assert err <= 1e-6
    assert its[2] < its[0], its
