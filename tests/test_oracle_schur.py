"""Pins of the oracle's Schur-complement block preconditioner (oracle/schur.py).

The preconditioner is a design of this library (section 2.4 names block
preconditioners from the sub-matrices, not a member), so the pins check that
each piece does what its definition states, by routes that share no code with
it: the pressure stiffness against the separately pinned VMS element matrices
(the PSPG block is tau_m times that stiffness), a closed form, an energy by
Gauss quadrature of the interpolant's gradient, exact reproduction of
trilinear fields by the prolongation, the multigrid contraction, and the
effect on FGMRES iteration counts.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import fsi_workloads as W
from oracle import dlm, jacobian, krylov, schur, vms


def _prm(cfg=None):
    cfg = cfg or W.CONFIGS["c2"]
    return vms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)


def test_box_stiffness_and_tau_match_the_pspg_block():
    # constant a and s on one cell: the PSPG pressure-pressure block of the element matrix is
    # tau_m * int grad N_A . grad N_B, so it pins the box stiffness and the tau_m part of alpha
    h = (0.1, 0.07, 0.13)
    g = W.Grid((1, 1, 1), 1, h=h)
    prm = _prm()
    a_e = np.tile(np.array([0.7, -0.4, 1.1])[:, None], (1, 8))
    s_e = np.full(8, 3.0)
    K = vms.element_matrix(1, np.array(h), prm, a_e, s_e, terms=vms.PSPG)
    pp = K[24:32, 24:32]
    alpha = schur.cell_alpha(g, prm, a_e, s_e, np.zeros(8))
    assert alpha.shape == (1,)
    k = schur.box_stiffness(h)
    np.testing.assert_allclose(pp, alpha[0] * k, rtol=1e-12, atol=1e-12 * np.abs(pp).max())


def test_stiffness_closed_form_on_quadratic():
    # interior rows of K applied to the nodal samples of x^2 (constant alpha): -2 alpha v
    ncell = (6, 5, 4)
    l = (0.3, 0.2, 0.25)
    nn = tuple(c + 1 for c in ncell)
    N = nn[0] * nn[1] * nn[2]
    alpha = 1.7
    lev = schur.Level(ncell, l, np.full(ncell[0] * ncell[1] * ncell[2], alpha), np.zeros(N, dtype=bool))
    K, _ = schur.assemble(lev)
    kz, jy, ix = np.meshgrid(*(np.arange(v) for v in nn[::-1]), indexing="ij")
    for d, coord in enumerate((ix, jy, kz)):
        x = (coord.ravel() * l[d]) ** 2
        y = K @ x
        inner = ((ix > 0) & (ix < nn[0] - 1) & (jy > 0) & (jy < nn[1] - 1) & (kz > 0) & (kz < nn[2] - 1)).ravel()
        np.testing.assert_allclose(y[inner], -2.0 * alpha * l[0] * l[1] * l[2], rtol=1e-12)


def test_stiffness_energy_by_quadrature():
    # x^T K x = sum_c alpha_c int_c |grad p_h|^2, with the gradient of the trilinear interpolant
    # evaluated at 2-point Gauss points (exact for this integrand)
    rng = np.random.default_rng(5)
    ncell = (3, 2, 4)
    l = (0.2, 0.35, 0.15)
    nn = tuple(c + 1 for c in ncell)
    N = nn[0] * nn[1] * nn[2]
    alpha = rng.uniform(0.5, 2.0, ncell[0] * ncell[1] * ncell[2])
    lev = schur.Level(ncell, l, alpha, np.zeros(N, dtype=bool))
    K, _ = schur.assemble(lev)
    x = rng.standard_normal(N)
    gp = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    E = 0.0
    c = 0
    for cz in range(ncell[2]):
        for cy in range(ncell[1]):
            for cx in range(ncell[0]):
                xv = np.zeros((2, 2, 2))
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            xv[dz, dy, dx] = x[(cx + dx) + nn[0] * ((cy + dy) + nn[1] * (cz + dz))]
                for t2 in gp:
                    for t1 in gp:
                        for t0 in gp:
                            w0 = np.array([1 - t0, t0]); w1 = np.array([1 - t1, t1]); w2 = np.array([1 - t2, t2])
                            d0 = np.array([-1.0, 1.0])
                            gx = np.einsum("k,j,i,kji->", w2, w1, d0, xv) / l[0]
                            gy = np.einsum("k,j,i,kji->", w2, d0, w0, xv) / l[1]
                            gz = np.einsum("k,j,i,kji->", d0, w1, w0, xv) / l[2]
                            E += alpha[c] * 0.125 * l[0] * l[1] * l[2] * (gx * gx + gy * gy + gz * gz)
                c += 1
    assert abs(x @ (K @ x) - E) <= 1e-12 * abs(E)


def test_prolongation_reproduces_trilinear_fields():
    fine = schur.Level((8, 6, 4), (0.1, 0.1, 0.1), np.ones(8 * 6 * 4), np.zeros(9 * 7 * 5, dtype=bool))
    coarse = schur.coarsen(fine)
    P = schur._prolongation(coarse, fine)

    def field(nn, step):
        kz, jy, ix = np.meshgrid(*(np.arange(v) * step for v in nn[::-1]), indexing="ij")
        X, Y, Z = ix.ravel(), jy.ravel(), kz.ravel()
        return 1.0 + 2.0 * X - Y + 3.0 * Z + X * Y - Y * Z + 2.0 * X * Y * Z

    np.testing.assert_allclose(P @ field(coarse.nn, 2.0), field(fine.nn, 1.0), rtol=1e-14)
    # coarse alpha is the children's mean; coarse Dirichlet set by injection
    assert coarse.ncell == (4, 3, 2)
    fine.dset[:] = False
    fine.dset[0] = True
    assert schur.coarsen(fine).dset[0] and schur.coarsen(fine).dset.sum() == 1


def test_level_shapes_rule():
    assert schur.level_shapes((192, 192, 192)) == [(192,) * 3, (96,) * 3, (48,) * 3, (24,) * 3, (12,) * 3,
                                                   (6,) * 3, (3,) * 3]
    assert schur.level_shapes((64, 64, 64))[-1] == (2, 2, 2)
    assert schur.level_shapes((8, 8, 8)) == [(8, 8, 8), (4, 4, 4), (2, 2, 2)]
    assert schur.level_shapes((10, 12, 14)) == [(10, 12, 14), (5, 6, 7)]


def _poisson_levels(n, jump=1.0):
    g = W.Grid((n, n, n), 1)
    N = g.num_nodes
    lv = schur.build_hierarchy(g, _prm(), np.zeros((3, N)))
    if jump != 1.0:
        L = lv[0]
        nc = L.ncell
        cz, cy, cx = np.meshgrid(*(np.arange(c) for c in nc[::-1]), indexing="ij")
        r = np.sqrt(((cx + .5) / nc[0] - .5) ** 2 + ((cy + .5) / nc[1] - .5) ** 2 + ((cz + .5) / nc[2] - .5) ** 2)
        L.alpha = np.where(r.ravel() < 0.3, L.alpha / jump, L.alpha)
        lv = [L]
        for _ in schur.level_shapes(L.ncell)[1:]:
            lv.append(schur.coarsen(lv[-1]))
        schur.finish_hierarchy(lv)
    return lv


@pytest.mark.parametrize("jump,bound", [(1.0, 0.1), (20.0, 0.4)])
def test_vcycle_contraction(jump, bound):
    lv = _poisson_levels(16, jump)
    K = lv[0].K
    keep = ~lv[0].dset
    idx = np.flatnonzero(keep)
    rng = np.random.default_rng(1)
    b = np.where(keep, rng.standard_normal(K.shape[0]), 0.0)
    xs = np.zeros_like(b)
    xs[idx] = sla.spsolve(K[idx][:, idx].tocsc(), b[idx])
    x = np.zeros_like(b)
    errs = []
    for _ in range(5):
        x = x + schur.vcycle(lv, b - K @ x)
        errs.append(np.linalg.norm(x - xs))
    rate = (errs[-1] / errs[0]) ** 0.25
    assert rate < bound, rate


def test_single_level_solves_exactly_and_dirichlet_rows():
    g = W.Grid((3, 3, 3), 1)
    N = g.num_nodes
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, N))
    lv = schur.build_hierarchy(g, _prm(), a)
    assert len(lv) == 1
    b = rng.standard_normal(N)
    x = schur.schur_solve(lv, b)
    keep = ~lv[0].dset
    np.testing.assert_allclose((lv[0].K @ x)[keep], b[keep], rtol=1e-10, atol=1e-10 * np.abs(b).max())
    np.testing.assert_allclose(x[~keep], b[~keep] / lv[0].diag[~keep], rtol=1e-15)


def test_dirichlet_set_and_node_weights():
    g = W.Grid((4, 3, 5), 1)
    nn = g.nodes_per_axis
    m = W.channel_dirichlet_mask(g)
    ds = schur.dirichlet_set(nn, m)
    kz, jy, ix = np.meshgrid(*(np.arange(v) for v in nn[::-1]), indexing="ij")
    ix, jy, kz = ix.ravel(), jy.ravel(), kz.ravel()
    outlet_face = (ix == nn[0] - 1) & (jy > 0) & (jy < nn[1] - 1) & (kz > 0) & (kz < nn[2] - 1)
    assert np.array_equal(ds, outlet_face)
    assert schur.dirichlet_set(nn, None).sum() == g.num_nodes - (nn[0] - 2) * (nn[1] - 2) * (nn[2] - 2)
    prm = _prm()
    beta = schur.node_beta(g, prm, np.zeros(g.num_nodes))
    np.testing.assert_allclose(beta, 1.0 / prm[1], rtol=1e-15)
    # DLM row sums conserve the total kappa (partition of unity of the shape functions)
    X = W.plate_points(3000, 7)
    cell, xi = dlm.locate(g, X)
    kappa = np.random.default_rng(3).uniform(1.0, 2.0, X.shape[1])
    d = schur.dlm_row_sums(g, cell, xi, kappa)
    assert abs(d.sum() - kappa[cell >= 0].sum()) <= 1e-12 * kappa.sum()


def test_preconditioner_cuts_fgmres_iterations():
    # 16^3 channel with clustered plate points: block-Jacobi needs about 290 iterations to 1e-8,
    # the Schur-complement preconditioner (a multigrid V-cycle for the pressure) about 110 / 90,
    # with two minimal-residual velocity steps fewer still
    cfg = W.CONFIGS["c2"]
    g = W.Grid((16, 16, 16), 1)
    N = g.num_nodes
    prm = _prm(cfg)
    a = W.advection_field(g, cfg.seed_fields)
    X = W.plate_points(20000, cfg.seed_fields)
    cell, xi = dlm.locate(g, X)
    kappa = W.kappa_weights(X.shape[1], W.plate_volume(), cfg.c_m, cfg.alpha)
    s = dlm.s_field(g, cell, cfg.s_max)
    m = W.channel_dirichlet_mask(g)

    def mv(x):
        return jacobian.apply(g, prm, a, x, cell, xi, kappa, s=s, mask=m).ravel()

    b = W.smooth_fourier_field(g, cfg.seed_vectors).reshape(4, N).copy()
    b[:3][m] = 0.0
    b = b.ravel()
    blocks = jacobian.diag_blocks(g, prm, a, cell, xi, kappa, s=s, mask=m)
    lv = schur.build_hierarchy(g, prm, a, s=s, mask=m, cell=cell, xi=xi, kappa=kappa)
    finv = schur.velocity_inverses(blocks)
    its = {}
    for name, pc in (("bj", lambda v: jacobian.block_jacobi_apply(blocks, v).ravel()),
                     ("diag", lambda v: schur.precond_apply(lv, finv, v, "diag").ravel()),
                     ("tri", lambda v: schur.precond_apply(lv, finv, v, "tri", jac=mv).ravel()),
                     ("tri_mr2", lambda v: schur.precond_apply(lv, finv, v, "tri", jac=mv, vel_steps=2).ravel())):
        x, info = krylov.fgmres(mv, b, precond=pc, restart=50, rtol=1e-8, max_iters=2000)
        assert np.linalg.norm(b - mv(x)) <= 1.0001e-8 * np.linalg.norm(b)
        its[name] = info["iters"]
    assert its["diag"] < 0.5 * its["bj"] and its["tri"] <= its["diag"], its
    assert its["tri_mr2"] < 0.8 * its["tri"], its


def test_minimal_residual_velocity_steps_reduce_the_velocity_residual():
    # each minimal-residual step can only lower ||t - F z|| (alpha minimises it along F p)
    cfg = W.CONFIGS["c2"]
    g = W.Grid((8, 8, 8), 1)
    N = g.num_nodes
    prm = _prm(cfg)
    a = W.advection_field(g, cfg.seed_fields)
    X = W.plate_points(4000, cfg.seed_fields)
    cell, xi = dlm.locate(g, X)
    kappa = W.kappa_weights(X.shape[1], W.plate_volume(), cfg.c_m, cfg.alpha)
    s = dlm.s_field(g, cell, cfg.s_max)
    m = W.channel_dirichlet_mask(g)

    def jac(x):
        return jacobian.apply(g, prm, a, x, cell, xi, kappa, s=s, mask=m)

    blocks = jacobian.diag_blocks(g, prm, a, cell, xi, kappa, s=s, mask=m)
    finv = schur.velocity_inverses(blocks)
    t = np.random.default_rng(4).standard_normal((3, N))
    prev = np.inf
    for k in range(0, 5):
        z = schur.velocity_solve(finv, t, k, jac)
        xp = np.zeros((4, N))
        xp[:3] = z
        res = np.linalg.norm(t - jac(xp)[:3])
        if k >= 1:
            assert res <= prev * (1 + 1e-12), (k, res, prev)
        prev = res if k >= 1 else np.linalg.norm(t)
