"""Pins of the oracle's solvers on the 8^3 sphere case: FGMRES against LAPACK's
dense LU (numpy.linalg.solve) of the explicitly assembled reduced system of
section 2.4, the matrix-free Jacobian against that dense matrix, the block
diagonal against the dense diagonal blocks, and Newton's convergence."""
import numpy as np
import pytest

import fsi_workloads as W
from oracle import dlm, jacobian, krylov, newton, vms


def c1_problem(mask=True):
    cfg = W.CONFIGS["c1"]
    g = cfg.grid
    prm = vms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    a = W.advection_field(g, cfg.seed_fields)
    X = W.sphere_points()
    cell, xi = dlm.locate(g, X)
    kappa = W.kappa_weights(X.shape[1], W.sphere_volume(), cfg.c_m, cfg.alpha)
    s = dlm.s_field(g, cell, cfg.s_max)
    m = W.channel_dirichlet_mask(g) if mask else None
    return cfg, g, prm, a, cell, xi, kappa, s, m


def test_matrix_free_jacobian_equals_dense_and_blocks():
    cfg, g, prm, a, cell, xi, kappa, s, m = c1_problem()
    N = g.num_nodes
    J = jacobian.dense(g, prm, a, cell, xi, kappa, s=s, mask=m)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    y = jacobian.apply(g, prm, a, x, cell, xi, kappa, s=s, mask=m).ravel()
    assert np.abs(J @ x - y).max() <= 1e-13 * np.abs(y).max()
    blocks = jacobian.diag_blocks(g, prm, a, cell, xi, kappa, s=s, mask=m)
    for node in [0, 100, 364, 500, N - 1]:
        idx = [f * N + node for f in range(4)]
        assert np.allclose(blocks[node], J[np.ix_(idx, idx)], rtol=0, atol=1e-13 * np.abs(J).max())


def test_fgmres_matches_dense_lu():
    cfg, g, prm, a, cell, xi, kappa, s, m = c1_problem()
    N = g.num_nodes
    J = jacobian.dense(g, prm, a, cell, xi, kappa, s=s, mask=m)
    b = W.smooth_fourier_field(g, cfg.seed_vectors).ravel()
    mm = np.concatenate([m.ravel(), np.zeros(N, bool)])
    b[mm] = 0.0
    x_ref = np.linalg.solve(J, b)
    blocks = jacobian.diag_blocks(g, prm, a, cell, xi, kappa, s=s, mask=m)
    x, info = krylov.fgmres(lambda v: J @ v, b,
                            precond=lambda v: jacobian.block_jacobi_apply(blocks, v).ravel(),
                            restart=50, rtol=1e-10, max_iters=2000)
    assert info["res"] <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(b - J @ x) <= 1e-10 * np.linalg.norm(b)
    cond = np.linalg.cond(J)
    assert np.linalg.norm(x - x_ref) <= 10 * cond * 1e-10 * np.linalg.norm(x_ref)
    assert info["iters"] < 2000


def test_newton_step_converges_dense_and_fgmres_agree():
    cfg, g, prm, a, cell, xi, kappa, s, m = c1_problem()
    N = g.num_nodes
    X, Y, Z = W.node_coords(g)
    u_old = 0.5 * W.advection_field(g, cfg.seed_fields)
    gD = np.zeros((3, N))
    gD[0] = np.where(X == 0.0, 1.0, 0.0)          # plug inflow on x = 0
    gD[:, ~m[0]] = 0.0
    g_pts = np.zeros((3, cell.size))               # solid at rest
    x0 = np.concatenate([u_old, np.zeros((1, N))])
    x0[:3][m] = gD[m]
    x1, info1 = newton.solve_step(g, prm, x0, u_old, cell, xi, kappa, g_pts, s=s, mask=m, gD=gD,
                                  linear="dense")
    assert info1["converged"], info1["history"]
    h = info1["history"]
    assert h[-1] <= 1e-8 * h[0]
    assert len(h) <= 12
    x2, info2 = newton.solve_step(g, prm, x0, u_old, cell, xi, kappa, g_pts, s=s, mask=m, gD=gD,
                                  linear="fgmres", tol_abs=info1["tol_abs"])
    assert info2["converged"]
    # both satisfy the same absolute residual bound; the states agree accordingly
    assert np.linalg.norm(x1 - x2) <= 1e-6 * np.linalg.norm(x1)
    R = newton.residual(g, prm, x1, u_old, cell, xi, kappa, g_pts, s=s, mask=m, gD=gD)
    assert np.linalg.norm(R) <= info1["tol_abs"]


def _small_newton_case():
    g = W.Grid((3, 3, 3), 1)
    N = g.num_nodes
    cfg = W.CONFIGS["c1"]
    prm = vms.params_array(cfg.nu, cfg.c_m, cfg.dt)
    rng = np.random.default_rng(1)
    u_old = 0.5 * W.advection_field(g, 3)
    X = rng.uniform(0.3, 0.7, (3, 40))
    cell, xi = dlm.locate(g, X)
    kap = np.full(40, 50.0)
    gp = np.zeros((3, 40))
    m = W.channel_dirichlet_mask(g)
    gD = np.zeros((3, N))
    x0 = np.concatenate([u_old, np.zeros((1, N))])
    x0[:3][m] = 0.0
    return g, N, prm, u_old, cell, xi, kap, gp, m, gD, x0


def _central(fun, x, v, h):
    """Richardson-extrapolated central difference of fun at x along v (error O(h^4))."""
    d1 = (fun(x + h * v) - fun(x - h * v)) / (2 * h)
    d2 = (fun(x + 0.5 * h * v) - fun(x - 0.5 * h * v)) / h
    return (4.0 * d2 - d1) / 3.0


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("c_m", [1000.0, 5.0])
def test_element_tangent_is_the_derivative_of_the_element_residual(order, c_m):
    """The analytic element tangent (reactive convection, SUPG test-function and tau derivatives)
    against central differences of the element residual K(a=u, tau(u)) x - L(a=u, tau(u)) f,
    which the element-matrix pins fix; a jump in s exercises the Q2 clamp."""
    nen = (order + 1) ** 3
    h = np.array([0.3, 0.25, 0.2])
    prm = vms.params_array(0.05, c_m, 1e-2)
    rng = np.random.default_rng(40 + order)
    x_e = rng.standard_normal(4 * nen)
    f_e = rng.standard_normal(3 * nen)
    s_e = np.where(rng.uniform(size=nen) < 0.4, 100.0, 1.0)

    def r_e(xx):
        a_e = xx[:3 * nen]
        K = vms.element_matrix(order, h, prm, a_e, s_e)
        L = vms.source_matrix(order, h, prm, a_e, s_e)
        return K @ xx - L @ f_e

    T = vms.element_tangent(order, h, prm, x_e, f_e, s_e)
    for k in range(6):
        v = rng.standard_normal(4 * nen)
        ref = _central(r_e, x_e, v, 1e-3)
        got = T @ v
        for f in range(4):
            sl = slice(f * nen, (f + 1) * nen)
            assert np.linalg.norm(got[sl] - ref[sl]) <= 1e-8 * np.linalg.norm(ref[sl]), (k, f)
    # not vacuous: the full tangent differs from the Picard/Oseen element matrix
    K = vms.element_matrix(order, h, prm, x_e[:3 * nen], s_e)
    assert np.linalg.norm(T - K) > 1e-3 * np.linalg.norm(K)


@pytest.mark.parametrize("order", [1, 2])
def test_full_tangent_is_the_derivative_of_the_residual(order):
    """Global full tangent (with s, the DLM block and Dirichlet rows) against central differences
    of the step residual along directions with zero Dirichlet entries; Dirichlet rows give v."""
    g = W.Grid((3, 3, 2), order)
    N = g.num_nodes
    prm = vms.params_array(0.01, 1000.0, 1e-3)
    rng = np.random.default_rng(3 + order)
    u_old = 0.5 * W.advection_field(g, 3)
    X = rng.uniform(0.3, 0.7, (3, 40))
    cell, xi = dlm.locate(g, X)
    kap = np.full(40, 50.0)
    gp = rng.standard_normal((3, 40))
    s = dlm.s_field(g, cell, 100.0)
    m = W.channel_dirichlet_mask(g)
    gD = np.zeros((3, N))
    x = np.concatenate([u_old, np.zeros((1, N))]) + 0.3 * rng.standard_normal((4, N))

    def R(xx):
        return newton.residual(g, prm, xx, u_old, cell, xi, kap, gp, s=s, mask=m, gD=gD)

    for k in range(3):
        v = rng.standard_normal((4, N))
        vm = v.copy()
        vm[:3][m] = 0.0
        ref = _central(R, x, vm, 1e-4)
        got = newton.tangent_apply(g, prm, x, v, u_old, cell, xi, kap, s=s, mask=m)
        ref[:3][m] = v[:3][m]
        for f in range(4):
            assert np.linalg.norm(got[f] - ref[f]) <= 1e-8 * np.linalg.norm(ref[f]), (k, f)
    # the dropped derivatives are not small relative to rounding
    yp = jacobian.apply(g, prm, x[:3], v, cell, xi, kap, s=s, mask=m)
    assert np.linalg.norm(got - yp) > 1e-5 * np.linalg.norm(yp)


def test_full_tangent_newton_converges_quadratically():
    g, N, prm, u_old, cell, xi, kap, gp, m, gD, x0 = _small_newton_case()
    R0 = newton.residual(g, prm, x0, u_old, cell, xi, kap, gp, mask=m, gD=gD)
    tol = 1e-13 * np.linalg.norm(R0)
    hist = {}
    for tg in ("picard", "full"):
        x, info = newton.solve_step(g, prm, x0, u_old, cell, xi, kap, gp, mask=m, gD=gD, tol_abs=tol, tangent=tg)
        assert info["converged"]
        hist[tg] = info["history"]
    # second step: linear contraction for Picard, quadratic for the full tangent
    rp, rf = hist["picard"], hist["full"]
    assert rf[2] <= 1e-2 * rp[2], (rp, rf)
    assert rf[2] / rf[1] <= 1e-2 * (rp[2] / rp[1]), (rp, rf)
