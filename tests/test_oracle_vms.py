"""Pins of the oracle's VMS operator against closed forms, exact integrals and
consistency (section 2.1: fluid weak form and the tau_m / tau_c / G equations).

Nothing here compares the oracle with itself: every expected value comes from
analytic integrals of polynomial fields (evaluated with numpy's Gauss-Legendre
rule of much higher order than the oracle's), textbook 1D element matrices,
limits of the stabilisation parameters, or the residual-based consistency of
the stabilised form.
"""
import math

import numpy as np
import pytest

import fsi_workloads as W
from oracle import vms

NU, DT = 1.0e-2, 1.0e-3


def prm(nu=NU, c_m=1.0 / DT, dt=DT, C_T=4.0, C_I=36.0):
    return vms.params_array(nu, c_m, dt, C_T, C_I)


# ---------------------------------------------------------------- helpers
def gauss_integrate(grid, fun, npts=6):
    """Integral over the grid's box of fun(x, y, z) by tensor Gauss-Legendre per cell."""
    t, w = np.polynomial.legendre.leggauss(npts)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    total = 0.0
    for cz in range(grid.n[2]):
        for cy in range(grid.n[1]):
            for cx in range(grid.n[0]):
                xs = grid.x0[0] + (cx + t) * grid.h[0]
                ys = grid.x0[1] + (cy + t) * grid.h[1]
                zs = grid.x0[2] + (cz + t) * grid.h[2]
                Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
                WW = (w[:, None, None] * w[None, :, None] * w[None, None, :])
                total += np.sum(WW * fun(X, Y, Z)) * grid.h[0] * grid.h[1] * grid.h[2]
    return total


class Poly:
    """Tensor-product-free polynomial field given by coefficients of monomials x^i y^j z^k."""

    def __init__(self, coeffs):
        self.c = dict(coeffs)

    def __call__(self, X, Y, Z):
        out = 0.0 * X
        for (i, j, k), v in self.c.items():
            out = out + v * X ** i * Y ** j * Z ** k
        return out

    def d(self, axis):
        out = {}
        for (i, j, k), v in self.c.items():
            e = [i, j, k]
            if e[axis] == 0:
                continue
            f = v * e[axis]
            e[axis] -= 1
            out[tuple(e)] = out.get(tuple(e), 0.0) + f
        return Poly(out)


def random_poly(rng, order):
    """Random polynomial of degree <= order in each variable (exactly representable in Q_order)."""
    return Poly({(i, j, k): rng.standard_normal()
                 for i in range(order + 1) for j in range(order + 1) for k in range(order + 1)})


def nodal(grid, f):
    X, Y, Z = W.node_coords(grid)
    return f(X, Y, Z)


GRIDS = {
    1: W.Grid((3, 2, 2), 1, x0=(0.1, -0.2, 0.3), h=(0.3, 0.25, 0.2)),
    2: W.Grid((2, 2, 1), 2, x0=(0.1, -0.2, 0.3), h=(0.3, 0.25, 0.2)),
}


def quad_form(grid, prm_, a_nodal, s, terms, w, q, u, p):
    N = grid.num_nodes
    K = vms.assemble_dense(grid, prm_, a_nodal, s=s, terms=terms)
    wv = np.concatenate([nodal(grid, w[i]) for i in range(3)] + [nodal(grid, q)])
    uv = np.concatenate([nodal(grid, u[i]) for i in range(3)] + [nodal(grid, p)])
    assert wv.size == 4 * N
    return wv @ K @ uv


# --------------------------------------------------- Galerkin terms: exact integrals
@pytest.mark.parametrize("order", [1, 2])
def test_mass_integrates_polynomials_exactly(order):
    grid = GRIDS[order]
    rng = np.random.default_rng(7)
    P = random_poly(rng, order)
    N = grid.num_nodes
    a = np.zeros((3, N))
    K = vms.assemble_dense(grid, prm(c_m=1.0), a, terms=vms.MASS)
    u = nodal(grid, P)
    got = np.ones(N) @ K[:N, :N] @ u
    exact = gauss_integrate(grid, P)
    assert abs(got - exact) <= 1e-13 * max(1.0, abs(exact))
    # total mass of the constant field is the volume
    vol = np.prod(np.array(grid.n) * np.array(grid.h))
    assert abs(np.ones(N) @ K[:N, :N] @ np.ones(N) - vol) < 1e-14


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("term", ["conv", "visc", "pdiv", "cont", "mass"])
def test_galerkin_terms_match_exact_bilinear_forms(order, term):
    grid = GRIDS[order]
    rng = np.random.default_rng(11 + order)
    w = [random_poly(rng, order) for _ in range(3)]
    u = [random_poly(rng, order) for _ in range(3)]
    q, p = random_poly(rng, order), random_poly(rng, order)
    # advection field linear in each variable so that the oracle's (p+1)-point rule is exact
    a = [Poly({(0, 0, 0): rng.standard_normal(), (1, 0, 0): rng.standard_normal(),
               (0, 1, 0): rng.standard_normal(), (0, 0, 1): rng.standard_normal()}) for _ in range(3)]
    a_nodal = np.stack([nodal(grid, a[i]) for i in range(3)])
    nu, c_m = 0.37, 2.5
    flags = {"conv": vms.CONV, "visc": vms.VISC, "pdiv": vms.PDIV, "cont": vms.CONT,
             "mass": vms.MASS}[term]
    got = quad_form(grid, prm(nu=nu, c_m=c_m), a_nodal, None, flags, w, q, u, p)

    def integrand(X, Y, Z):
        if term == "mass":
            return c_m * sum(w[i](X, Y, Z) * u[i](X, Y, Z) for i in range(3))
        if term == "conv":
            return sum(w[i](X, Y, Z) * sum(a[k](X, Y, Z) * u[i].d(k)(X, Y, Z) for k in range(3))
                       for i in range(3))
        if term == "visc":
            tot = 0.0
            for i in range(3):
                for j in range(3):
                    ew = 0.5 * (w[i].d(j)(X, Y, Z) + w[j].d(i)(X, Y, Z))
                    eu = 0.5 * (u[i].d(j)(X, Y, Z) + u[j].d(i)(X, Y, Z))
                    tot = tot + 2.0 * nu * ew * eu
            return tot
        if term == "pdiv":
            return -sum(w[i].d(i)(X, Y, Z) for i in range(3)) * p(X, Y, Z)
        return q(X, Y, Z) * sum(u[i].d(i)(X, Y, Z) for i in range(3))

    exact = gauss_integrate(grid, integrand)
    scale = max(1.0, abs(exact))
    assert abs(got - exact) <= 1e-11 * scale, (got, exact)


# ------------------------------------------------ stabilisation terms (constant coefficients)


def lap_1d(order, h):
    if order == 1:
        return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h, np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    K = np.array([[7.0, -8.0, 1.0], [-8.0, 16.0, -8.0], [1.0, -8.0, 7.0]]) / (3.0 * h)
    M = np.array([[4.0, 2.0, -1.0], [2.0, 16.0, 2.0], [-1.0, 2.0, 4.0]]) * h / 30.0
    return K, M


def conv_1d(order):
    """C_ab = int_0^1 N_a N_b' (reference), closed form."""
    if order == 1:
        return np.array([[-0.5, 0.5], [-0.5, 0.5]])
    return np.array([[-0.5, 2.0 / 3.0, -1.0 / 6.0], [-2.0 / 3.0, 0.0, 2.0 / 3.0],
                     [1.0 / 6.0, -2.0 / 3.0, 0.5]])


def kron3(Ax, Ay, Az):
    # local node A = ax + q (ay + q az): z slowest
    return np.kron(Az, np.kron(Ay, Ax))


def laplacian_stiffness(order, h):
    Kx, Mx = lap_1d(order, h[0])
    Ky, My = lap_1d(order, h[1])
    Kz, Mz = lap_1d(order, h[2])
    return kron3(Kx, My, Mz) + kron3(Mx, Ky, Mz) + kron3(Mx, My, Kz)


@pytest.mark.parametrize("order", [1, 2])
def test_pspg_block_is_tau_times_textbook_laplacian(order):
    """With constant a and s, the PSPG pressure block is tau_m * int grad N_A . grad N_B."""
    h = np.array([0.3, 0.25, 0.2])
    nen = (order + 1) ** 3
    a_const = np.array([0.7, -1.3, 0.4])
    a_e = np.repeat(a_const, nen)
    s_val = 3.0
    P = prm()
    K = vms.element_matrix(order, h, P, a_e, np.full(nen, s_val), terms=vms.PSPG)
    Kpp = K[3 * nen:, 3 * nen:]
    L = laplacian_stiffness(order, h)
    tau = Kpp.ravel() @ L.ravel() / (L.ravel() @ L.ravel())
    assert np.allclose(Kpp, tau * L, rtol=0, atol=1e-14 * np.abs(Kpp).max())
    # PSPG pressure block: symmetric positive semidefinite with the constants in its kernel
    assert np.allclose(Kpp, Kpp.T, atol=1e-15 * np.abs(Kpp).max())
    ev = np.linalg.eigvalsh(Kpp)
    assert ev.min() > -1e-12 * ev.max()
    assert np.abs(Kpp @ np.ones(nen)).max() < 1e-12 * np.abs(Kpp).max()


def _pspg_tau(order, h, a_const, s_val, P):
    nen = (order + 1) ** 3
    K = vms.element_matrix(order, np.asarray(h), P, np.repeat(a_const, nen), np.full(nen, s_val),
                           terms=vms.PSPG | vms.LSIC)
    L = laplacian_stiffness(order, h)
    Kpp = K[3 * nen:, 3 * nen:]
    tau_m = Kpp.ravel() @ L.ravel() / (L.ravel() @ L.ravel())
    # LSIC block: tau_c * int d_i N_A d_j N_B ; take the (x,x) block vs Kx (x) My (x) Mz
    Kx, Mx = lap_1d(order, h[0])
    Ky, My = lap_1d(order, h[1])
    Kz, Mz = lap_1d(order, h[2])
    Gxx = kron3(Kx, My, Mz)
    Kuu = K[:nen, :nen]
    tau_c = Kuu.ravel() @ Gxx.ravel() / (Gxx.ravel() @ Gxx.ravel())
    return tau_m, tau_c


@pytest.mark.parametrize("order", [1, 2])
def test_tau_limits(order):
    """tau_m in its three limits and the s scaling (section 2.1, G = I/h^2 for [0,1] elements)."""
    h = np.array([0.125, 0.125, 0.125])
    trG = 3.0 / h[0] ** 2
    # 1) transient limit: a = 0, nu = 0, s = 1 -> tau_m = dt / sqrt(C_T)
    tm, tc = _pspg_tau(order, h, np.zeros(3), 1.0, prm(nu=0.0, dt=1e-3))
    assert math.isclose(tm, 1e-3 / 2.0, rel_tol=1e-12)
    assert math.isclose(tc, 1.0 / (tm * trG), rel_tol=1e-12)
    # 2) s scaling: tau_m ~ s^(-1/2), tau_c ~ s^(1/2)
    tm4, tc4 = _pspg_tau(order, h, np.zeros(3), 4.0, prm(nu=0.0, dt=1e-3))
    assert math.isclose(tm4, tm / 2.0, rel_tol=1e-12)
    assert math.isclose(tc4, tc * 2.0, rel_tol=1e-12)
    # 3) advective limit: dt -> inf, nu = 0, |a| = A along x -> tau_m = h / A
    A = 3.0
    tm, _ = _pspg_tau(order, h, np.array([A, 0.0, 0.0]), 1.0, prm(nu=0.0, dt=1e30, c_m=0.0))
    assert math.isclose(tm, h[0] / A, rel_tol=1e-12)
    # 4) diffusive limit: dt -> inf, a = 0 -> tau_m = h^2 / (nu sqrt(3 C_I))
    nu = 0.05
    tm, _ = _pspg_tau(order, h, np.zeros(3), 1.0, prm(nu=nu, dt=1e30, c_m=0.0))
    assert math.isclose(tm, h[0] ** 2 / (nu * math.sqrt(3.0 * 36.0)), rel_tol=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_stabilisation_terms_match_exact_forms_constant_coefficients(order):
    """SUPG + PSPG + LSIC for constant a, s: tau_m int ((a.grad)w + grad q).r_m + tau_c int div w div u."""
    grid = GRIDS[order]
    rng = np.random.default_rng(23 + order)
    w = [random_poly(rng, order) for _ in range(3)]
    u = [random_poly(rng, order) for _ in range(3)]
    q, p = random_poly(rng, order), random_poly(rng, order)
    a_c = np.array([0.9, -0.4, 1.7])
    N = grid.num_nodes
    a_nodal = np.repeat(a_c[:, None], N, axis=1)
    nu, c_m = 0.21, 3.0
    P = prm(nu=nu, c_m=c_m)
    # tau values measured from the closed-form PSPG/LSIC blocks of one cell (pinned above)
    tau_m, tau_c = _pspg_tau(order, np.array(grid.h), a_c, 1.0, P)
    got = quad_form(grid, P, a_nodal, None, vms.SUPG | vms.PSPG | vms.LSIC, w, q, u, p)

    def integrand(X, Y, Z):
        div_u = sum(u[i].d(i)(X, Y, Z) for i in range(3))
        div_w = sum(w[i].d(i)(X, Y, Z) for i in range(3))
        tot = tau_c * div_w * div_u
        for i in range(3):
            lap = sum(u[i].d(k).d(k)(X, Y, Z) for k in range(3))
            graddiv = sum(u[j].d(j).d(i)(X, Y, Z) for j in range(3))
            r = (c_m * u[i](X, Y, Z) + sum(a_c[k] * u[i].d(k)(X, Y, Z) for k in range(3))
                 + p.d(i)(X, Y, Z) - nu * (lap + graddiv))
            test = sum(a_c[k] * w[i].d(k)(X, Y, Z) for k in range(3)) + q.d(i)(X, Y, Z)
            tot = tot + tau_m * test * r
        return tot

    exact = gauss_integrate(grid, integrand)
    assert abs(got - exact) <= 1e-10 * max(1.0, abs(exact)), (got, exact)


# ------------------------------------------------ consistency (patch) tests, any tau
def interior_rows(grid):
    nx, ny, nz = grid.nodes_per_axis
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inner = ((i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    return np.concatenate([inner] * 4)


@pytest.mark.parametrize("order", [1, 2])
def test_patch_exact_solution_with_zero_strong_residual(order):
    """u = M x (M symmetric, zero diagonal), p = -c_m (m xy + n xz + k yz) - (M a).x has
    div u = 0 and r_m = 0 for constant a, so every interior row of A x vanishes for any s, tau."""
    grid = W.Grid((4, 3, 3), order, x0=(0.0, 0.0, 0.0), h=(0.25, 0.3, 0.2))
    rng = np.random.default_rng(5)
    m, n_, k = rng.standard_normal(3)
    Mx = np.array([[0, m, n_], [m, 0, k], [n_, k, 0]])
    a_c = np.array([0.8, -1.1, 0.6])
    c_m = 7.0
    X, Y, Z = W.node_coords(grid)
    u = Mx @ np.stack([X, Y, Z])
    Ma = Mx @ a_c
    p = -c_m * (m * X * Y + n_ * X * Z + k * Y * Z) - (Ma[0] * X + Ma[1] * Y + Ma[2] * Z)
    x = np.concatenate([u.ravel(), p])
    N = grid.num_nodes
    s = rng.uniform(1.0, 100.0, size=N)
    y = vms.apply(grid, prm(nu=0.3, c_m=c_m), np.repeat(a_c[:, None], N, axis=1), x, s=s)
    inner = interior_rows(grid)
    assert inner.sum() > 0
    assert np.abs(y.ravel()[inner]).max() <= 1e-11 * np.abs(y).max()
    # the boundary rows are not zero (the test is not vacuous)
    assert np.abs(y.ravel()[~inner]).max() > 1e-3


def test_patch_q2_viscous_strong_residual():
    """Q2, c_m = 0, a = (a_x,0,0): u = (phi(y,z),0,0), p = nu (phi_yy + phi_zz) x gives r_m = 0
    only if the strong residual keeps -nu lap u; dropping it must break the patch test."""
    grid = W.Grid((3, 3, 3), 2, h=(0.3, 0.25, 0.2))
    X, Y, Z = W.node_coords(grid)
    nu = 0.4
    phi = Y ** 2 + 2.0 * Z ** 2 + Y * Z + Y
    lap = 2.0 + 4.0
    N = grid.num_nodes
    x = np.concatenate([phi, 0 * phi, 0 * phi, nu * lap * X])
    a = np.stack([np.full(N, 1.3), np.zeros(N), np.zeros(N)])
    s = np.random.default_rng(3).uniform(1.0, 50.0, size=N)
    inner = interior_rows(grid)
    y = vms.apply(grid, prm(nu=nu, c_m=0.0, dt=1e30), a, x, s=s, visc_strong=True)
    assert np.abs(y.ravel()[inner]).max() <= 1e-11 * np.abs(y).max()
    y2 = vms.apply(grid, prm(nu=nu, c_m=0.0, dt=1e30), a, x, s=s, visc_strong=False)
    assert np.abs(y2.ravel()[inner]).max() > 1e-4 * np.abs(y2).max()


# ------------------------------------------------ structure and mask semantics
@pytest.mark.parametrize("order", [1, 2])
def test_structure(order):
    grid = W.Grid((3, 3, 2), order)
    N = grid.num_nodes
    rng = np.random.default_rng(1)
    a = rng.standard_normal((3, N))
    P = prm()
    # constant pressure, zero velocity: pressure rows vanish, interior momentum rows vanish
    x = np.concatenate([np.zeros(3 * N), np.full(N, 2.5)])
    y = vms.apply(grid, P, a, x, s=rng.uniform(1, 10, N))
    assert np.abs(y[3]).max() < 1e-13
    inner = interior_rows(grid)[:3 * N]
    assert np.abs(y[:3].ravel()[inner]).max() < 1e-12
    # Galerkin coupling blocks are negative transposes; mass + viscous is symmetric
    K = vms.assemble_dense(grid, P, a, terms=vms.PDIV | vms.CONT)
    assert np.allclose(K[:3 * N, 3 * N:], -K[3 * N:, :3 * N].T, atol=1e-15)
    K = vms.assemble_dense(grid, P, a, terms=vms.MASS | vms.VISC)
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())


def test_dense_apply_rows_and_mask_consistency():
    cfg = W.CONFIGS["c1"]
    g = cfg.grid
    N = g.num_nodes
    P = prm()
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    rng = np.random.default_rng(0)
    s = rng.uniform(1, 100, N)
    mask = W.channel_dirichlet_mask(g)
    y = vms.apply(g, P, a, x, s=s, mask=mask)
    A = vms.assemble_dense(g, P, a, s=s)
    m = np.concatenate([mask.ravel(), np.zeros(N, bool)])
    xm = x.copy()
    xm[m] = 0.0
    ref = A @ xm
    ref[m] = x[m]
    assert np.abs(y.ravel() - ref).max() <= 1e-13 * np.abs(ref).max()
    rows = rng.choice(4 * N, 200, replace=False)
    yr = vms.apply_rows(g, P, a, x, rows, s=s, mask=mask)
    assert np.abs(yr - y.ravel()[rows]).max() <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------ the step residual's source weighting
def _residual_patch_case(order=2):
    """Q2 grid and an exact steady state of the nonlinear step residual with a = u:
    u = M x (M symmetric, trace free: div u = 0, (u.grad)u = M^2 x), p = -x.M^2 x / 2 - phi
    (phi quadratic), u_old = u - grad(phi) / c_m, so r_m(u, p) - c_m u_old = 0 at every point."""
    grid = W.Grid((3, 3, 3), order, x0=(0.1, -0.2, 0.3), h=(0.3, 0.25, 0.2))
    rng = np.random.default_rng(17)
    A = rng.standard_normal((3, 3))
    M = A + A.T
    M -= np.trace(M) / 3.0 * np.eye(3)
    Q = rng.standard_normal((3, 3))
    Q = Q + Q.T
    b = rng.standard_normal(3)
    c_m = 40.0
    X, Y, Z = W.node_coords(grid)
    xs = np.stack([X, Y, Z])
    u = M @ xs
    M2 = M @ M
    phi = 0.5 * np.einsum("in,ij,jn->n", xs, Q, xs) + b @ xs
    p = -0.5 * np.einsum("in,ij,jn->n", xs, M2, xs) - phi
    u_old = u - (Q @ xs + b[:, None]) / c_m
    N = grid.num_nodes
    s = rng.uniform(1.0, 100.0, size=N)
    prm_ = prm(nu=0.3, c_m=c_m, dt=0.05)
    return grid, prm_, np.concatenate([u, p[None]]), c_m * u_old, s


def _assemble_residual(grid, prm_, x, f, s, src_terms):
    """Element-by-element K(a=u) x - L(a=u) f with the chosen source test functions."""
    N = grid.num_nodes
    p = grid.order
    nen = (p + 1) ** 3
    R = np.zeros(4 * N)
    for cz in range(grid.n[2]):
        for cy in range(grid.n[1]):
            for cx in range(grid.n[0]):
                ids = vms.cell_node_ids(grid, cx, cy, cz)
                x_e = np.concatenate([x[f_][ids] for f_ in range(4)])
                f_e = np.concatenate([f[d][ids] for d in range(3)])
                K = vms.element_matrix(p, grid.h, prm_, x_e[:3 * nen], s[ids])
                L = vms.source_matrix(p, grid.h, prm_, x_e[:3 * nen], s[ids], terms=src_terms)
                dofs = np.concatenate([f_ * N + ids for f_ in range(4)])
                R[dofs] += K @ x_e - L @ f_e
    return R


def test_residual_patch_exact_steady_state_with_source():
    """Interior rows of the step residual vanish for any s and tau when the source c_m u_old
    balances the strong residual: pins the Galerkin + SUPG + PSPG weighting of the source and
    a = u in the convection and in tau."""
    grid, prm_, x, f, s = _residual_patch_case()
    R = vms.residual_fluid(grid, prm_, x, f, s=s).ravel()
    inner = interior_rows(grid)
    scale = np.abs(_assemble_residual(grid, prm_, x, f, s, 0)).max()   # K x alone
    assert np.abs(R[inner]).max() <= 1e-11 * scale, np.abs(R[inner]).max() / scale
    assert np.abs(R[~inner]).max() > 1e-3 * scale   # boundary rows are not zero
    # the element-by-element sum with every source term reproduces the oracle's residual
    R_all = _assemble_residual(grid, prm_, x, f, s, vms.SRC_ALL)
    assert np.abs(R_all - R).max() <= 1e-12 * scale


@pytest.mark.parametrize("variant", ["no_supg", "no_pspg", "supg_sign", "pspg_sign", "no_gal"])
def test_residual_patch_detects_a_wrong_source_weighting(variant):
    """A plausible mistake in the source weighting (a dropped or sign-flipped SUPG / PSPG / Galerkin
    test function) breaks the patch test above."""
    grid, prm_, x, f, s = _residual_patch_case()
    terms = {"no_supg": vms.SRC_GAL | vms.SRC_PSPG, "no_pspg": vms.SRC_GAL | vms.SRC_SUPG,
             "no_gal": vms.SRC_SUPG | vms.SRC_PSPG}
    if variant in terms:
        R = _assemble_residual(grid, prm_, x, f, s, terms[variant])
    else:
        flip = vms.SRC_SUPG if variant == "supg_sign" else vms.SRC_PSPG
        R = (_assemble_residual(grid, prm_, x, f, s, vms.SRC_ALL)
             + 2.0 * (_assemble_residual(grid, prm_, x, f, s, vms.SRC_ALL & ~flip)
                      - _assemble_residual(grid, prm_, x, f, s, vms.SRC_ALL)))
    inner = interior_rows(grid)
    scale = np.abs(_assemble_residual(grid, prm_, x, f, s, 0)).max()
    assert np.abs(R[inner]).max() > 1e-6 * scale


# ------------------------------------------------ s at the quadrature points
def _lagrange_1d(order, t):
    """Values and derivatives of the 1D Lagrange polynomials on the nodes k/order at t."""
    nodes = np.arange(order + 1) / order
    val = np.ones((order + 1, t.size))
    der = np.zeros((order + 1, t.size))
    for k in range(order + 1):
        others = [m for m in range(order + 1) if m != k]
        for m in others:
            val[k] *= (t - nodes[m]) / (nodes[k] - nodes[m])
        for m in others:
            term = np.full(t.size, 1.0 / (nodes[k] - nodes[m]))
            for l in others:
                if l != m:
                    term = term * (t - nodes[l]) / (nodes[k] - nodes[l])
            der[k] += term
    return val, der


def _pspg_block_from_point_s(order, h, a_c, s_at, P):
    """tau_m(s(x_q)) int grad N_A . grad N_B by (order+1)-point Gauss with s given per point."""
    nu, dt, C_T, C_I = P[0], P[2], P[3], P[4]
    t, w = np.polynomial.legendre.leggauss(order + 1)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    val, der = _lagrange_1d(order, t)
    q = order + 1
    nen = q ** 3
    G = 1.0 / np.asarray(h) ** 2
    K = np.zeros((nen, nen))
    for iz in range(q):
        for iy in range(q):
            for ix in range(q):
                grads = np.zeros((nen, 3))
                for az in range(q):
                    for ay in range(q):
                        for ax in range(q):
                            A = ax + q * (ay + q * az)
                            grads[A] = [der[ax, ix] * val[ay, iy] * val[az, iz] / h[0],
                                        val[ax, ix] * der[ay, iy] * val[az, iz] / h[1],
                                        val[ax, ix] * val[ay, iy] * der[az, iz] / h[2]]
                sq = s_at(t[ix], t[iy], t[iz])
                bracket = C_T / dt ** 2 + np.sum(G * a_c ** 2) + C_I * nu ** 2 * np.sum(G ** 2)
                tau_m = 1.0 / np.sqrt(sq * bracket)
                K += w[ix] * w[iy] * w[iz] * np.prod(h) * tau_m * grads @ grads.T
    return K


def _nodal_s(order, fun):
    q = order + 1
    s = np.zeros(q ** 3)
    for az in range(q):
        for ay in range(q):
            for ax in range(q):
                s[ax + q * (ay + q * az)] = fun(ax / order, ay / order, az / order)
    return s


@pytest.mark.parametrize("order", [1, 2])
def test_s_is_interpolated_to_the_gauss_points(order):
    """s linear in x (so the clamp cannot act): the PSPG block equals the closed-form tau_m of
    the analytic s at each Gauss point times grad N_A . grad N_B (section 2.1 interpolates s
    with the pressure space)."""
    h = np.array([0.3, 0.25, 0.2])
    a_c = np.array([0.7, -1.3, 0.4])
    P = prm(nu=0.05, dt=2e-3)
    s_fun = lambda x, y, z: 2.0 + 60.0 * x + 25.0 * y + 9.0 * z
    nen = (order + 1) ** 3
    K = vms.element_matrix(order, h, P, np.repeat(a_c, nen), _nodal_s(order, s_fun), terms=vms.PSPG)
    ref = _pspg_block_from_point_s(order, h, a_c, s_fun, P)
    got = K[3 * nen:, 3 * nen:]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # a constant s equal to the cell mean would be a different block (the pin is not vacuous)
    ref_mean = _pspg_block_from_point_s(order, h, a_c, lambda x, y, z: s_fun(0.5, 0.5, 0.5), P)
    assert np.abs(ref_mean - ref).max() > 1e-3 * np.abs(ref).max()


def test_q2_s_clamp_keeps_tau_at_most_its_s1_value():
    """Q2 with a nodal jump of s (1 next to 100): the interpolant dips below 1 at Gauss points,
    which would give tau_m above its s = 1 value or no real tau_m at all; clamped below by the
    cell's smallest nodal s (reading of section 2.1's s), every point keeps s >= 1, so the PSPG
    block stays below the s = 1 block in the Loewner order and equals the block of the clamped
    pointwise s."""
    order = 2
    h = np.array([0.2, 0.2, 0.2])
    a_c = np.array([0.3, 0.2, -0.5])
    P = prm()
    nodal = _nodal_s(order, lambda x, y, z: 100.0 if x == 1.0 else 1.0)
    nen = 27
    # the interpolant at the first Gauss abscissa in x: 1 + 99 N_2(t0) < 1
    t0 = 0.5 * (1.0 - np.sqrt(3.0 / 5.0))
    val, _ = _lagrange_1d(order, np.array([t0]))
    assert 1.0 + 99.0 * val[2, 0] < 0.0
    K = vms.element_matrix(order, h, P, np.repeat(a_c, nen), nodal, terms=vms.PSPG)[3 * nen:, 3 * nen:]
    K1 = vms.element_matrix(order, h, P, np.repeat(a_c, nen), np.ones(nen), terms=vms.PSPG)[3 * nen:, 3 * nen:]
    assert np.all(np.isfinite(K))
    ev = np.linalg.eigvalsh(K1 - K)
    assert ev.min() >= -1e-12 * np.abs(K1).max()

    def s_clamped(x, y, z):
        vx, _ = _lagrange_1d(order, np.array([x]))
        return max(1.0 + 99.0 * vx[2, 0], 1.0)

    ref = _pspg_block_from_point_s(order, h, a_c, s_clamped, P)
    assert np.abs(K - ref).max() <= 1e-13 * np.abs(ref).max()
