"""Pins of the oracle's DLM coupling (section 2.3, eqs. nodal_solid_velo and
fsi_constraint_matrix; appendix A's locate -> parametric position -> shape
function steps): brute-force location, partition of unity, Kronecker property,
exact reproduction of Q_p fields, adjointness and force conservation."""
import numpy as np
import pytest

import fsi_workloads as W
from oracle import dlm


def special_points(grid, rng, m_random=300):
    """Random points plus points exactly on nodes, faces, edges, the boundary and outside."""
    pts = [rng.uniform(-0.05, 1.05, size=(3, m_random))]
    nodes = []
    for i in (0, 1, grid.n[0] // 2, grid.n[0]):
        for j in (0, grid.n[1] // 2, grid.n[1]):
            for k in (0, 1, grid.n[2]):
                nodes.append([grid.x0[0] + i * grid.h[0], grid.x0[1] + j * grid.h[1],
                              grid.x0[2] + k * grid.h[2]])
    nodes = np.array(nodes).T
    pts.append(nodes)
    face = rng.uniform(0.0, 1.0, size=(3, 50))
    face[0] = grid.x0[0] + 2 * grid.h[0]          # on an interior face
    pts.append(face)
    edge = rng.uniform(0.0, 1.0, size=(3, 30))
    edge[0] = grid.x0[0] + 1 * grid.h[0]
    edge[1] = grid.x0[1] + 3 * grid.h[1]
    pts.append(edge)
    out = np.array([[1.0 + 1e-12, 0.5, 0.5], [-1e-300, 0.5, 0.5], [0.5, 2.0, 0.5],
                    [np.nextafter(1.0, 2.0), 0.2, 0.2], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0]]).T
    pts.append(out)
    return np.ascontiguousarray(np.concatenate(pts, axis=1))


@pytest.mark.parametrize("n", [4, 8])
def test_locate_matches_brute_force(n):
    grid = W.Grid((n, n, n), 1)
    X = special_points(grid, np.random.default_rng(n))
    c0, xi0 = dlm.locate_bruteforce(grid, X)
    c1, xi1 = dlm.locate(grid, X)
    assert np.array_equal(c0, c1)
    assert np.array_equal(xi0.view(np.int64), xi1.view(np.int64))   # bitwise
    assert (c0 < 0).sum() >= 4
    inside = c0 >= 0
    assert np.all((xi0[:, inside] >= 0.0) & (xi0[:, inside] <= 1.0))


def test_locate_anisotropic_offset_grid_brute_force():
    grid = W.Grid((5, 3, 4), 2, x0=(-0.3, 0.1, 0.25), h=(0.2, 0.3, 0.15))
    rng = np.random.default_rng(3)
    lo = np.array(grid.x0) - 0.05
    hi = np.array(grid.x0) + np.array(grid.n) * np.array(grid.h) + 0.05
    X = lo[:, None] + (hi - lo)[:, None] * rng.uniform(size=(3, 400))
    c0, xi0 = dlm.locate_bruteforce(grid, X)
    c1, xi1 = dlm.locate(grid, X)
    assert np.array_equal(c0, c1)
    assert np.array_equal(xi0, xi1)


@pytest.mark.parametrize("order", [1, 2])
def test_B_partition_of_unity_kronecker_and_reproduction(order):
    grid = W.Grid((4, 3, 5), order)
    rng = np.random.default_rng(order)
    X = rng.uniform(0.0, 1.0, size=(3, 500))
    cell, xi = dlm.locate(grid, X)
    N = grid.num_nodes
    ones = np.ones((3, N))
    assert np.allclose(dlm.apply_B(grid, cell, xi, ones), 1.0, atol=1e-15)
    # Kronecker: points placed exactly on nodes return the nodal values
    NX, NY, NZ = W.node_coords(grid)
    pick = rng.choice(N, 60, replace=False)
    Xn = np.stack([NX[pick], NY[pick], NZ[pick]])
    cn, xin = dlm.locate(grid, Xn)
    u = rng.standard_normal((3, N))
    assert np.allclose(dlm.apply_B(grid, cn, xin, u), u[:, pick], atol=1e-13)
    # exact reproduction of a field of degree <= order in each variable
    coef = rng.standard_normal((order + 1, order + 1, order + 1))

    def P(x, y, z):
        return sum(coef[i, j, k] * x ** i * y ** j * z ** k
                   for i in range(order + 1) for j in range(order + 1) for k in range(order + 1))

    uP = np.stack([P(NX, NY, NZ), 2 * P(NX, NY, NZ), -P(NX, NY, NZ)])
    Bu = dlm.apply_B(grid, cell, xi, uP)
    exact = P(X[0], X[1], X[2])
    assert np.allclose(Bu[0], exact, atol=1e-12)
    assert np.allclose(Bu[1], 2 * exact, atol=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_BT_adjoint_dense_and_conservation(order):
    grid = W.Grid((3, 4, 3), order)
    rng = np.random.default_rng(10 + order)
    X = rng.uniform(-0.1, 1.1, size=(3, 300))
    cell, xi = dlm.locate(grid, X)
    N = grid.num_nodes
    u = rng.standard_normal((3, N))
    lam = rng.standard_normal((3, X.shape[1]))
    kappa = rng.uniform(0.5, 2.0, X.shape[1])
    Bu = dlm.apply_B(grid, cell, xi, u)
    BTl = dlm.apply_BT(grid, cell, xi, lam, kappa)
    lhs = np.sum(Bu * lam * kappa)
    rhs = np.sum(u * BTl)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    # dense B agrees with the point-by-point gather and scatter
    Bs = dlm.dense_B(grid, cell, xi)
    assert np.allclose(Bs @ u.T, Bu.T, atol=1e-13)
    assert np.allclose((Bs.T @ (kappa[:, None] * lam.T)).T, BTl, atol=1e-12)
    # force conservation: spreading preserves the total force of the inside points
    inside = cell >= 0
    assert np.allclose(BTl.sum(axis=1), (lam * kappa)[:, inside].sum(axis=1), atol=1e-12)
    # outside points contribute nothing
    assert np.all(Bu[:, ~inside] == 0.0)


def test_sort_by_cell_and_s_field():
    grid = W.Grid((4, 4, 4), 1)
    rng = np.random.default_rng(2)
    X = rng.uniform(-0.1, 1.1, size=(3, 1000))
    cell, xi = dlm.locate(grid, X)
    perm, occ, start = dlm.sort_by_cell(grid, cell)
    assert sorted(perm.tolist()) == list(range(1000))
    keys = np.where(cell[perm] >= 0, cell[perm], grid.num_cells)
    assert np.all(np.diff(keys) >= 0)
    # stable: equal keys keep increasing point index
    same = np.diff(keys) == 0
    assert np.all(np.diff(perm)[same] > 0)
    assert start[-1] == (cell >= 0).sum()
    for k in range(occ.size):
        assert np.all(cell[perm[start[k]:start[k + 1]]] == occ[k])
    s = dlm.s_field(grid, cell, 100.0)
    # brute force: a node is marked iff some occupied cell has it as a vertex
    NX, NY, NZ = W.node_coords(grid)
    inside = cell >= 0
    marked = np.zeros(grid.num_nodes, bool)
    for b in np.nonzero(inside)[0]:
        c = cell[b]
        cx, cy, cz = c % 4, (c // 4) % 4, c // 16
        lo = np.array([cx, cy, cz]) * 0.25
        near = ((NX >= lo[0] - 1e-12) & (NX <= lo[0] + 0.25 + 1e-12) & (NY >= lo[1] - 1e-12)
                & (NY <= lo[1] + 0.25 + 1e-12) & (NZ >= lo[2] - 1e-12) & (NZ <= lo[2] + 0.25 + 1e-12))
        marked |= near
    assert np.array_equal(s == 100.0, marked)
    assert np.all(s[~marked] == 1.0)
