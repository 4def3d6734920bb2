"""Pins of the oracle's hyperelastic solid block (oracle/solid.py; section 2.2's solid weak
form with section 4.3's nearly-incompressible neo-Hookean energy, eq. inc_neoHk).

* The reference state is stress free; a pure dilation stores only the volumetric energy.
* P is the gradient of psi, and dP the derivative of P (central differences).
* At F = I the tangent is isotropic linear elasticity with shear modulus C0 and bulk
  modulus kappa_s, and on a box element the stiffness equals the textbook
  int B^T D B with engineering strains in Voigt form (an independent construction);
  the viscous matrix equals the same with (lambda, mu) = (0, mu_f).
* Element force = gradient of element energy; element tangent = derivative of the
  element force; the force is objective (rotates with the configuration).
* Rigid translations are in the null space of the stiffness, rigid motions of the
  current configuration in that of the viscous matrix.
* The consistent mass matrix of a box matches the tensor product of the 1D linear mass
  matrices; the mesh volume matches the shells' analytic volume.
"""
import math

import numpy as np
import pytest

import fsi_workloads as W
from oracle import solid

PRM = dict(C0=1.0e5, kappa_s=1.0e4, rho_s0=1.5, rho_f=1.0, mu_f=0.01)


def _rand_F(rng, amp=0.3):
    F = np.eye(3) + amp * rng.standard_normal((3, 3))
    if np.linalg.det(F) <= 0.2:
        F[0] *= -1.0 if np.linalg.det(F) < 0 else 1.0
        F += np.eye(3)
    assert np.linalg.det(F) > 0.1
    return F


def test_reference_state_is_stress_free_and_dilation_is_volumetric():
    C0, kap = PRM["C0"], PRM["kappa_s"]
    assert solid.energy(np.eye(3), C0, kap) == pytest.approx(0.0, abs=1e-12)
    assert np.abs(solid.piola(np.eye(3), C0, kap)).max() <= 1e-9
    for s in (0.9, 1.05, 1.3):
        J = s ** 3
        expect = 0.5 * kap * (0.5 * (J * J - 1.0) - math.log(J))
        assert solid.energy(s * np.eye(3), C0, kap) == pytest.approx(expect, rel=1e-12)
        # the isochoric stress vanishes: P = kap/2 (J^2 - 1) F^{-T}
        np.testing.assert_allclose(solid.piola(s * np.eye(3), C0, kap),
                                   0.5 * kap * (J * J - 1.0) / s * np.eye(3), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_piola_is_energy_gradient(seed):
    rng = np.random.default_rng(seed)
    F = _rand_F(rng)
    C0, kap = PRM["C0"], PRM["kappa_s"]
    P = solid.piola(F, C0, kap)
    h = 1e-6
    Pfd = np.empty((3, 3))
    for i in range(3):
        for K in range(3):
            E = np.zeros((3, 3))
            E[i, K] = h
            Pfd[i, K] = (solid.energy(F + E, C0, kap) - solid.energy(F - E, C0, kap)) / (2 * h)
    assert np.abs(P - Pfd).max() <= 1e-6 * np.abs(P).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tangent_is_piola_derivative(seed):
    rng = np.random.default_rng(10 + seed)
    F = _rand_F(rng)
    dF = rng.standard_normal((3, 3))
    C0, kap = PRM["C0"], PRM["kappa_s"]
    h = 1e-6
    fd = (solid.piola(F + h * dF, C0, kap) - solid.piola(F - h * dF, C0, kap)) / (2 * h)
    dP = solid.piola_tangent(F, dF, C0, kap)
    assert np.abs(dP - fd).max() <= 1e-6 * np.abs(dP).max()
    # major symmetry of the elasticity tensor (hyperelastic)
    A = solid.elasticity_tensor(F, C0, kap)
    assert np.abs(A - A.transpose(2, 3, 0, 1)).max() <= 1e-9 * np.abs(A).max()


def _voigt_stiffness(Xe, lam, mu):
    """Textbook int B^T D B over a hex (engineering strains, Voigt order xx yy zz yz xz xy)."""
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[[0, 1, 2], [0, 1, 2]] += 2 * mu
    D[[3, 4, 5], [3, 4, 5]] = mu
    K = np.zeros((24, 24))
    for q in range(8):
        _, dN = solid.shape(solid.GAUSS[q])
        J0 = Xe.T @ dN
        G = dN @ np.linalg.inv(J0)
        B = np.zeros((6, 24))
        for a in range(8):
            gx, gy, gz = G[a]
            B[0, 3 * a] = gx
            B[1, 3 * a + 1] = gy
            B[2, 3 * a + 2] = gz
            B[3, 3 * a + 1], B[3, 3 * a + 2] = gz, gy
            B[4, 3 * a], B[4, 3 * a + 2] = gz, gx
            B[5, 3 * a], B[5, 3 * a + 1] = gy, gx
        K += solid.GAUSS_W * np.linalg.det(J0) * B.T @ D @ B
    return K


def _box(a=0.02, b=0.01, c=0.005, skew=0.0):
    Xe = np.array([[(i & 1) * a, ((i >> 1) & 1) * b, (i >> 2) * c] for i in range(8)], dtype=np.float64)
    Xe[:, 0] += skew * Xe[:, 1]
    return Xe


def test_small_strain_limit_is_linear_elasticity():
    C0, kap = PRM["C0"], PRM["kappa_s"]
    lam, mu = kap - 2.0 / 3.0 * C0, C0
    d = np.eye(3)
    iso = lam * np.einsum("iK,jL->iKjL", d, d) + mu * (np.einsum("ij,KL->iKjL", d, d) +
                                                       np.einsum("iL,Kj->iKjL", d, d))
    A = solid.elasticity_tensor(np.eye(3), C0, kap)
    assert np.abs(A - iso).max() <= 1e-9 * np.abs(iso).max()
    for skew in (0.0, 0.4):
        Xe = _box(skew=skew)
        M, K, Kv = solid.element_matrices(Xe, np.zeros((8, 3)), PRM)
        Kref = _voigt_stiffness(Xe, lam, mu)
        assert np.abs(K - Kref).max() <= 1e-10 * np.abs(Kref).max()
        Kvref = _voigt_stiffness(Xe, 0.0, PRM["mu_f"])
        assert np.abs(Kv - Kvref).max() <= 1e-10 * np.abs(Kvref).max()


def _deformed_element(seed=3):
    X, conn = W.plate_solid_mesh(6, 8)
    U = W.solid_displacement(X, seed, rotation_deg=25.0, amp=0.004)
    e = 17
    return X[:, conn[e]].T.copy(), U[:, conn[e]].T.copy()


def test_element_force_is_energy_gradient_and_tangent_its_derivative():
    Xe, Ue = _deformed_element()
    f = solid.element_force(Xe, Ue, PRM)
    h = 1e-8
    ffd = np.empty((8, 3))
    for a in range(8):
        for i in range(3):
            E = np.zeros((8, 3))
            E[a, i] = h
            ffd[a, i] = (solid.element_energy(Xe, Ue + E, PRM) - solid.element_energy(Xe, Ue - E, PRM)) / (2 * h)
    assert np.abs(f - ffd).max() <= 1e-5 * np.abs(f).max()
    _, K, _ = solid.element_matrices(Xe, Ue, PRM)
    h = 1e-7
    Kfd = np.empty((24, 24))
    for col in range(24):
        E = np.zeros(24)
        E[col] = h
        E = E.reshape(8, 3)
        Kfd[:, col] = ((solid.element_force(Xe, Ue + E, PRM) - solid.element_force(Xe, Ue - E, PRM))
                       / (2 * h)).reshape(24)
    assert np.abs(K - Kfd).max() <= 1e-6 * np.abs(K).max()
    assert np.abs(K - K.T).max() <= 1e-9 * np.abs(K).max()


def test_force_is_objective():
    Xe, Ue = _deformed_element()
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0.0], [math.sin(th), math.cos(th), 0.0], [0.0, 0.0, 1.0]])
    x = Xe + Ue
    Ur = x @ R.T - Xe
    f = solid.element_force(Xe, Ue, PRM)
    fr = solid.element_force(Xe, Ur, PRM)
    assert np.abs(fr - f @ R.T).max() <= 1e-9 * np.abs(f).max()


def test_rigid_motions_null_spaces():
    Xe, Ue = _deformed_element()
    M, K, Kv = solid.element_matrices(Xe, Ue, PRM)
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1.0
        assert np.abs(K @ t.reshape(24)).max() <= 1e-9 * np.abs(K).max()
        assert np.abs(Kv @ t.reshape(24)).max() <= 1e-9 * np.abs(Kv).max()
    # rigid rotation of the current configuration: v = w x (X + U)
    x = Xe + Ue
    for w in np.eye(3):
        v = np.cross(w, x)
        assert np.abs(Kv @ v.reshape(24)).max() <= 1e-9 * np.abs(Kv).max() * np.abs(v).max()


def test_box_mass_matrix_is_tensor_product_of_1d_mass():
    a, b, c = 0.02, 0.01, 0.005
    Xe = _box(a, b, c)
    M, _, _ = solid.element_matrices(Xe, np.zeros((8, 3)), PRM)
    rho = PRM["rho_s0"] - PRM["rho_f"]
    ref = np.zeros((24, 24))
    for A in range(8):
        for B in range(8):
            f = 1.0
            for d in range(3):
                f *= 2.0 if ((A >> d) & 1) == ((B >> d) & 1) else 1.0
            ref[3 * A:3 * A + 3, 3 * B:3 * B + 3] = rho * a * b * c / 216.0 * f * np.eye(3)
    assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()


def test_mesh_volume_matches_shells():
    X, conn = W.plate_solid_mesh(40, 60)
    vol = 0.0
    for e in range(0, conn.shape[0]):
        Xe = X[:, conn[e]].T
        for q in range(8):
            _, dN = solid.shape(solid.GAUSS[q])
            d = np.linalg.det(Xe.T @ dN)
            assert d > 0
            vol += solid.GAUSS_W * d
    r0, r1 = W.PLATE_R
    t0, t1 = (math.radians(v) for v in W.PLATE_T_DEG)
    dphi = math.radians(120.0 - 2 * W.PLATE_MARGIN_DEG)
    exact = 3 * (r1 ** 3 - r0 ** 3) / 3.0 * (math.cos(t0) - math.cos(t1)) * dphi
    assert abs(vol / exact - 1.0) <= 2e-3, vol / exact


def test_mesh_apply_is_symmetric_sum_of_element_blocks():
    X, conn = W.plate_solid_mesh(3, 4)
    U = W.solid_displacement(X, 5)
    rng = np.random.default_rng(0)
    M = X.shape[1]
    cM, cK, cV = 1000.0, 1e-3, 1.0
    # dense operator from unit vectors
    D = np.empty((3 * M, 3 * M))
    for k in range(3 * M):
        e = np.zeros(3 * M)
        e[k] = 1.0
        D[:, k] = solid.apply(X, conn, U, e.reshape(3, M), PRM, cM, cK, cV).reshape(-1)
    assert np.abs(D - D.T).max() <= 1e-10 * np.abs(D).max()
    v = rng.standard_normal((3, M))
    y = solid.apply(X, conn, U, v, PRM, cM, cK, cV)
    np.testing.assert_allclose(y.reshape(-1), D @ v.reshape(-1), rtol=1e-12, atol=1e-12 * np.abs(y).max())
    rows = np.array([0, 5, M - 1])
    np.testing.assert_allclose(solid.apply_rows(X, conn, U, v, PRM, cM, cK, cV, rows), y[:, rows],
                               rtol=1e-12, atol=1e-12 * np.abs(y).max())


def test_mass_total_is_solid_minus_displaced_fluid():
    """t^T M t for a unit translation t = rho_s0 V_0 - rho_f V_t, with the current volume V_t
    measured on the current coordinates (det of dx/dxi)."""
    Xe, Ue = _deformed_element()
    M, _, _ = solid.element_matrices(Xe, Ue, PRM)
    V0 = Vt = 0.0
    for q in range(8):
        _, dN = solid.shape(solid.GAUSS[q])
        V0 += solid.GAUSS_W * np.linalg.det(Xe.T @ dN)
        Vt += solid.GAUSS_W * np.linalg.det((Xe + Ue).T @ dN)
    assert abs(Vt / V0 - 1.0) > 1e-4          # the state really changes the volume
    for d in range(3):
        t = np.zeros((8, 3))
        t[:, d] = 1.0
        tv = t.reshape(24)
        expect = PRM["rho_s0"] * V0 - PRM["rho_f"] * Vt
        assert tv @ M @ tv == pytest.approx(expect, rel=1e-12)


def test_dense_assemblies_match_the_applies():
    from oracle import dlm, vms
    X, conn = W.plate_solid_mesh(3, 4)
    U = W.solid_displacement(X, 5)
    M = X.shape[1]
    v = np.random.default_rng(1).standard_normal((3, M))
    K = solid.dense(X, conn, U, PRM, 1e3, 1e-3, 1.0)
    y = solid.apply(X, conn, U, v, PRM, 1e3, 1e-3, 1.0)
    assert np.abs(K @ v.reshape(-1) - y.reshape(-1)).max() <= 1e-12 * np.abs(y).max()
    g = W.Grid((4, 4, 4), 1)
    N = g.num_nodes
    cell, xi = dlm.locate(g, X + U)
    a = W.advection_field(g, 1001)
    prm_f = vms.params_array(0.01, 1000.0, 1e-3)
    mask = W.channel_dirichlet_mask(g)
    x = np.random.default_rng(2).standard_normal(4 * N)
    J = solid.jacobian_dense(g, prm_f, a, cell, xi, X, conn, U, PRM, 1e3, 1e-3, 1.0, mask=mask)
    yj = solid.jacobian_apply(g, prm_f, a, x, cell, xi, X, conn, U, PRM, 1e3, 1e-3, 1.0, mask=mask)
    assert np.abs(J @ x - yj.reshape(-1)).max() <= 1e-12 * np.abs(yj).max()


def test_solid_residual_pins():
    """R^s vanishes for a rigid rotation at rest; uniform acceleration gives the net inertia
    (rho_s0 - rho_f) V a; and its derivative along the backward-Euler path (U + e dt d,
    V + e d, A + e d / dt) is the tangent block with (1/dt, dt, 1): exactly (to difference
    accuracy) without the fluid-density and viscous terms, whose geometric derivatives the
    block drops, and to 1e-5 with them."""
    X, conn = W.plate_solid_mesh(3, 4)
    M = X.shape[1]
    U = W.solid_displacement(X, 5)
    rng = np.random.default_rng(0)
    V = 0.1 * rng.standard_normal((3, M))
    A = rng.standard_normal((3, M))
    d = rng.standard_normal((3, M))
    dt = 1e-3
    th = 0.3
    rel = X - 0.5
    Ur = np.stack([np.zeros(M), (math.cos(th) - 1) * rel[1] - math.sin(th) * rel[2],
                   math.sin(th) * rel[1] + (math.cos(th) - 1) * rel[2]])
    zero = np.zeros((3, M))
    Rd = solid.residual(X, conn, U, zero, zero, PRM)
    assert np.abs(solid.residual(X, conn, Ur, zero, zero, PRM)).max() <= 1e-9 * np.abs(Rd).max()
    a = np.array([0.3, -1.0, 2.0])
    R0 = solid.residual(X, conn, zero, zero, np.tile(a[:, None], (1, M)), PRM)
    vol = 0.0
    for e in range(conn.shape[0]):
        Xe = X[:, conn[e]].T
        for q in range(8):
            _, dN = solid.shape(solid.GAUSS[q])
            vol += solid.GAUSS_W * np.linalg.det(Xe.T @ dN)
    np.testing.assert_allclose(R0.sum(axis=1), (PRM["rho_s0"] - PRM["rho_f"]) * vol * a, rtol=1e-12)
    for prm, tol in ((dict(PRM, rho_f=0.0, mu_f=0.0), 1e-7), (PRM, 1e-5)):
        e = 1e-6
        fd = (solid.residual(X, conn, U + e * dt * d, V + e * d, A + e * d / dt, prm)
              - solid.residual(X, conn, U - e * dt * d, V - e * d, A - e * d / dt, prm)) / (2 * e)
        K = solid.apply(X, conn, U, d, prm, 1.0 / dt, dt, 1.0)
        assert np.linalg.norm(fd - K) <= tol * np.linalg.norm(K)


def test_coupled_newton_step_converges():
    """One backward-Euler step of the channel with the solid block (4^3 grid, 72-node plates):
    Newton with the Picard/frozen-configuration matrix reaches 1e-8 of the initial residual."""
    from oracle import dlm, vms
    g = W.Grid((4, 4, 4), 1)
    N = g.num_nodes
    X, conn = W.plate_solid_mesh(3, 4)
    M = X.shape[1]
    U_n = W.solid_displacement(X, 5)
    V_n = np.zeros((3, M))
    dt = 1e-3
    cell, xi = dlm.locate(g, X + U_n)
    prm_f = vms.params_array(0.01, 1.0 / dt, dt)
    mask = W.channel_dirichlet_mask(g)
    nx = g.nodes_per_axis[0]
    gD = np.zeros((3, N))
    inflow = (np.arange(N) % nx == 0)
    gD[0][inflow] = 1.0
    x0 = np.zeros((4, N))
    x0[:3][mask] = gD[mask]
    f = (1.0 / dt) * np.zeros((3, N))
    x, U, V, info = solid.newton_step(g, prm_f, x0, f, cell, xi, X, conn, solid.be_state(U_n, V_n, dt), PRM,
                                      mask=mask, gD=gD)
    print("coupled step residuals", ["%.2e" % h for h in info["history"]])
    assert info["converged"] and len(info["history"]) <= 8
    np.testing.assert_allclose(U, U_n + dt * V, rtol=1e-14, atol=1e-16)


def test_coupled_genalpha_with_unit_coefficients_is_backward_euler():
    from oracle import dlm, vms
    g = W.Grid((4, 4, 4), 1)
    N = g.num_nodes
    X, conn = W.plate_solid_mesh(3, 4)
    M = X.shape[1]
    U_n = W.solid_displacement(X, 5)
    rng = np.random.default_rng(2)
    V_n = 0.05 * rng.standard_normal((3, M))
    dt = 1e-3
    cell, xi = dlm.locate(g, X + U_n)
    prm_f = vms.params_array(0.01, 1.0 / dt, dt)
    mask = W.channel_dirichlet_mask(g)
    gD = np.zeros((3, N))
    gD[0][np.arange(N) % g.nodes_per_axis[0] == 0] = 1.0
    x_n = np.zeros((4, N))
    x_n[:3][mask] = gD[mask]
    x1, xdot1, Vs1, _, U1, x_st, info = solid.genalpha_step(g, prm_f, (1.0, 1.0, 1.0), dt, x_n, np.zeros((4, N)),
                                                            V_n, np.zeros((3, M)), U_n, cell, xi, X, conn, PRM,
                                                            mask=mask, gD_stage=gD)
    xb, Ub, Vb, _ = solid.newton_step(g, prm_f, x_n, (1.0 / dt) * x_n[:3], cell, xi, X, conn,
                                      solid.be_state(U_n, V_n, dt), PRM, mask=mask, gD=gD)
    assert info["converged"]
    assert np.abs(x1 - xb).max() <= 1e-12 * np.abs(xb).max()
    assert np.abs(U1 - Ub).max() <= 1e-12 * np.abs(Ub).max()
    np.testing.assert_allclose(Vs1, Vb, rtol=1e-10, atol=1e-12 * np.abs(Vb).max())


def test_body_force_enters_as_a_shift_of_the_acceleration():
    """R^s(U, V, A; f) = R^s(U, V, A - f): the body force of eq. solid_weak_form's inertia term;
    a stress-free solid at rest in free fall (A = f) has zero residual."""
    X, conn = W.plate_solid_mesh(3, 4)
    M = X.shape[1]
    U = W.solid_displacement(X, 5)
    rng = np.random.default_rng(4)
    V = 0.1 * rng.standard_normal((3, M))
    A = rng.standard_normal((3, M))
    fb = np.array([0.0, 0.0, -9.81])
    np.testing.assert_allclose(solid.residual(X, conn, U, V, A, PRM, body=fb),
                               solid.residual(X, conn, U, V, A - fb[:, None], PRM), rtol=1e-14, atol=1e-14)
    zero = np.zeros((3, M))
    R = solid.residual(X, conn, zero, zero, np.tile(fb[:, None], (1, M)), PRM, body=fb)
    assert np.abs(R).max() <= 1e-15 * np.abs(solid.residual(X, conn, zero, zero, np.tile(fb[:, None], (1, M)), PRM)).max()
