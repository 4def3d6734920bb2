"""Hyperelastic solid block of the reduced system (test infrastructure only).

Section 2.4's momentum-momentum block is dR^{f,m}/dV + C^lambda dR^s/dU (C^lambda)^T.
This module replaces the per-point stand-in kappa_B I of ``jacobian`` with the solid's
own tangent, from the solid weak form of section 2.2 (eq. solid_weak_form) and the
nearly-incompressible neo-Hookean energy of section 4.3 (eq. inc_neoHk):

    psi(F) = C0/2 (tr Cbar - 3) + kappa_s/2 ((J^2 - 1)/2 - ln J),
    Cbar = Fbar^T Fbar,  Fbar = J^{-1/3} F,  J = det F.

The solid is discretised by trilinear hexahedra on the reference configuration (2x2x2
Gauss points on [0,1]^3); its nodes are the multiplier points (section 2.3: delta
functions at the solid nodes), so C^lambda couples them to the fluid through the same
B / B^T as the point stand-in.  Readings (where the paper is silent or garbled):

* the isochoric split is Fbar = J^{-1/3} F (the printed exponent +1/3 would not give
  det Fbar = 1);
* the inertia term of eq. solid_weak_form uses rho^s dOmega_t = rho^s_0 dOmega_0 (mass
  conservation) and rho^f dOmega_t = rho^f J dOmega_0, so its mass matrix is
  int (rho^s_0 - rho^f J) N_A N_B dOmega_0;
* the subtracted viscous work -int 2 mu^f eps(w):eps(v) is taken with the solid
  velocity interpolant (the velocities agree at the solid nodes by eq.
  nodal_solid_velo) on the current configuration (grad_x N = F^{-T} grad_X N,
  dOmega_t = J dOmega_0);
* within one linear solve the configuration is frozen for the mass and viscous terms
  (their geometric derivatives are dropped, as the Picard linearisation of the fluid
  does); the stress term enters with its full material tangent dP/dF.

In velocity form (the unknowns of the linear solves here), the block applied to the
solid-node velocities is

    K_s = c_M M + c_K K(U) - c_V K_v(U)

with c_M, c_K, c_V the time integrator's derivatives of (acceleration, displacement,
velocity) with respect to the new velocity (backward Euler: 1/dt, dt, 1).
"""
from __future__ import annotations

import numpy as np

# 2-point Gauss-Legendre on [0, 1]: points and the equal weight 1/8 per 3D point
_G = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
GAUSS = np.array([[_G[i & 1], _G[(i >> 1) & 1], _G[i >> 2]] for i in range(8)])
GAUSS_W = 0.125


def shape(xi):
    """Trilinear shape functions on [0,1]^3 and their xi-derivatives at one point.

    Corner c = a + 2b + 4c' sits at (a, b, c').  Returns (N [8], dN [8][3]).
    """
    N = np.empty(8)
    dN = np.empty((8, 3))
    for c in range(8):
        o = (c & 1, (c >> 1) & 1, c >> 2)
        f = [xi[d] if o[d] else 1.0 - xi[d] for d in range(3)]
        df = [1.0 if o[d] else -1.0 for d in range(3)]
        N[c] = f[0] * f[1] * f[2]
        dN[c] = (df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2])
    return N, dN


# ---- constitutive law (eq. inc_neoHk) ----

def energy(F, C0, kap):
    """psi(F) of eq. inc_neoHk with Fbar = J^{-1/3} F."""
    J = np.linalg.det(F)
    I1bar = J ** (-2.0 / 3.0) * np.sum(F * F)
    return 0.5 * C0 * (I1bar - 3.0) + 0.5 * kap * (0.5 * (J * J - 1.0) - np.log(J))


def piola(F, C0, kap):
    """First Piola-Kirchhoff stress P = dpsi/dF:
    C0 J^{-2/3} (F - I1/3 F^{-T}) + kap/2 (J^2 - 1) F^{-T}."""
    J = np.linalg.det(F)
    Fit = np.linalg.inv(F).T
    I1 = np.sum(F * F)
    return C0 * J ** (-2.0 / 3.0) * (F - I1 / 3.0 * Fit) + 0.5 * kap * (J * J - 1.0) * Fit


def piola_tangent(F, dF, C0, kap):
    """dP = (dP/dF) : dF, differentiating piola() term by term:
    d(J^{-2/3}) = -2/3 J^{-2/3} (F^{-T}:dF),  d(I1) = 2 F:dF,
    d(F^{-T}) = -F^{-T} dF^T F^{-T},  d(J^2) = 2 J^2 (F^{-T}:dF)."""
    J = np.linalg.det(F)
    Fit = np.linalg.inv(F).T
    I1 = np.sum(F * F)
    tr = np.sum(Fit * dF)
    a = J ** (-2.0 / 3.0)
    dFit = -Fit @ dF.T @ Fit
    d_iso = C0 * a * (-2.0 / 3.0 * tr * (F - I1 / 3.0 * Fit) + dF - 2.0 / 3.0 * np.sum(F * dF) * Fit
                      - I1 / 3.0 * dFit)
    d_vol = kap * J * J * tr * Fit + 0.5 * kap * (J * J - 1.0) * dFit
    return d_iso + d_vol


def elasticity_tensor(F, C0, kap):
    """A[i,K,j,L] = dP_iK / dF_jL, column by column from piola_tangent."""
    A = np.empty((3, 3, 3, 3))
    for j in range(3):
        for L in range(3):
            E = np.zeros((3, 3))
            E[j, L] = 1.0
            A[:, :, j, L] = piola_tangent(F, E, C0, kap)
    return A


# ---- one element ----

def _kinematics(Xe, Ue, q):
    """Gauss point q: shape values, reference gradients G [8][3], det of dX/dxi, F."""
    N, dN = shape(GAUSS[q])
    J0 = Xe.T @ dN                       # J0[i][k] = dX_i / dxi_k
    det0 = np.linalg.det(J0)
    G = dN @ np.linalg.inv(J0)           # G[A][K] = dN_A / dX_K
    F = np.eye(3) + Ue.T @ G             # F[i][K] = delta_iK + dU_i / dX_K
    return N, G, det0, F


def element_energy(Xe, Ue, prm):
    """Stored energy sum_q w det0 psi(F_q) of one element (Xe, Ue: [8][3])."""
    return sum(GAUSS_W * d * energy(F, prm["C0"], prm["kappa_s"])
               for _, _, d, F in (_kinematics(Xe, Ue, q) for q in range(8)))


def element_force(Xe, Ue, prm):
    """Internal force f[A][i] = sum_q w det0 P(F_q)_iK G_AK (the weak form's grad w : sigma
    term, pulled back to the reference configuration)."""
    f = np.zeros((8, 3))
    for q in range(8):
        _, G, d, F = _kinematics(Xe, Ue, q)
        f += GAUSS_W * d * G @ piola(F, prm["C0"], prm["kappa_s"]).T
    return f


def element_matrices(Xe, Ue, prm):
    """(M, K, Kv), each [24][24] with DOF 3A + i: the mass matrix with density
    rho_s0 - rho_f J, the material tangent of the stress term and the viscous matrix
    2 mu_f int eps(N_A e_i) : eps(N_B e_j) dOmega_t."""
    M = np.zeros((24, 24))
    K = np.zeros((24, 24))
    Kv = np.zeros((24, 24))
    for q in range(8):
        N, G, d, F = _kinematics(Xe, Ue, q)
        J = np.linalg.det(F)
        w = GAUSS_W * d
        rho = prm["rho_s0"] - prm["rho_f"] * J
        A = elasticity_tensor(F, prm["C0"], prm["kappa_s"])
        g = G @ np.linalg.inv(F)            # g[A][k] = dN_A / dx_k (current configuration)
        I3 = np.eye(3)
        # blocks [a][i][b][j] for every node pair (a, b)
        M += (w * rho * np.einsum("a,b,ij->aibj", N, N, I3)).reshape(24, 24)
        K += (w * np.einsum("aK,iKjL,bL->aibj", G, A, G)).reshape(24, 24)
        Kv += (w * J * prm["mu_f"] * (np.einsum("ak,bk,ij->aibj", g, g, I3)
                                      + np.einsum("bi,aj->aibj", g, g))).reshape(24, 24)
    return M, K, Kv


def element_block(Xe, Ue, prm, cM, cK, cV):
    M, K, Kv = element_matrices(Xe, Ue, prm)
    return cM * M + cK * K - cV * Kv


# ---- whole mesh ----

def apply(X0, conn, U, v, prm, cM, cK, cV):
    """y = K_s v at the solid nodes ([3][M] in and out): sum over elements of the dense
    element block applied to the element's nodal values."""
    X0 = np.asarray(X0, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    y = np.zeros_like(v)
    for e in range(conn.shape[0]):
        nodes = conn[e]
        Ke = element_block(X0[:, nodes].T, U[:, nodes].T, prm, cM, cK, cV)
        ye = Ke @ v[:, nodes].T.reshape(24)
        np.add.at(y.T, nodes, ye.reshape(8, 3))
    return y


def apply_rows(X0, conn, U, v, prm, cM, cK, cV, nodes):
    """Rows of K_s v at the listed solid nodes only ([3][len(nodes)]): the elements that
    touch each node, summed."""
    nodes = np.asarray(nodes)
    touch = {}
    for e in range(conn.shape[0]):
        for c, n in enumerate(conn[e]):
            touch.setdefault(int(n), []).append((e, c))
    out = np.zeros((3, nodes.size))
    X0 = np.asarray(X0, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    blocks = {}     # each element's block computed once
    for k, n in enumerate(nodes):
        for e, c in touch.get(int(n), []):
            el = conn[e]
            if e not in blocks:
                blocks[e] = element_block(X0[:, el].T, U[:, el].T, prm, cM, cK, cV)
            out[:, k] += blocks[e][3 * c:3 * c + 3] @ v[:, el].T.reshape(24)
    return out


def jacobian_apply(grid, prm_f, a, x, cell, xi, X0, conn, U, prm_s, cM, cK, cV, s=None, mask=None,
                   visc_strong=True):
    """J x of section 2.4's reduced system with the solid tangent:
    J = A_VMS + [[C^lambda K_s (C^lambda)^T, 0], [0, 0]], C^lambda = B^T over the solid nodes
    (located by (cell, xi)); Dirichlet velocity DOFs have zero columns and identity rows."""
    from . import dlm, vms
    N = grid.num_nodes
    x = np.asarray(x, dtype=np.float64).reshape(4, N)
    xm = x.copy()
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        xm[:3][m] = 0.0
    y = vms.apply(grid, prm_f, a, xm, s=s, mask=None, visc_strong=visc_strong)
    us = dlm.apply_B(grid, cell, xi, xm[:3])
    y[:3] += dlm.apply_BT(grid, cell, xi, apply(X0, conn, U, us, prm_s, cM, cK, cV))
    if mask is not None:
        y[:3][m] = x[:3][m]
    return y


def dense(X0, conn, U, prm, cM, cK, cV):
    """K_s assembled densely ([3M][3M], DOF i*M + node, matching [3][M] vectors); small meshes."""
    M = X0.shape[1]
    K = np.zeros((3 * M, 3 * M))
    for e in range(conn.shape[0]):
        nodes = conn[e]
        Ke = element_block(X0[:, nodes].T, U[:, nodes].T, prm, cM, cK, cV)
        idx = np.array([[i * M + n for i in range(3)] for n in nodes]).reshape(24)  # 3A + i -> i*M + node
        K[np.ix_(idx, idx)] += Ke
    return K


def jacobian_dense(grid, prm_f, a, cell, xi, X0, conn, U, prm_s, cM, cK, cV, s=None, mask=None,
                   visc_strong=True):
    """Dense J = A_VMS + [[B^T K_s B, 0], [0, 0]] with Dirichlet rows/columns (small cases)."""
    from . import dlm, vms
    N = grid.num_nodes
    M = X0.shape[1]
    A = vms.assemble_dense(grid, prm_f, a, s=s, visc_strong=visc_strong)
    Bs = dlm.dense_B(grid, cell, xi)
    Ks = dense(X0, conn, U, prm_s, cM, cK, cV)
    for i in range(3):
        for j in range(3):
            A[i * N:(i + 1) * N, j * N:(j + 1) * N] += Bs.T @ Ks[i * M:(i + 1) * M, j * M:(j + 1) * M] @ Bs
    if mask is not None:
        m = np.concatenate([np.asarray(mask, dtype=bool).reshape(-1), np.zeros(N, dtype=bool)])
        A[:, m] = 0.0
        A[m, :] = 0.0
        A[m, m] = 1.0
    return A


# ---- the solid's nonlinear residual and one coupled time step ----
#
# Solid residual at the nodes (eq. solid_weak_form tested with each nodal shape function; no
# body force or traction on the solid), with the readings above:
#   R^s(U, V, A) = M_rho(U) A + f_int(U) - K_v(U) V.
# The solid velocity is the fluid's at the solid nodes (eq. nodal_solid_velo): V = B u, and the
# displacement and acceleration are affine in it, U = U_base + c_U V, A = c_A V - A_base:
# backward Euler in velocity form has U_base = U_n, c_U = dt, A_base = V_n / dt, c_A = 1 / dt;
# generalized-alpha in stage unknowns (the solid displacement advancing through its rate V with
# the fluid's gamma) has c_U = gamma dt, U_base = U_n + (alpha_f - gamma) dt V_n,
# c_A = alpha_m / (gamma dt alpha_f), A_base = c_A V_n - (1 - alpha_m / gamma) Vdot_n.  The fluid
# momentum residual gains C^lambda R^s = B^T R^s (the multiplier eliminated by eq.
# nodal_lagrange, lambda = -R^s), and the solid moves with the fluid (Delta U = (C^lambda)^T
# Delta V integrated).  Its derivative with respect to u is B^T (c_M M + c_K K - c_V K_v) B with
# (c_A, c_U, 1) up to the geometric derivatives of M_rho and K_v, which the Newton matrix drops.


def residual(X0, conn, U, V, A, prm, body=None):
    """R^s(U, V, A) at the solid nodes ([3][M] arrays); body: an optional body force per unit mass
    f ([3] or [3][M]) of the inertia term (rho_s - rho_f)(A - f)."""
    X0 = np.asarray(X0, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    if body is not None:
        A = A - np.broadcast_to(np.asarray(body, dtype=np.float64).reshape(3, -1), A.shape)
    R = np.zeros_like(U)
    for e in range(conn.shape[0]):
        nodes = conn[e]
        Xe, Ue = X0[:, nodes].T, U[:, nodes].T
        M, _, Kv = element_matrices(Xe, Ue, prm)
        re = M @ A[:, nodes].T.reshape(24) - Kv @ V[:, nodes].T.reshape(24) + element_force(Xe, Ue, prm).reshape(24)
        np.add.at(R.T, nodes, re.reshape(8, 3))
    return R


def be_state(U_n, V_n, dt):
    """(U_base, A_base, c_U, c_A) of a backward-Euler step."""
    return U_n, V_n / dt, dt, 1.0 / dt


def step_state(grid, cell, xi, x, Ub, Ab, cU, cA):
    """(V, U, A) of the solid for the fluid state x: V = B u, U = Ub + cU V, A = cA V - Ab."""
    from . import dlm
    N = grid.num_nodes
    V = dlm.apply_B(grid, cell, xi, np.asarray(x, dtype=np.float64).reshape(4, N)[:3])
    return V, Ub + cU * V, cA * V - Ab


def step_residual(grid, prm_f, x, f, cell, xi, X0, conn, state, prm_s, s=None, mask=None, gD=None,
                  visc_strong=True, body=None):
    """R(x) = R_fluid(x; f) + [B^T R^s(Ub + cU B u, B u, cA B u - Ab); 0], Dirichlet rows u - gD
    (state = (Ub, Ab, cU, cA); R_fluid: the VMS step residual with nodal source f)."""
    from . import dlm, vms
    N = grid.num_nodes
    x = np.asarray(x, dtype=np.float64).reshape(4, N)
    R = vms.residual_fluid(grid, prm_f, x, np.asarray(f, dtype=np.float64).reshape(3, N), s=s,
                           visc_strong=visc_strong)
    V, U, A = step_state(grid, cell, xi, x, *state)
    R[:3] += dlm.apply_BT(grid, cell, xi, residual(X0, conn, U, V, A, prm_s, body=body))
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        gd = np.zeros((3, N)) if gD is None else np.asarray(gD).reshape(3, N)
        R[:3][m] = x[:3][m] - gd[m]
    return R


def newton_step(grid, prm_f, x0, f, cell, xi, X0, conn, state, prm_s, s=None, mask=None, gD=None,
                tol_abs=None, rel=1e-8, max_newton=30, visc_strong=True, body=None):
    """Newton on step_residual from x0 with the matrix A(a = u_k) + B^T K_s(U_k) B, K_s with
    (c_A, c_U, 1) (dense solves); returns (x, U, V, info) at the converged x."""
    N = grid.num_nodes
    Ub, Ab, cU, cA = state
    x = np.asarray(x0, dtype=np.float64).reshape(4, N).copy()
    R = step_residual(grid, prm_f, x, f, cell, xi, X0, conn, state, prm_s, s, mask, gD, visc_strong, body)
    hist = [np.linalg.norm(R)]
    if tol_abs is None:
        tol_abs = rel * hist[0]
    for _ in range(max_newton):
        if hist[-1] <= tol_abs:
            break
        _, U, _ = step_state(grid, cell, xi, x, *state)
        J = jacobian_dense(grid, prm_f, x[:3].copy(), cell, xi, X0, conn, U, prm_s, cA, cU, 1.0, s=s,
                           mask=mask, visc_strong=visc_strong)
        x = x + np.linalg.solve(J, -R.ravel()).reshape(4, N)
        R = step_residual(grid, prm_f, x, f, cell, xi, X0, conn, state, prm_s, s, mask, gD, visc_strong, body)
        hist.append(np.linalg.norm(R))
    V, U, _ = step_state(grid, cell, xi, x, *state)
    return x, U, V, {"history": hist, "tol_abs": tol_abs, "converged": hist[-1] <= tol_abs}


def genalpha_step(grid, prm_stage, coefs, dt, x_n, xdot_n, Vs_n, Vsdot_n, U_n, cell, xi, X0, conn, prm_s,
                  s=None, mask=None, gD_stage=None, tol_abs=None, rel=1e-8, body=None):
    """One generalized-alpha step of the coupled system in stage unknowns (the fluid as in
    oracle.genalpha: mass coefficient c = alpha_m / (gamma dt alpha_f) in prm_stage, source
    c V_n - (1 - alpha_m/gamma) Vdot_n; the solid velocity Vs = B u, its rate Vsdot and its
    displacement U advancing through Vs with the same gamma).  Returns the new fluid state and
    rates, the new solid velocity, rate and displacement, the stage state and Newton's info."""
    am, af, gm = coefs
    c = am / (gm * dt * af)
    N = grid.num_nodes
    x_n = np.asarray(x_n, dtype=np.float64).reshape(4, N)
    xdot_n = np.asarray(xdot_n, dtype=np.float64).reshape(4, N)
    f = c * x_n[:3] - (1.0 - am / gm) * xdot_n[:3]
    state = (U_n + (af - gm) * dt * Vs_n, c * Vs_n - (1.0 - am / gm) * Vsdot_n, gm * dt, c)
    x0 = x_n.copy()
    if mask is not None:
        m = np.asarray(mask, dtype=bool).reshape(3, N)
        x0[:3][m] = np.asarray(gD_stage).reshape(3, N)[m]
    x_st, _, Vs_st, info = newton_step(grid, prm_stage, x0, f, cell, xi, X0, conn, state, prm_s, s=s, mask=mask,
                                       gD=gD_stage, tol_abs=tol_abs, rel=rel, body=body)
    x1 = x_n + (x_st - x_n) / af
    xdot1 = xdot_n + (x1 - x_n - dt * xdot_n) / (gm * dt)
    Vs1 = Vs_n + (Vs_st - Vs_n) / af
    Vsdot1 = Vsdot_n + (Vs1 - Vs_n - dt * Vsdot_n) / (gm * dt)
    U1 = U_n + dt * Vs_n + gm * dt * (Vs1 - Vs_n)
    return x1, xdot1, Vs1, Vsdot1, U1, x_st, info
