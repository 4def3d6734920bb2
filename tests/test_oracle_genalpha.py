"""Pins of the oracle's generalized-alpha stepping (oracle/genalpha.py; section 2.4
integrates with the second-order generalized-alpha method, in the variant that
keeps the pressure second order).

* (alpha_m, alpha_f, gamma) = (1, 1, 1) is backward Euler: the step equals the
  oracle's backward-Euler Newton step.
* Temporal order on a 4^3 channel driven by a smooth inflow (from rest, every
  rate consistent at t = 0): successive halvings of dt give error ratios of
  about 4 for the velocity and for the pressure with rho_inf = 0.5, and about 2
  with backward Euler (Richardson estimates from four step sizes).
"""
import math

import numpy as np
import pytest

import fsi_workloads as W
from oracle import genalpha, newton, vms


def _channel(n=4, nu=0.1, dt_tau=1e-2):
    g = W.Grid((n, n, n), 1)
    N = g.num_nodes
    prm = vms.params_array(nu, 1.0 / dt_tau, dt_tau)
    mask = W.channel_dirichlet_mask(g)
    nx, ny, nz = g.nodes_per_axis
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inflow = ((i == 0) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    pattern = np.zeros((3, N))
    pattern[0][inflow] = 1.0
    empty = (np.zeros(0, dtype=np.int64), np.zeros((3, 0)), np.zeros(0), np.zeros((3, 0)))
    return g, N, prm, mask, pattern, empty


def _inflow(t, T=0.2):
    return math.sin(math.pi * t / T) ** 4


def _run(coefs, nsteps, t_end=0.1):
    g, N, prm, mask, pattern, (cell, xi, kappa, gpts) = _channel()
    dt = t_end / nsteps
    x = np.zeros((4, N))
    xdot = np.zeros((4, N))
    for n in range(nsteps):
        af = coefs[1]
        gD_stage = pattern * ((1.0 - af) * _inflow(n * dt) + af * _inflow((n + 1) * dt))
        x, xdot, _, info = genalpha.step(g, prm, coefs, dt, x, xdot, cell, xi, kappa, gpts, mask=mask,
                                         gD_stage=gD_stage, rel=1e-13)
        assert info["converged"]
    return x


def test_unit_coefficients_are_backward_euler():
    g, N, prm, mask, pattern, (cell, xi, kappa, gpts) = _channel()
    rng = np.random.default_rng(3)
    dt = 0.01
    x_n = 0.1 * rng.standard_normal((4, N))
    x_n[:3][mask] = (pattern * _inflow(0.05))[mask]
    gD = pattern * _inflow(0.06)
    x1, xdot1, xs, info = genalpha.step(g, prm, (1.0, 1.0, 1.0), dt, x_n, np.zeros((4, N)), cell, xi,
                                        kappa, gpts, mask=mask, gD_stage=gD, rel=1e-13)
    p_be = prm.copy()
    p_be[1] = 1.0 / dt
    x0 = x_n.copy()
    x0[:3][mask] = gD[mask]
    xb, _ = newton.solve_step(g, p_be, x0, x_n[:3], cell, xi, kappa, gpts, mask=mask, gD=gD, rel=1e-13)
    assert np.abs(x1 - xb).max() <= 1e-12 * np.abs(xb).max()
    np.testing.assert_allclose(xdot1, (x1 - x_n) / dt, rtol=1e-10, atol=1e-10 * np.abs(xdot1).max())


def _orders(coefs):
    xs = [_run(coefs, m) for m in (10, 20, 40, 80)]
    out = {}
    for f, name in ((slice(0, 3), "velocity"), (slice(3, 4), "pressure")):
        d = [np.linalg.norm(xs[i][f] - xs[i + 1][f]) for i in range(3)]
        out[name] = [math.log2(d[i] / d[i + 1]) for i in range(2)]
    return out


def test_generalized_alpha_is_second_order_in_velocity_and_pressure():
    o = _orders(genalpha.coefficients(0.5))
    print("generalized-alpha orders", o)
    for name in ("velocity", "pressure"):
        assert o[name][-1] >= 1.8, (name, o)


def test_backward_euler_is_first_order_on_the_same_problem():
    o = _orders((1.0, 1.0, 1.0))
    print("backward Euler orders", o)
    assert 0.8 <= o["velocity"][-1] <= 1.3, o
