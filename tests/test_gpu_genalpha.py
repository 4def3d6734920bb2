"""GPU parity of the time stepping (section 2.4: generalized-alpha steps, each solved
by Newton on the monolithic system): three steps of the rotating-plates channel on
an 8^3 grid through the library (stepper.ChannelRun: residual, Newton, FGMRES with
the Schur-complement preconditioner, rate updates with fsi_axpby) against the
oracle's stepping (oracle/genalpha.py with dense Newton), for backward Euler and
for generalized-alpha with rho_inf = 0.5.  Both stop every step at 1e-8 times the
residual of the same plain guess, so the states agree to about that level.
"""
import dataclasses

import numpy as np
import pytest

import fsi_workloads as W
from oracle import dlm as odlm
from oracle import genalpha as oga
from oracle import vms as ovms

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("integrator", ["be", "genalpha"])
def test_channel_steps_match_oracle(integrator):
    import torch
    from paper_2601_08266_amd.stepper import ChannelRun
    cfg = dataclasses.replace(W.CONFIGS["c4"], grid=W.Grid((8, 8, 8), 1), m_points=2000)
    g = cfg.grid
    N = g.num_nodes
    run = ChannelRun(cfg, inner=torch.float64, precond="schur_tri", integrator=integrator, rho_inf=0.5)
    coefs = run.coefs
    nsteps = 3
    for _ in range(nsteps):
        rec = run.step()
        print(f"{integrator} step {rec.n}: {rec.newton_iters} Newton / {rec.krylov_iters} Krylov", flush=True)
    x_gpu = run.x.cpu().numpy().reshape(4, N)
    xd_gpu = run.xdot.cpu().numpy().reshape(4, N)

    prm = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    mask = W.channel_dirichlet_mask(g)
    pattern = W.channel_inflow_pattern(g)
    kappa = W.kappa_weights(cfg.m_points, W.plate_volume(), cfg.c_m, cfg.alpha)
    x = np.zeros((4, N))
    xdot = np.zeros((4, N))
    dt = cfg.dt
    am, af, gm = coefs
    for n in range(nsteps):
        t_s = (n + af) * dt
        X, gp = W.rotating_plate_points(cfg.m_points, cfg.seed_fields, t_s, period=run.period,
                                        amp_deg=run.amp)
        cell, xi = odlm.locate(g, X)
        s = odlm.s_field(g, cell, cfg.s_max)
        inflow = ((1.0 - af) * W.channel_inflow_value(n * dt, run.period)
                  + af * W.channel_inflow_value((n + 1) * dt, run.period))
        x, xdot, _, info = oga.step(g, prm, coefs, dt, x, xdot, cell, xi, kappa, gp, s=s, mask=mask,
                                    gD_stage=pattern * inflow, rel=run.rel_tol)
        assert info["converged"]
    ex = np.linalg.norm(x_gpu - x) / np.linalg.norm(x)
    print(f"{integrator}: state rel diff {ex:.3e}")
    assert ex <= 1e-6
    if integrator == "genalpha":
        ed = np.linalg.norm(xd_gpu - xdot) / np.linalg.norm(xdot)
        print(f"{integrator}: rate rel diff {ed:.3e}")
        assert ed <= 1e-4
