"""Failure paths forced from the host and checkpoint/resume (every kernel still exits
normally: the conditions are NaN inputs, iteration caps and broken network weights).

* FGMRES: NaN in the right-hand side -> FSI_ERR_NAN; an iteration cap of one Arnoldi step ->
  FSI_ERR_NOT_CONVERGED with x the last iterate (its residual below ||b||); the solve without
  a caller ring takes the same iterates as with one.
* Newton: NaN in the initial guess -> FSI_ERR_NAN; a Newton cap below what the tolerance needs
  -> FSI_ERR_NOT_CONVERGED.
* Learned warm start: NaN weights give a NaN guess, which the safeguard rejects in favour of
  the extrapolation; zero weights give a zero correction, i.e. the extrapolation itself.
* A channel run checkpointed after 5 steps and resumed in a fresh stepper reaches, after 5
  more, bitwise the state of an uninterrupted 10-step run.
"""
import dataclasses

import numpy as np
import pytest

import fsi_workloads as W

from test_gpu_solve import _t, build, newton_case

pytestmark = pytest.mark.gpu


def _c1_problem():
    cfg = W.CONFIGS["c1"]
    P = build(cfg, W.advection_field(cfg.grid, cfg.seed_fields))
    g = P["g"]
    N = g.num_nodes
    b = W.smooth_fourier_field(g, cfg.seed_vectors).ravel()
    b[:3 * N][P["mask"].ravel()] = 0.0
    return cfg, P, g, N, b


def test_fgmres_nan_rhs_and_iteration_cap():
    import torch
    import paper_2601_08266_amd as fsi
    import paper_2601_08266_amd._lib as L
    cfg, P, g, N, b = _c1_problem()
    pinv64, pinv32, _, _ = fsi.bjacobi_setup(P["J64"])
    bn = b.copy()
    bn[17] = np.nan
    x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    opts = fsi.solve_opts(restart=50, max_iters=500, rtol=1e-10, inner=torch.float32)
    rc, st = fsi.fgmres_solve(P["J64"], _t(bn), x, opts, J32=P["J32"], pinv=pinv32, check=False)
    print(f"NaN rhs: rc {rc} ({L.lib().fsi_last_error().decode()})")
    assert rc == L.FSI_ERR_NAN
    # one Arnoldi step allowed: not converged, x is the iterate after that step
    x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
    opts = fsi.solve_opts(restart=50, max_iters=1, rtol=1e-10, inner=torch.float32)
    rc, st = fsi.fgmres_solve(P["J64"], _t(b), x, opts, J32=P["J32"], pinv=pinv32, check=False)
    r = _t(b) - fsi.jacobian_apply(P["J64"], x)
    rn = float(torch.linalg.norm(r))
    print(f"cap 1: rc {rc}, iters {st.iters}, residual {rn:.3e} of {st.bnorm:.3e}")
    assert rc == L.FSI_ERR_NOT_CONVERGED
    assert st.iters == 1
    assert 0.0 < rn < st.bnorm
    assert abs(rn - st.res_final) <= 1e-10 * st.bnorm
    # without the caller's pinned ring: the same iterates, bitwise
    xs = {}
    for pinned in (True, False):
        x = torch.zeros(4 * N, dtype=torch.float64, device="cuda")
        opts = fsi.solve_opts(restart=50, max_iters=3000, rtol=1e-10, inner=torch.float32, pinned=pinned)
        assert (opts.host_ring is not None) == pinned
        rc, st = fsi.fgmres_solve(P["J64"], _t(b), x, opts, J32=P["J32"], pinv=pinv32)
        xs[pinned] = (x.cpu().numpy(), st.iters)
    assert xs[True][1] == xs[False][1]
    assert np.array_equal(xs[True][0], xs[False][0])


def test_newton_nan_guess_and_newton_cap():
    import torch
    import paper_2601_08266_amd as fsi
    import paper_2601_08266_amd._lib as L
    cfg = W.CONFIGS["c1"]
    X, g_pts, kappa, u_old, mask, gD, x0 = newton_case(cfg)
    g = cfg.grid
    N = g.num_nodes
    P = build(cfg, u_old, X=X, kappa=kappa)
    lamg = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    fsi.dlm_BT(g, P["J64"].tables, _t(g_pts), lamg, kappa=_t(P["kappa"]))
    xn = x0.copy()
    xn[3, 5] = np.nan
    x = _t(xn)
    opts = fsi.newton_opts(tol_abs=1e-8, inner=torch.float32)
    rc, st = fsi.newton_solve(P["J64"], _t(cfg.c_m * u_old), x, opts, P32=P["J32"], lamg=lamg,
                              gD=_t(gD), check=False)
    print(f"NaN guess: rc {rc}")
    assert rc == L.FSI_ERR_NAN
    assert st.newton_iters == 0
    x = _t(x0)
    opts = fsi.newton_opts(tol_abs=1e-30, max_newton=1, inner=torch.float32)
    rc, st = fsi.newton_solve(P["J64"], _t(cfg.c_m * u_old), x, opts, P32=P["J32"], lamg=lamg,
                              gD=_t(gD), check=False)
    print(f"cap 1: rc {rc}, hist {list(st.res_hist[:st.newton_iters + 1])}")
    assert rc == L.FSI_ERR_NOT_CONVERGED
    assert st.newton_iters == 1
    assert st.res_hist[1] < st.res_hist[0]


def test_learned_guess_safeguard_with_broken_weights():
    import torch
    from paper_2601_08266_amd.learned import LearnedWarmStart, linear_extrapolation_guess
    from paper_2601_08266_amd.stepper import ChannelRun
    cfg = dataclasses.replace(W.CONFIGS["c4"], grid=W.Grid((8, 8, 8), 1), m_points=2000)
    run = ChannelRun(cfg, precond="schur_tri", vel_steps=2)
    run.record_extrap = True
    for _ in range(4):
        run.step()
    lw = LearnedWarmStart(run, seed=0)
    lw.fit_normalisation(run.history, [1, 2])   # statistics only; the weights are set below
    recs = {}
    for name, fill in (("nan", float("nan")), ("zero", 0.0)):
        for lay in lw.net.layers:
            lay.w32.fill_(fill)
            lay.b32.fill_(fill)
        lw.net.refresh()
        run.restore(4)
        recs[name] = run.step(guess_fn=lw.guess, record=False)
    run.restore(4)
    recs["extrap"] = run.step(guess_fn=linear_extrapolation_guess, record=False)
    for k, r in recs.items():
        print(f"{k}: used {r.used_guess}, res_guess {r.res_guess:.3e}, res_plain {r.res_plain:.3e}, "
              f"{r.newton_iters} Newton / {r.krylov_iters} Krylov")
    # NaN network: the safeguard takes the extrapolation instead
    assert recs["nan"].used_guess == "extrapolation"
    assert recs["nan"].res_guess == recs["extrap"].res_guess
    assert torch.equal(recs["nan"].x, recs["extrap"].x)
    # zero network: no correction, i.e. the extrapolation
    assert recs["zero"].res_guess == recs["extrap"].res_guess
    assert torch.equal(recs["zero"].x, recs["extrap"].x)


def test_checkpoint_resume_is_bitwise(tmp_path):
    import torch
    from paper_2601_08266_amd.stepper import ChannelRun
    from paper_2601_08266_amd.learned import linear_extrapolation_guess
    cfg = dataclasses.replace(W.CONFIGS["c4"], grid=W.Grid((8, 8, 8), 1), m_points=2000)
    for integrator in ("be", "genalpha"):
        full = ChannelRun(cfg, precond="schur_tri", integrator=integrator)
        for _ in range(10):
            full.step(guess_fn=linear_extrapolation_guess)
        first = ChannelRun(cfg, precond="schur_tri", integrator=integrator)
        for _ in range(5):
            first.step(guess_fn=linear_extrapolation_guess)
        path = tmp_path / f"ckpt_{integrator}.npz"
        first.checkpoint(path)
        del first
        second = ChannelRun(cfg, precond="schur_tri", integrator=integrator)
        second.resume(path)
        assert second.n == 5
        for _ in range(5):
            second.step(guess_fn=linear_extrapolation_guess)
        print(f"{integrator}: resumed state equal: {torch.equal(second.x, full.x)}")
        assert second.n == full.n == 10
        assert torch.equal(second.x, full.x)
        assert torch.equal(second.xdot, full.xdot)
