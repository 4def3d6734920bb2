"""Measurement drivers for the Newton-step workloads (orchestration only).

warmstart: a channel run (64^3 Q1 with three rotating plates and 200k points,
  or 192^3 with 2M points) stepped with the plain guess (mixed-precision Newton);
  the network is trained on samples from the first steps (1-100 of 200 at 64^3,
  1-20 of 40 at 192^3) and evaluated on the rest, where every step is re-solved
  from the recorded state: plain guess with FP64 inner Krylov applies, plain
  guess with FP32 inner applies, extrapolated and learned guesses with FP32
  inner applies.  All stop at the same absolute residual.
large_c5: 192^3 Q1 channel, 2M points: after warm-up steps, one Newton step
  plain FP64 vs mixed precision + learned warm start (a 64^3-trained network
  applied fully convolutionally to the finer lattice).
"""
from __future__ import annotations

import json
import math
import re
import statistics
import sys
import time

import torch

import fsi_workloads as W

from . import axpby, norm2
from .learned import LearnedWarmStart, linear_extrapolation_guess, quadratic_extrapolation_guess
from .stepper import ChannelRun


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def mode_precond(mode):
    """(preconditioner, velocity steps, tangent) named by a mode's suffixes: _st / _sd the Schur
    block-triangular / block-diagonal form, followed by an optional number of minimal-residual
    steps on the velocity block (_st2), then an optional _ft for the full Newton tangent;
    None: the run's defaults."""
    tangent = None
    if mode.endswith("_ft"):
        mode, tangent = mode[:-3], "full"
    m = re.search(r"_(st|sd)(\d*)$", mode)
    if m is None:
        return None, None, tangent
    return ("schur_tri" if m.group(1) == "st" else "schur_diag"), int(m.group(2) or 0), tangent


def _solve_modes(run, lw, k, modes):
    out = {}
    sols = {}
    for mode in modes:
        run.restore(k)
        inner = torch.float64 if "f64" in mode else torch.float32
        gf = None
        if lw is not None and mode.startswith("nn"):
            gf = lw.guess
        elif mode.startswith("extrap3"):
            gf = quadratic_extrapolation_guess
        elif mode.startswith("extrap"):
            gf = linear_extrapolation_guess
        pc, vs, tg = mode_precond(mode)
        rec = run.step(guess_fn=gf, inner=inner, record=False, precond=pc, vel_steps=vs, tangent=tg)
        out[mode] = dict(newton=rec.newton_iters, krylov=rec.krylov_iters, ms_newton=rec.ms_newton,
                         ms_guess=rec.ms_guess, res_plain=rec.res_plain, res_guess=rec.res_guess,
                         used_guess=rec.used_guess, hist=rec.res_hist, phases_ms=rec.phases_ms)
        sols[mode] = rec.x
    ref = sols[modes[0]]
    nref = norm2(ref)
    for mode in modes[1:]:
        d = sols[mode].clone()
        axpby(-1.0, ref, 1.0, d)
        out[mode]["rel_diff_vs_" + modes[0]] = norm2(d) / nref
    return out


WARMSTART_WORKLOADS = {
    "c4": "64^3 Q1 channel, 200k points on three rotating plates, dt=1e-3",
    "c5": "192^3 Q1 channel, 2M points on three rotating plates, dt=1e-3",
}


def warmstart(cfg_key="c4", steps=200, train_end=100, epochs=20, lr=1e-3, eval_stride=1, seed=0,
              save_path=None, precond="bjacobi", integrator="be", rho_inf=0.5, vel_steps=0):
    cfg = W.CONFIGS[cfg_key]
    run = ChannelRun(cfg, precond=precond, integrator=integrator, rho_inf=rho_inf, vel_steps=vel_steps)
    run.record_extrap = True
    t0 = time.perf_counter()
    for n in range(steps):
        rec = run.step()
        if (n + 1) % 10 == 0 or n < 3:
            _log(f"{cfg_key} step {rec.n}: t={rec.t:.3f} inflow={rec.inflow:+.3f} newton={rec.newton_iters} "
                 f"krylov={rec.krylov_iters} {rec.ms_newton:.1f} ms")
    sim_s = time.perf_counter() - t0
    lw = LearnedWarmStart(run, seed=seed)
    ks = list(range(1, train_end))
    lw.fit_normalisation(run.history, ks)
    lw.build_dataset(run.history, ks)
    _log(f"training on {len(ks)} samples, {lw.net.n_params} parameters")
    lw.train(epochs=epochs, lr=lr, seed=seed, log=_log)
    if save_path:
        sd = lw.net.state_dict()
        sd["norm"] = dict(in_shift=[float(v) for v in lw.in_shift],
                          in_scale=[float(v) for v in lw.in_scale],
                          out_shift=[float(v) for v in lw.out_shift],
                          out_scale=[float(v) for v in lw.out_scale])
        torch.save(sd, save_path)
    modes = ["plain_f64", "plain_mixed", "extrap_mixed", "extrap3_mixed", "nn_mixed"]
    rows = []
    for k in range(train_end, steps, eval_stride):
        r = _solve_modes(run, lw, k, modes)
        rows.append(r)
        if len(rows) % 10 == 1:
            _log(f"eval step {k + 1}: " + ", ".join(
                f"{m} {r[m]['newton']}N/{r[m]['krylov']}K {r[m]['ms_newton'] + r[m]['ms_guess']:.1f}ms"
                for m in modes))

    def agg(mode, key):
        return statistics.mean(r[mode][key] for r in rows)

    summary = {
        "workload": WARMSTART_WORKLOADS[cfg_key],
        "precond": precond, "vel_steps": vel_steps, "integrator": integrator,
        "steps": steps, "train_steps": [2, train_end], "eval_steps": [train_end + 1, steps],
        "epochs": epochs, "params": lw.net.n_params, "train_ms": round(lw.train_ms, 1),
        "final_train_loss": lw.losses[-1] if lw.losses else None,
        "simulate_s": round(sim_s, 1),
    }
    for m in modes:
        summary[m] = {
            "ms_per_step": round(agg(m, "ms_newton") + agg(m, "ms_guess"), 2),
            "ms_newton": round(agg(m, "ms_newton"), 2),
            "ms_guess": round(agg(m, "ms_guess"), 2),
            "newton_iters": round(agg(m, "newton"), 3),
            "krylov_iters": round(agg(m, "krylov"), 1),
        }
    for m in ("extrap_mixed", "extrap3_mixed", "nn_mixed"):
        summary[m]["guess_used_frac"] = statistics.mean(1.0 if r[m]["used_guess"] is True else 0.0 for r in rows)
        summary[m]["extrapolation_fallback_frac"] = statistics.mean(
            1.0 if r[m]["used_guess"] == "extrapolation" else 0.0 for r in rows)
        summary[m]["res_ratio_median"] = statistics.median(r[m]["res_guess"] / r[m]["res_plain"] for r in rows)
    for m in modes[1:]:
        summary[m]["max_rel_diff_vs_plain_f64"] = max(r[m]["rel_diff_vs_plain_f64"] for r in rows)
    summary["newton_hist_example"] = {m: ["%.2e" % h for h in rows[len(rows) // 2][m]["hist"]] for m in modes}
    summary["speedup_nn_mixed_vs_plain_f64"] = round(summary["plain_f64"]["ms_per_step"] / summary["nn_mixed"]["ms_per_step"], 3)
    summary["speedup_plain_mixed_vs_plain_f64"] = round(summary["plain_f64"]["ms_per_step"] / summary["plain_mixed"]["ms_per_step"], 3)
    return summary, lw


def large_c5(lw_c4=None, warmup_steps=3, state_path=None, modes=None, warmup_precond="schur_tri",
             integrator="be", rho_inf=0.5):
    cfg = W.CONFIGS["c5"]
    run = ChannelRun(cfg, integrator=integrator, rho_inf=rho_inf)
    for n in range(warmup_steps):
        rec = run.step(precond=warmup_precond)
        _log(f"c5 warm-up step {rec.n}: newton={rec.newton_iters} krylov={rec.krylov_iters} "
             f"{rec.ms_newton:.0f} ms")
    lw = None
    if lw_c4 is not None or state_path is not None:
        lw = LearnedWarmStart(run)
        sd = torch.load(state_path, weights_only=True) if state_path else None
        if sd is None:
            sd = lw_c4.net.state_dict()
            sd["norm"] = dict(in_shift=lw_c4.in_shift, in_scale=lw_c4.in_scale,
                              out_shift=lw_c4.out_shift, out_scale=lw_c4.out_scale)
        lw.net.load_state_dict(sd)
        nm = sd["norm"]
        lw.in_shift, lw.in_scale = list(nm["in_shift"]), list(nm["in_scale"])
        lw.out_shift, lw.out_scale = list(nm["out_shift"]), list(nm["out_scale"])
    k = run.n
    if modes is None:
        modes = ["plain_f64", "plain_mixed", "extrap_mixed", "extrap3_mixed"] + (["nn_mixed"] if lw is not None else [])
    modes = list(modes)
    r = _solve_modes(run, lw, k, modes)
    for m in modes:
        _log(f"c5 step {k + 1} {m}: {r[m]['newton']}N/{r[m]['krylov']}K "
             f"{r[m]['ms_newton'] + r[m]['ms_guess']:.0f} ms")
    summary = {"workload": "192^3 Q1 channel, 2M points on three rotating plates",
               "step": k + 1, "dof": 4 * run.N, "warmup_precond": warmup_precond, "integrator": integrator,
               "modes": r}
    if "plain_f64" in r:
        base = r["plain_f64"]["ms_newton"] + r["plain_f64"]["ms_guess"]
        for m in modes[1:]:
            summary["speedup_" + m + "_vs_plain_f64"] = round(base / (r[m]["ms_newton"] + r[m]["ms_guess"]), 3)
    return summary


def solve_c3(rtol=1e-10, restart=50, max_iters=6000, profile=True, chunk=1000, modes=("mixed", "f64"),
             precond="bjacobi", vel_steps=0):
    """96^3 Q2-Q2 channel (28.8M DOF), 500k plate points, seeded smooth right-hand side zeroed
    on the Dirichlet rows: FGMRES(50) with nodal block-Jacobi to rtol, FP32 inner applies
    (FP64 residual, orthogonalisation and restarts) and, for comparison, FP64 inner applies.
    The final residual of each solve is recomputed with a separate FP64 Jacobian apply."""
    import numpy as np

    from . import (Problem, bjacobi_setup, dlm_gram, dlm_locate, fgmres_solve, jacobian_apply,
                   make_params, profile_enable, profile_read, schur_setup, solve_opts)

    cfg = W.CONFIGS["c3"]
    g = cfg.grid
    N = g.num_nodes
    dev = torch.device("cuda")

    def t(v, dt=torch.float64):
        return torch.tensor(np.ascontiguousarray(v).ravel(), dtype=dt, device=dev)

    X = W.plate_points(cfg.m_points, cfg.seed_fields)
    kap = W.kappa_weights(X.shape[1], W.plate_volume(), cfg.c_m, cfg.alpha)
    a = W.advection_field(g, cfg.seed_fields)
    mask = W.channel_dirichlet_mask(g)
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device=dev)
    b = W.smooth_fourier_field(g, cfg.seed_vectors)
    b[:3][mask] = 0.0
    prm = make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    Xt = t(X)
    out = {"workload": f"96^3 Q2-Q2 channel, {cfg.m_points} plate points", "dof": 4 * N,
           "cells": g.num_cells, "rtol": rtol, "restart": restart, "precond": precond, "vel_steps": vel_steps}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tab64 = dlm_locate(g, Xt, dtype=torch.float64, s_max=cfg.s_max)
    tab32 = dlm_locate(g, Xt, dtype=torch.float32, s_max=cfg.s_max)
    k64, k32 = t(kap), t(kap, torch.float32)
    P64 = Problem(g, prm, t(a), tab64, k64, s=tab64.s, mask=mt, gram=dlm_gram(g, tab64, k64))
    P32 = Problem(g, prm, t(a, torch.float32), tab32, k32, s=tab32.s, mask=mt,
                  gram=dlm_gram(g, tab32, k32))
    if precond == "bjacobi":
        pinv64, pinv32, _, nsing = bjacobi_setup(P64)
    else:
        _, _, blocks, nsing = bjacobi_setup(P64, want32=False, want_blocks=True)
        pinv64 = pinv32 = schur_setup(P64, blocks)
        del blocks
    torch.cuda.synchronize()
    out["setup_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    out["n_occupied_cells"] = tab64.n_occ
    out["bjacobi_singular_blocks"] = nsing
    bt = t(b)
    bnorm = norm2(bt)
    y = torch.empty_like(bt)
    # mixed_b32: FP32 inner solves that also keep the Krylov basis in FP32
    sols = {}
    for inner, pinv, name in ((torch.float32, pinv32, "mixed"), (torch.float32, pinv32, "mixed_b32"),
                              (torch.float64, pinv64, "f64")):
        if name not in modes:
            continue
        x = torch.zeros(4 * N, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # chunks of `chunk` iterations (each call restarts from the current x, as a restart
        # of the cycle would), to log the convergence history; target stays rtol ||b||
        hist = []
        iters = cycles = 0
        rc = -4
        while iters < max_iters:
            opts = solve_opts(restart=restart, max_iters=min(chunk, max_iters - iters), rtol=rtol,
                              inner=inner, precond=precond, vel_steps=vel_steps,
                              basis=torch.float32 if name == "mixed_b32" else torch.float64)
            rc, st = fgmres_solve(P64, bt, x, opts, J32=P32 if inner == torch.float32 else None,
                                  pinv=pinv, check=False)
            iters += st.iters
            cycles += st.cycles
            hist.append((iters, round((time.perf_counter() - t0) * 1e3, 1), st.res_final / bnorm))
            _log(f"c3 {name}: {iters} iterations, residual {st.res_final / bnorm:.3e}")
            if rc == 0 or rc not in (-4,):
                break
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        jacobian_apply(P64, x, y)
        r = bt.clone()
        axpby(-1.0, y, 1.0, r)
        res = norm2(r) / bnorm
        row = {"status": rc, "iters": iters, "cycles": cycles, "ms": round(ms, 1),
               "solver_rel_residual": st.res_final / bnorm, "recomputed_rel_residual": res,
               "ms_per_iter": round(ms / max(iters, 1), 3), "history": hist}
        _log(f"c3 {name}: rc {rc} iters {iters} cycles {cycles} {ms:.0f} ms residual {res:.3e}")
        out[name] = row
        sols[name] = x.clone()
    # the mixed-precision solutions against the FP64 one (or the FP32-basis one against the FP64-basis one)
    ref_name = "f64" if "f64" in sols else ("mixed" if "mixed_b32" in sols else None)
    for name in ("mixed", "mixed_b32"):
        if ref_name is not None and name in sols and name != ref_name:
            d = sols[name].clone()
            axpby(-1.0, sols[ref_name], 1.0, d)
            out[f"rel_diff_{name}_vs_{ref_name}"] = norm2(d) / norm2(sols[ref_name])
    if profile:
        # per-phase GPU time of 500 iterations of one more mixed solve, from the library's per-range events
        x = torch.zeros(4 * N, dtype=torch.float64, device=dev)
        profile_enable(True)
        fgmres_solve(P64, bt, x, solve_opts(restart=restart, max_iters=500, rtol=rtol,
                                            inner=torch.float32, precond=precond, vel_steps=vel_steps),
                     J32=P32, pinv=pinv32,
                     check=False)
        torch.cuda.synchronize()
        ph = {}
        for name in ("fgmres_apply", "fgmres_precond", "fgmres_orth", "fgmres_residual",
                     "vms_q2_cells", "vms_gather", "schur_apply"):
            tot, n = profile_read(name)
            ph[name] = {"ms_total": round(tot, 2), "calls": n}
        profile_enable(False)
        out["phases_mixed"] = ph
    for m in ("mixed", "mixed_b32"):
        if m in out and "f64" in out:
            out[f"speedup_{m}_vs_f64"] = round(out["f64"]["ms"] / out[m]["ms"], 3)
    return out


def solid_kappa(cfg, M, c_stiff=0.0):
    """Per-point weight through which the preconditioners see the solid block: its lumped inertia
    c_M (rho_s0 - rho_f) V / M plus, with c_stiff > 0, a stiffness share c_stiff dt C0 (V / M) / h^2
    (h the fluid cell size: the block's diagonal at a fluid node is the strain energy of the
    node's shape function over the solid, about dt C0 V_support / h^2)."""
    import numpy as np
    vb = W.plate_volume() / M
    h = cfg.grid.h[0]
    mat = W.SOLID_MATERIAL
    return np.full(M, cfg.c_m * (mat["rho_s0"] - mat["rho_f"]) * vb + c_stiff * cfg.dt * mat["C0"] * vb / (h * h))


def solid_solve(rtol=1e-8, restart=50, max_iters=3000, precond="schur_tri", vel_steps=2, workload="c2",
                c_stiff=0.0):
    """One linear solve of the reduced system with the hyperelastic solid block (64^3 channel,
    the plates meshed by ~200k-node hexahedra at a deformed state), FP32 inner applies and
    FP64 outer FGMRES to rtol, against the same solve with the per-point stand-in kappa on the
    same points.  The preconditioners see a per-point kappa in both: the stand-in's own, and
    for the solid block its lumped inertia c_M (rho_s0 - rho_f) V / M."""
    import numpy as np

    from . import (Problem, Solid, bjacobi_setup, dlm_gram, dlm_locate, fgmres_solve, jacobian_apply,
                   make_params, schur_setup, solve_opts)

    cfg = W.CONFIGS[workload]
    g = cfg.grid
    N = g.num_nodes
    dev = torch.device("cuda")

    def t(v, dt=torch.float64):
        return torch.tensor(np.ascontiguousarray(v).ravel(), dtype=dt, device=dev)

    n_t, n_f = W.solid_mesh_size(cfg.m_points)
    X0, conn = W.plate_solid_mesh(n_t, n_f)
    U = W.solid_displacement(X0, cfg.seed_fields)
    M = X0.shape[1]
    cM, cK, cV = cfg.c_m, cfg.dt, 1.0
    S = Solid(t(X0), torch.tensor(conn.ravel(), dtype=torch.int32, device=dev), **W.SOLID_MATERIAL)
    Ut = t(U)
    a = W.advection_field(g, cfg.seed_fields)
    mask = W.channel_dirichlet_mask(g)
    mt = torch.tensor(W.mask_to_bits(mask).view(np.int32), device=dev)
    b = W.smooth_fourier_field(g, cfg.seed_vectors)
    b[:3][mask] = 0.0
    bt = t(b)
    bnorm = norm2(bt)
    prm = make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    Xt = t(X0 + U)
    tab64 = dlm_locate(g, Xt, dtype=torch.float64, s_max=cfg.s_max)
    tab32 = dlm_locate(g, Xt, dtype=torch.float32, s_max=cfg.s_max)
    out = {"workload": f"{g.n[0]}^3 Q1 channel, plates meshed by {conn.shape[0]} hexahedra ({M} nodes)",
           "rtol": rtol, "restart": restart, "precond": precond, "vel_steps": vel_steps, "c_stiff": c_stiff,
           "n_occupied_cells": tab64.n_occ}
    kap_standin = W.kappa_weights(M, W.plate_volume(), cfg.c_m, cfg.alpha)
    kap_inertia = solid_kappa(cfg, M, c_stiff)
    y = torch.empty_like(bt)
    for name, kap, solid in (("standin", kap_standin, False), ("solid", kap_inertia, True)):
        k64, k32 = t(kap), t(kap, torch.float32)
        extra = dict(solid=S, solid_U=Ut, solid_coefs=(cM, cK, cV)) if solid else {}
        P64 = Problem(g, prm, t(a), tab64, k64, s=tab64.s, mask=mt, gram=dlm_gram(g, tab64, k64), **extra)
        P32 = Problem(g, prm, t(a, torch.float32), tab32, k32, s=tab32.s, mask=mt, gram=dlm_gram(g, tab32, k32),
                      **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if precond == "bjacobi":
            _, pc, _, _ = bjacobi_setup(P64)
        else:
            _, _, blocks, _ = bjacobi_setup(P64, want32=False, want_blocks=True)
            pc = schur_setup(P64, blocks)
            del blocks
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        x = torch.zeros(4 * N, dtype=torch.float64, device=dev)
        t0 = time.perf_counter()
        rc, st = fgmres_solve(P64, bt, x, solve_opts(restart=restart, max_iters=max_iters, rtol=rtol,
                                                      inner=torch.float32, precond=precond, vel_steps=vel_steps),
                              J32=P32, pinv=pc, check=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        jacobian_apply(P64, x, y)
        r = bt.clone()
        axpby(-1.0, y, 1.0, r)
        out[name] = {"status": rc, "iters": st.iters, "ms": round(ms, 1), "setup_ms": round(setup_ms, 1),
                     "ms_per_iter": round(ms / max(st.iters, 1), 3),
                     "recomputed_rel_residual": norm2(r) / bnorm}
        _log(f"solid solve {name}: rc {rc}, {st.iters} it, {ms:.0f} ms, residual {norm2(r) / bnorm:.3e}")
    return out


def solid_steps(steps=3, precond="schur_tri", vel_steps=8, inner="f32", workload="c2", inflow=1.0, c_stiff=0.0,
                integrator="be", rho_inf=0.5, gravity=None, basis32=False):
    """Coupled time steps with the elastic plates moving with the fluid (the configuration's
    channel, the plates meshed by hexahedra with about the configuration's point count, stress
    free at rest; inflow u_x = `inflow` on x = 0 from a fluid at rest) through
    solid_stepper.SolidChannel: per step, locate the solid nodes at X0 + U_n, then Newton on the
    step residual with the solid to 1e-8 of the initial residual, FGMRES with `precond` built from
    the per-point kappa of solid_kappa.  Reports Newton / Krylov iterations and wall time per
    step, and the solid's motion."""
    from .solid_stepper import SolidChannel

    cfg = W.CONFIGS[workload]
    n_t, n_f = W.solid_mesh_size(cfg.m_points)
    X0, conn = W.plate_solid_mesh(n_t, n_f)
    run = SolidChannel(cfg, X0, conn, integrator=integrator, rho_inf=rho_inf, precond=precond, vel_steps=vel_steps,
                       inner=inner, inflow=inflow, kappa=solid_kappa(cfg, X0.shape[1], c_stiff), gravity=gravity,
                       basis32=basis32)
    rows = []
    for _ in range(steps):
        rec = run.step()
        rec.pop("stage_x")
        rec.pop("tol")
        rec["solid_speed_max"] = float(run.Vs.abs().max())
        rec["solid_disp_max"] = float(run.U.abs().max())
        rows.append(rec)
        _log(f"solid step {rec['step']}: rc {rec['status']}, {rec['newton']} Newton / {rec['krylov']} Krylov, "
             f"{rec['ms_newton']:.0f} ms")
    g = cfg.grid
    return {"workload": f"{g.n[0]}^3 Q1 channel, elastic plates meshed by {conn.shape[0]} hexahedra "
                        f"({X0.shape[1]} nodes), inflow {inflow}, dt {cfg.dt}",
            "integrator": integrator, "rho_inf": rho_inf if integrator != "be" else None, "precond": precond,
            "vel_steps": vel_steps, "inner": inner, "c_stiff": c_stiff, "gravity": gravity, "steps": rows}
