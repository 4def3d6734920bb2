"""Measurement drivers for the Newton-step workloads (orchestration only).

warmstart_c4: 64^3 Q1 channel, three rotating plates (200k points), 200
  implicit steps with the plain guess (mixed-precision Newton); the network is
  trained on samples from steps 1-100 and evaluated on steps 101-200, where
  every step is re-solved from the recorded state three ways: plain guess with
  FP64 inner Krylov applies, plain guess with FP32 inner applies, learned guess
  with FP32 inner applies.  All three stop at the same absolute residual.
large_c5: 192^3 Q1 channel, 2M points: after warm-up steps, one Newton step
  plain FP64 vs mixed precision + learned warm start (the 64^3 network applied
  fully convolutionally to the finer lattice).
"""
from __future__ import annotations

import json
import math
import statistics
import sys
import time

import torch

import fsi_workloads as W

from . import axpby, norm2
from .learned import LearnedWarmStart
from .stepper import ChannelRun


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _solve_modes(run, lw, k, modes):
    out = {}
    sols = {}
    for mode in modes:
        run.x = run.history[k].x.clone()
        run.n = k
        inner = torch.float64 if mode.endswith("f64") else torch.float32
        gf = None
        if lw is not None and mode.startswith("nn"):
            gf = lw.guess
        elif lw is not None and mode.startswith("extrap"):
            gf = lw.extrapolation_guess
        rec = run.step(guess_fn=gf, inner=inner, record=False)
        out[mode] = dict(newton=rec.newton_iters, krylov=rec.krylov_iters, ms_newton=rec.ms_newton,
                         ms_guess=rec.ms_guess, res_plain=rec.res_plain, res_guess=rec.res_guess,
                         used_guess=rec.used_guess, hist=rec.res_hist)
        sols[mode] = rec.x
    ref = sols[modes[0]]
    nref = norm2(ref)
    for mode in modes[1:]:
        d = sols[mode].clone()
        axpby(-1.0, ref, 1.0, d)
        out[mode]["rel_diff_vs_" + modes[0]] = norm2(d) / nref
    return out


def warmstart_c4(steps=200, train_end=100, epochs=20, lr=1e-3, eval_stride=1, seed=0,
                 save_path=None):
    cfg = W.CONFIGS["c4"]
    run = ChannelRun(cfg)
    run.record_extrap = True
    t0 = time.perf_counter()
    for n in range(steps):
        rec = run.step()
        if (n + 1) % 10 == 0 or n < 3:
            _log(f"c4 step {rec.n}: t={rec.t:.3f} inflow={rec.inflow:+.3f} newton={rec.newton_iters} "
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
    modes = ["plain_f64", "plain_mixed", "extrap_mixed", "nn_mixed"]
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
        "workload": "64^3 Q1 channel, 200k points on three rotating plates, dt=1e-3",
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
    for m in ("extrap_mixed", "nn_mixed"):
        summary[m]["guess_used_frac"] = statistics.mean(1.0 if r[m]["used_guess"] else 0.0 for r in rows)
        summary[m]["res_ratio_median"] = statistics.median(r[m]["res_guess"] / r[m]["res_plain"] for r in rows)
    for m in modes[1:]:
        summary[m]["max_rel_diff_vs_plain_f64"] = max(r[m]["rel_diff_vs_plain_f64"] for r in rows)
    summary["newton_hist_example"] = {m: ["%.2e" % h for h in rows[len(rows) // 2][m]["hist"]] for m in modes}
    summary["speedup_nn_mixed_vs_plain_f64"] = round(summary["plain_f64"]["ms_per_step"] / summary["nn_mixed"]["ms_per_step"], 3)
    summary["speedup_plain_mixed_vs_plain_f64"] = round(summary["plain_f64"]["ms_per_step"] / summary["plain_mixed"]["ms_per_step"], 3)
    return summary, lw


def large_c5(lw_c4=None, warmup_steps=3, state_path=None):
    cfg = W.CONFIGS["c5"]
    run = ChannelRun(cfg)
    for n in range(warmup_steps):
        rec = run.step()
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
    modes = ["plain_f64", "plain_mixed"] + (["extrap_mixed", "nn_mixed"] if lw is not None else [])
    r = _solve_modes(run, lw, k, modes)
    for m in modes:
        _log(f"c5 step {k + 1} {m}: {r[m]['newton']}N/{r[m]['krylov']}K "
             f"{r[m]['ms_newton'] + r[m]['ms_guess']:.0f} ms")
    best = "nn_mixed" if lw is not None else "plain_mixed"
    summary = {"workload": "192^3 Q1 channel, 2M points on three rotating plates",
               "step": k + 1, "dof": 4 * run.N, "modes": r,
               "speedup_" + best + "_vs_plain_f64":
                   round((r["plain_f64"]["ms_newton"] + r["plain_f64"]["ms_guess"]) /
                         (r[best]["ms_newton"] + r[best]["ms_guess"]), 3)}
    return summary
