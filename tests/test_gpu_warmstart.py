"""What the trained warm-start network gains over the method without it (the learned warm
start is an addition to the predictor of section 2.4's Newton steps), and over its own backbone.

A 16^3 rotating-plates channel is advanced 30 backward-Euler steps; the network is trained
with the library's own forward / backward kernels and Adam on steps 2-20, and steps 21-30
are then re-solved from the same states with the plain previous-step guess, the linear
extrapolation (the network's backbone) and the network's guess.  Every solve stops at the
same absolute residual (1e-8 of the plain guess's residual), so the guess may only change
iteration counts, never the converged answer.
"""
import dataclasses
import statistics

import pytest

import fsi_workloads as W

pytestmark = pytest.mark.gpu


def test_learned_guess_gains_over_the_plain_guess():
    import torch
    from paper_2601_08266_amd import experiments as ex
    from paper_2601_08266_amd.learned import LearnedWarmStart
    from paper_2601_08266_amd.stepper import ChannelRun
    cfg = dataclasses.replace(W.CONFIGS["c4"], grid=W.Grid((16, 16, 16), 1), m_points=8000)
    run = ChannelRun(cfg, precond="schur_tri", vel_steps=2)
    run.record_extrap = True
    for _ in range(30):
        run.step()
    lw = LearnedWarmStart(run, seed=0)
    ks = list(range(1, 20))
    lw.fit_normalisation(run.history, ks)
    lw.build_dataset(run.history, ks)
    lw.train(epochs=15, lr=1e-3, seed=0)
    assert lw.losses[-1] < lw.losses[0]
    modes = ["plain_mixed", "extrap_mixed", "nn_mixed"]
    rows = [ex._solve_modes(run, lw, k, modes) for k in range(20, 30)]

    def mean(mode, key):
        return statistics.mean(r[mode][key] for r in rows)

    for m in modes:
        print(f"{m}: krylov {mean(m, 'krylov'):.1f}, newton {mean(m, 'newton'):.2f}, "
              f"initial residual / plain {statistics.mean(r[m]['res_guess'] / r[m]['res_plain'] for r in rows):.3e}, "
              f"ms {mean(m, 'ms_newton') + mean(m, 'ms_guess'):.1f}", flush=True)
    for r in rows:
        # the guess starts lower than the plain one (the safeguard never takes a worse guess) ...
        assert r["nn_mixed"]["res_guess"] < r["nn_mixed"]["res_plain"]
        # ... and the converged state is the same to the accuracy the common tolerance allows
        assert r["nn_mixed"]["rel_diff_vs_plain_mixed"] <= 1e-5
    # the network's own guess (not the safeguard's fallback) is the one used in most steps
    used = sum(1 for r in rows if r["nn_mixed"]["used_guess"] is True)
    assert used >= 0.8 * len(rows), used
    # fewer Krylov iterations than the plain guess
    assert mean("nn_mixed", "krylov") < mean("plain_mixed", "krylov")
    # what the network adds over its own backbone, the linear extrapolation it corrects: the
    # measured result is that it does not pay (Krylov counts within a fraction of an iteration,
    # wall time including the inference larger); recorded, not hidden
    nn_k, ex_k = mean("nn_mixed", "krylov"), mean("extrap_mixed", "krylov")
    nn_ms = mean("nn_mixed", "ms_newton") + mean("nn_mixed", "ms_guess")
    ex_ms = mean("extrap_mixed", "ms_newton") + mean("extrap_mixed", "ms_guess")
    print(f"network vs extrapolation: krylov {nn_k:.2f} vs {ex_k:.2f}, ms {nn_ms:.1f} vs {ex_ms:.1f}")
    if not (nn_k < ex_k and nn_ms < ex_ms):
        pytest.xfail(f"the learned correction does not beat the extrapolation it corrects: "
                     f"{nn_k:.2f} vs {ex_k:.2f} Krylov iterations, {nn_ms:.1f} vs {ex_ms:.1f} ms per step")
