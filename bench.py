#!/usr/bin/env python
"""Benchmark of the immersed FD/DLM Jacobian hot path on one MI355X.

Metric: GDOF/s of the VMS+DLM Jacobian apply, GDOF/s = 4 N_nodes / t_apply, and
the wall time of a Newton step to the 1e-8 residual.
Workload (default): 192^3 Q1-Q1 grid (7,189,057 nodes, 28,756,228 DOF), Oseen
linearisation about a seeded smooth advection field (nu = 1e-2, dt = 1e-3),
three thin curved plates with 2,000,000 solid points (apply mode, no Dirichlet
mask).  One step = one J x: the VMS operator (Galerkin + SUPG/PSPG/LSIC,
section 2.1) plus the DLM block B^T diag(kappa) B (sections 2.3/2.4), in FP64;
the FP32 rate and the point-by-point DLM path are reported beside it.  Inputs
are synthetic and resident in HBM before timing starts; the vectors (690 MB per
apply) do not fit the 256 MB Infinity Cache.

Also reported: the roofline of the dominant kernel (vms_q1_cells, FP64 vector-ALU
bound) from library-side hipEvents recorded on its launch stream over the timed
applies, the standalone B / B^T, the solid block, the Newton-step block on the
192^3 rotating-plates channel (plain FP64, mixed precision, extrapolated and
learned warm starts, Picard and full tangent, all to the same absolute
residual), and the oracle's apply on the host cores.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (fma) x 2.4 GHz
PEAK_HBM_GBS = 8000.0

# HBM traffic of vms_q1_cells<double> on the headline workload from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
# for a plain 512 MiB device copy (FETCH_SIZE reads half the copied bytes, WRITE_SIZE all).
# Valid only for the kernel sources it was taken on: the hash covers them.
CELL_TRAFFIC = {"workload": "c5", "sources_sha256_16": "97e17f3a7b1ed8d9", "fetch_kib": 379826.6, "write_kib": 351971.9,
                "fetch_scale": 524288.0 / 262171.5625, "write_scale": 1.0}
CELL_SOURCES = ("vms_q1.hip", "kernels.hpp", "common.hpp")


def cell_traffic_bytes(workload="c5"):
    """Scaled FETCH+WRITE bytes per launch, or None if the kernel changed since the counters
    or the workload is not the one they were taken on."""
    import hashlib
    if workload != CELL_TRAFFIC["workload"]:
        return None
    h = hashlib.sha256()
    for f in CELL_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_08266_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != CELL_TRAFFIC["sources_sha256_16"]:
        return None
    t = CELL_TRAFFIC
    return round(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def q1_cell_flops(has_s=True, visc_strong=True):
    """Flops vms_q1_cells spends on one Q1 cell in apply mode (fma = 2, add/mul = 1,
    the hardware 1/sqrt estimate = 1), counted from the kernel's arithmetic.

    Point table: Gauss values of s and of the 3 advection components by one
    interpolation pass per axis (12 x (sub + 2 fma) = 60 each), a/h (24), a.Ga (48);
    per point tau_b (2), 1/sqrt with two Newton steps (13), tau_c (2); the
    velocity/pressure fields to monomial form (4 x 12).
    Element loop, per x-pair of points: E and O of 4 fields (24 fma).  Per point:
    values and y/z derivatives (4 + 24 fma), div u (5), nu grad div u (21), the
    three momentum residuals times tau_m (33), tau_c div - p (2), the 9 test-side
    fluxes (45), the pressure fluxes (3), monomial moments of 4 fields (4 x 36).
    Then the Gauss weight (32) and the moments back to nodes (48).
    """
    table = (60 if has_s else 0) + 3 * 60 + 24 + 48 + 8 * 17 + 48
    per_point = 56 + 5 + (21 if visc_strong else 0) + 33 + 2 + 45 + 3 + 4 * 36
    loop = 4 * 48 + 8 * per_point
    return table + loop + 32 + 48


def q2_cell_flops(has_s=True):
    """Flops vms_q2_cells spends on one Q2 cell in apply mode (fma = 2, add/mul/sqrt/div = 1),
    counted from the kernel's arithmetic; a cell is 27 lanes, lane j one node / one Gauss point.
    Per lane: the sum-factorised interpolation of u, v, w with second derivatives (x pass 9,
    y pass 18, z pass 30 fma: 114 each), of p with its gradient (6 + 9 + 12 fma: 54), of the 3
    advection components and s (values only, 3 + 3 + 3 fma: 18 each); the pointwise terms
    (physical derivatives and Hessians 21 + lap 6, grad p 3, tau 10, div 2, the three momentum
    residuals times tau_m 45, tau_c div - p 2, the 12 test-side fluxes 39, Gauss weight and
    scaling 31: 159); the four transposed contractions (12 + 9 + 6 fma: 54 each); the ordered
    node accumulation (4).  Plus the cell's smallest nodal s (26 compares)."""
    per_lane = 3 * 114 + 54 + (4 if has_s else 3) * 18 + 159 + 4 * 54 + 4
    return 27 * per_lane + (26 if has_s else 0)


def q2_dlm_cell_flops():
    """Extra flops of an occupied Q2 cell: its 27x27 block on 3 velocity components."""
    return 2 * 27 * 27 * 3


def dlm_cell_flops():
    """Extra flops of an occupied cell: its 8x8 block on 3 velocity components (192 fma)
    and the velocity back to nodal form (3 x 12)."""
    return 2 * 192 + 36


def solid_elem_flops():
    """Flops solid_elem_k spends on one hexahedron (8 lanes, one per Gauss point; fma = 2,
    add/mul/div/cbrt = 1), counted from the kernel's arithmetic, per lane:
    23 trilinear shape evaluations (10 each); dX/dxi from 7 corner differences (7 x 21);
    its determinant, cofactors and inverse (51); reference gradients, displacement
    differences, v at the point, F and dF over 8 corners (8 x 60); F + I (3); det,
    cofactors and F^{-T} (51); I1, F^{-T}:dF, F:dF (54); d(F^{-T}) (99); J^{-2/3} and the
    scalar factors (13); grad_x v (45); the stress increment Q with the viscous term
    (9 x 26 + 2); inertia factor and weight (4); nodal forces of 8 corners (8 x 15
    gradients + 8 x 27) and their 8-lane sums (8 x 9)."""
    per_lane = (23 * 10 + 7 * 21 + 51 + 8 * 60 + 3 + 51 + 54 + 99 + 13 + 45 + 9 * 26 + 2 + 4 +
                8 * (15 + 27 + 9))
    return 8 * per_lane


def solid_cpu_baseline(X0, conn, U, cM, cK, cV, n_elem=300):
    """The oracle's solid apply (dense 24x24 element blocks, numpy, one core) on the first
    n_elem elements of the same mesh: elements per second."""
    import numpy as np

    import fsi_workloads as W
    from oracle import solid as osolid

    sub = conn[:n_elem]
    v = np.ones_like(U)
    t0 = time.perf_counter()
    y = osolid.apply(X0, sub, U, v, W.SOLID_MATERIAL, cM, cK, cV)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(y))
    return {"value": round(n_elem / dt, 1), "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"the oracle's FP64 solid apply on the first {n_elem} of the mesh's elements, {dt:.2f} s"}


def time_solid(fsi, torch, cfg, reps=50, cpu=True):
    """Hyperelastic solid block on the workload's plate mesh (nodes = the DLM points, about
    cfg.m_points of them): fsi_solid_apply and the reduced-system Jacobian with the solid
    block (fsi_jacobian_solid_apply), FP64 and FP32, timed with events on the launch stream;
    the element kernel's average duration from the library's per-kernel events."""
    import numpy as np

    import fsi_workloads as W

    g = cfg.grid
    N = g.num_nodes
    n_t, n_f = W.solid_mesh_size(cfg.m_points)
    X0, conn = W.plate_solid_mesh(n_t, n_f)
    U = W.solid_displacement(X0, cfg.seed_fields)
    M, ne = X0.shape[1], conn.shape[0]

    def t(v, dt=torch.float64):
        return torch.tensor(np.ascontiguousarray(v).ravel(), dtype=dt, device="cuda")

    S = fsi.Solid(t(X0), torch.tensor(conn.ravel(), dtype=torch.int32, device="cuda"), **W.SOLID_MATERIAL)
    Ut = t(U)
    cM, cK, cV = cfg.c_m, cfg.dt, 1.0
    prm = fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    v = W.random_vector(3 * M, cfg.seed_vectors + 1)
    out = {"mesh_nodes": M, "mesh_elements": ne}

    def timed(fn):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        vt, yt = t(v, dt), torch.empty(3 * M, dtype=dt, device="cuda")
        sws = torch.empty(int(fsi._lib.lib().fsi_solid_workspace(ne, fsi.dtype_code(dt))), dtype=torch.uint8,
                          device="cuda")
        ms = timed(lambda: fsi.solid_apply(S, Ut, vt, cM, cK, cV, y=yt, ws=sws))
        fsi.profile_enable(True)
        for _ in range(reps):
            fsi.solid_apply(S, Ut, vt, cM, cK, cV, y=yt, ws=sws)
        torch.cuda.synchronize()
        kern = {}
        for kname in ("solid_elem", "solid_gather"):
            tot, n = fsi.profile_read(kname)
            kern[kname] = round(tot / n, 6) if n else 0.0
        fsi.profile_enable(False)
        tab = fsi.dlm_locate(g, t(X0 + U), dtype=dt, s_max=cfg.s_max)
        prob = fsi.Problem(g, prm, t(a, dt), tab, None, s=tab.s)
        xt, jy = t(x, dt), torch.empty(4 * N, dtype=dt, device="cuda")
        jws = torch.empty(fsi.jacobian_solid_workspace(prob, S), dtype=torch.uint8, device="cuda")
        jms = timed(lambda: fsi.jacobian_solid_apply(prob, S, Ut, xt, cM, cK, cV, y=jy, ws=jws))
        elem_ms = kern["solid_elem"]
        out[name] = {
            "solid_apply_us": round(ms * 1e3, 2),
            "kernels_ms": kern,
            "solid_elem_TFLOPs": round(solid_elem_flops() * ne / (elem_ms * 1e-3) / 1e12, 3) if elem_ms else None,
            "jacobian_with_solid_us": round(jms * 1e3, 2),
            "jacobian_with_solid_gdofs": round(4 * N / (jms * 1e-3) / 1e9, 4),
        }
    out["solid_elem_flops_per_element"] = solid_elem_flops()
    out["gpu_elements_per_s_f64"] = round(ne / (out["f64"]["solid_apply_us"] * 1e-6), 1)
    if cpu:
        out["cpu_baseline"] = solid_cpu_baseline(X0, conn, U, cM, cK, cV)
    return out


def build_problem(cfg, dtype, dev):
    import numpy as np
    import torch

    import fsi_workloads as W
    import paper_2601_08266_amd as fsi

    g = cfg.grid
    N = g.num_nodes
    if cfg.solid == "sphere":
        X = W.sphere_points()
        vol = W.sphere_volume()
    else:
        X = W.plate_points(cfg.m_points, cfg.seed_fields)
        vol = W.plate_volume()
    kappa = W.kappa_weights(X.shape[1], vol, cfg.c_m, cfg.alpha)
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)

    def t(v, dt=dtype):
        return torch.tensor(np.ascontiguousarray(v).ravel(), dtype=dt, device=dev)

    Xt = t(X, torch.float64)
    fsi.dlm_locate(g, Xt, dtype=dtype, s_max=cfg.s_max)      # first call loads the code objects
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tab = fsi.dlm_locate(g, Xt, dtype=dtype, s_max=cfg.s_max)
    torch.cuda.synchronize()
    locate_ms = (time.perf_counter() - t0) * 1e3
    prm = fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    kt = t(kappa)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gram = fsi.dlm_gram(g, tab, kt)
    torch.cuda.synchronize()
    gram_ms = (time.perf_counter() - t0) * 1e3
    prob = fsi.Problem(g, prm, t(a), tab, kt, s=tab.s, mask=None, gram=gram)
    xt = t(x)
    y = torch.empty_like(xt)
    ws = torch.empty(prob.workspace_bytes(), dtype=torch.uint8, device=dev)
    return dict(prob=prob, x=xt, y=y, ws=ws, tab=tab, locate_ms=locate_ms, gram_ms=gram_ms, Xt=Xt, N=N,
                a_np=a, x_np=x, X_np=X, kappa_np=kappa)


def time_q2_apply(fsi, torch, steps=20, warmup=5):
    """The Q2 Jacobian apply of the 96^3 Q2-Q2 grid with 500k plate points (the mixed-precision
    solve configuration's operator), FP64 and FP32: GDOF/s and the cell kernel's rate against
    the FP64 vector peak, from the library's per-kernel events."""
    import fsi_workloads as W

    cfg = W.CONFIGS["c3"]
    g = cfg.grid
    out = {"workload": f"{cfg.name}: {g.n[0]}^3 Q2-Q2 VMS+DLM Jacobian apply, {cfg.m_points} points",
           "dof": 4 * g.num_nodes, "cells": g.num_cells}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        case = build_problem(cfg, dt, torch.device("cuda:0"))
        ms, _, kern = time_applies(fsi, torch, case, steps, warmup, profile=True,
                                   kernels=("vms_q2_cells", "vms_gather"))
        cell_ms = kern["vms_q2_cells"][0]
        flops = q2_cell_flops() * g.num_cells + q2_dlm_cell_flops() * case["tab"].n_occ
        tf = flops / (cell_ms * 1e-3) / 1e12 if cell_ms > 0 else 0.0
        out[name] = {"ms_per_apply": round(ms, 4), "gdofs": round(4 * case["N"] / (ms * 1e-3) / 1e9, 3),
                     "kernels_ms": {k: round(v[0], 4) for k, v in kern.items()},
                     "cell_TFLOPs": round(tf, 2), "cell_frac_of_78.6": round(tf / PEAK_FP64_VALU_TFLOPS, 4)}
        del case
    out["flops_per_cell"] = q2_cell_flops()
    return out


def time_dlm(fsi, torch, case, reps=50):
    """Standalone B u and y += B^T (kappa lam) (fsi_dlm_B / fsi_dlm_BT, FP64) on the workload's
    point set, timed with events on the launch stream over `reps` calls each; then the same with
    the per-point vectors in located order (fsi_dlm_B_located, fsi_dlm_BT with perm = NULL), and
    the one-off cost of moving 3 fields into located order (fsi_dlm_permute)."""
    g, tab, N = case["prob"].grid, case["tab"], case["N"]
    m = tab.m
    u = case["x"][: 3 * N]
    Bu = torch.empty(3 * m, dtype=torch.float64, device="cuda")
    lam = torch.ones(3 * m, dtype=torch.float64, device="cuda")
    y = torch.zeros(3 * N, dtype=torch.float64, device="cuda")
    kap = case["prob"].kappa
    ws = torch.empty(int(fsi._lib.lib().fsi_dlm_BT_workspace(ctypes.byref(g), tab.n_occ, 0)) or 1,
                     dtype=torch.uint8, device="cuda")
    xi_loc = fsi.dlm_permute(tab, tab.xi, 3)
    kap_loc = fsi.dlm_permute(tab, kap, 1)
    lam_loc = torch.empty_like(lam)
    out = {}
    for name, fn in (("B", lambda: fsi.dlm_B(g, tab, u, Bu)),
                     ("BT", lambda: fsi.dlm_BT(g, tab, lam, y, kappa=kap, ws=ws)),
                     ("B_located", lambda: fsi.dlm_B_located(g, tab, xi_loc, u, Bu)),
                     ("BT_located", lambda: fsi.dlm_BT(g, tab, lam_loc, y, kappa=kap_loc, ws=ws, xi_loc=xi_loc)),
                     ("permute3", lambda: fsi.dlm_permute(tab, lam, 3, dst=lam_loc))):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / reps * 1e3
        out[f"dlm_{name}_us"] = round(us, 2)
        out[f"dlm_{name}_Gpoints_per_s"] = round(m / us * 1e-3, 3)
    return out


def time_applies(fsi, torch, case, steps, warmup, profile, kernels=("vms_q1_cells", "vms_gather")):
    """Time `steps` back-to-back applies (no per-kernel events in this pass); then, if asked,
    the same number again with the library's per-kernel hipEvents for the kernel breakdown."""
    prob, x, y, ws = case["prob"], case["x"], case["y"], case["ws"]
    apply = prob.bind(x, y, ws)
    for _ in range(warmup):
        apply()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        apply()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = start.elapsed_time(stop) / steps
    kern = {}
    if profile:
        fsi.profile_enable(True)
        for _ in range(steps):
            apply()
        torch.cuda.synchronize()
        for name in kernels:
            tot, n = fsi.profile_read(name)
            kern[name] = (tot / n if n else 0.0, n)
        fsi.profile_enable(False)
    return ms, wall / steps * 1e3, kern


def time_blocks(fsi, torch, case, steps, warmup):
    """The Schur preconditioner's block products on the same problem: velocity rows of J on
    (x_u, 0) (block F) and on (0, x_p) (block G), `steps` back-to-back calls each, then the same
    again with the library's per-kernel events (cell pass and three-row gather)."""
    prob, x, y, ws = case["prob"], case["x"], case["y"], case["ws"]
    out = {}
    for name, blk, cell in (("F", fsi.BLOCK_F, "vms_q1_block_u"), ("G", fsi.BLOCK_G, "vms_q1_block_p")):
        def call():
            fsi.jacobian_apply_block(prob, blk, x, y, ws)
        for _ in range(warmup):
            call()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(steps):
            call()
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        fsi.profile_enable(True)
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        kern = {}
        for k in (cell, "vms_gather"):
            tot, n = fsi.profile_read(k)
            kern[k] = round(tot / n, 6) if n else 0.0
        fsi.profile_enable(False)
        out[name] = {"us": round(ms * 1e3, 2), "kernels_ms": kern}
    return out


def time_cold(torch, case, reps=20):
    """The same Jacobian apply with the 256 MB Infinity Cache flushed before each one: a 512 MiB
    buffer is overwritten between applies and only the apply is timed (events on the launch
    stream around each apply; mean over reps)."""
    prob, x, y, ws = case["prob"], case["x"], case["y"], case["ws"]
    apply = prob.bind(x, y, ws)
    flush = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i in range(reps + 2):
        flush.fill_(float(i))
        if i >= 2:
            ev[i - 2][0].record()
        apply()
        if i >= 2:
            ev[i - 2][1].record()
    torch.cuda.synchronize()
    ms = sum(a.elapsed_time(b) for a, b in ev) / reps
    del flush
    return ms


PROBE_MODES = ["plain_f64", "plain_mixed", "extrap_mixed", "plain_f64_st", "plain_mixed_st", "extrap_mixed_st",
               "plain_f64_st2", "plain_mixed_st2", "extrap_mixed_st2"]


def newton_step_probe(warm_steps=60, measure_steps=3, modes=None, integrator="be", rho_inf=0.5):
    """Short Newton-step comparison on the 64^3 rotating-plates channel: after a few plain steps,
    the next steps are re-solved from the same state with plain FP64, mixed precision, and mixed
    precision + extrapolated warm start, each with the block-Jacobi and (suffix _st) the
    Schur-complement block-triangular preconditioner, the latter also with two minimal-residual
    steps on its velocity block (_st2); all stop at the same absolute residual."""
    import torch

    import fsi_workloads as W
    from paper_2601_08266_amd import experiments as ex
    from paper_2601_08266_amd.stepper import ChannelRun

    run = ChannelRun(W.CONFIGS["c4"], integrator=integrator, rho_inf=rho_inf)
    for _ in range(warm_steps):
        run.step()
    rows = []
    for k in range(warm_steps, warm_steps + measure_steps):
        rows.append(ex._solve_modes(run, None, k, modes or PROBE_MODES))
        run.restore(k)
        run.step()
    out = {"workload": "64^3 Q1 channel, 200k rotating-plate points, steps "
                       f"{warm_steps + 1}-{warm_steps + measure_steps}, tol 1e-8*||R(x_plain)||",
           "integrator": integrator if integrator == "be" else f"{integrator} rho_inf={rho_inf}"}
    for m in modes or PROBE_MODES:
        out[m + "_ms"] = round(sum(r[m]["ms_newton"] + r[m]["ms_guess"] for r in rows) / len(rows), 2)
        out[m + "_krylov"] = round(sum(r[m]["krylov"] for r in rows) / len(rows), 1)
    if "plain_f64_ms" in out and "extrap_mixed_ms" in out:
        out["speedup_mixed_extrap_vs_plain_f64"] = round(out["plain_f64_ms"] / out["extrap_mixed_ms"], 3)
    if "plain_f64_ms" in out and "extrap_mixed_st_ms" in out:
        # the fastest form (mixed precision, extrapolated guess, Schur-complement preconditioner)
        # against plain FP64 Newton with block-Jacobi and against plain FP64 with the same preconditioner
        out["speedup_extrap_mixed_st_vs_plain_f64"] = round(out["plain_f64_ms"] / out["extrap_mixed_st_ms"], 3)
    if "plain_f64_st_ms" in out and "extrap_mixed_st_ms" in out:
        out["speedup_extrap_mixed_st_vs_plain_f64_st"] = round(out["plain_f64_st_ms"] / out["extrap_mixed_st_ms"], 3)
    if "plain_f64_ms" in out and "extrap_mixed_st2_ms" in out:
        # with two minimal-residual velocity steps in the Schur preconditioner (the fastest form)
        out["speedup_extrap_mixed_st2_vs_plain_f64"] = round(out["plain_f64_ms"] / out["extrap_mixed_st2_ms"], 3)
    if "plain_f64_st2_ms" in out and "extrap_mixed_st2_ms" in out:
        out["speedup_extrap_mixed_st2_vs_plain_f64_st2"] = round(out["plain_f64_st2_ms"] / out["extrap_mixed_st2_ms"], 3)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_jacobian(cfg, grid, a, x, X, kappa):
    import numpy as np

    from oracle import dlm as odlm
    from oracle import jacobian as ojac
    from oracle import vms as ovms

    prm = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    cell, xi = odlm.locate(grid, X)
    s = odlm.s_field(grid, cell, cfg.s_max)
    ovms.lib()
    t0 = time.perf_counter()
    y = ojac.apply(grid, prm, a, x, cell, xi, kappa, s=s)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(y))
    return dt


def slab_case(cfg, layers=4):
    """A slab of `layers` cell layers through the middle of the workload's grid (the same
    advection field, vector and points restricted to it): the oracle's one-core sample."""
    import numpy as np

    import fsi_workloads as W

    g = cfg.grid
    N = g.num_nodes
    nx, ny, nz = g.nodes_per_axis
    k0 = g.n[2] // 2 - layers // 2
    sg = W.Grid((g.n[0], g.n[1], layers), 1, x0=(g.x0[0], g.x0[1], g.x0[2] + k0 * g.h[2]), h=g.h)
    nodes = (np.arange(nx * ny)[None, :] + nx * ny * (k0 + np.arange(layers + 1))[:, None]).ravel()
    a = W.advection_field(g, cfg.seed_fields)[:, nodes]
    x = W.random_vector(4 * N, cfg.seed_vectors).reshape(4, N)[:, nodes]
    X = W.plate_points(cfg.m_points, cfg.seed_fields)
    z = X[2]
    inside = (z >= sg.x0[2]) & (z <= sg.x0[2] + layers * g.h[2])
    kappa = W.kappa_weights(cfg.m_points, W.plate_volume(), cfg.c_m, cfg.alpha)[inside]
    return sg, a, x, np.ascontiguousarray(X[:, inside]), kappa


def cpu_one_core_main(workload):
    """Child process (OMP_NUM_THREADS=1): the oracle's Jacobian apply on a slab of the
    workload; prints one JSON line."""
    import fsi_workloads as W

    cfg = W.CONFIGS[workload]
    sg, a, x, X, kappa = slab_case(cfg)
    times = [_oracle_jacobian(cfg, sg, a, x, X, kappa) for _ in range(3)]
    dt = sorted(times)[1]
    print(json.dumps({"value": round(4 * sg.num_nodes / dt / 1e9, 6), "unit": "GDOF/s", "cores": 1,
                      "seconds": round(dt, 3), "points": int(X.shape[1]),
                      "sample": f"{sg.n[0]}x{sg.n[1]}x{sg.n[2]}-cell slab through the middle of the grid "
                                f"({sg.num_nodes} nodes, {X.shape[1]} points), median of 3"}))
    return 0


def cpu_baseline(cfg, case, one_core=True):
    """The FP64 oracle's Jacobian apply (dense element matrices, point-by-point DLM) on the full
    workload on all host cores (median of 3), and on one core for a slab of it."""
    import subprocess

    times = [_oracle_jacobian(cfg, cfg.grid, case["a_np"], case["x_np"], case["X_np"], case["kappa_np"])
             for _ in range(3)]
    dt = sorted(times)[1]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = cfg.grid
    out = {"value": round(4 * g.num_nodes / dt / 1e9, 6), "unit": "GDOF/s", "cores": cores,
           "kind": "oracle",
           "sample": f"full FP64 Jacobian apply of the same workload ({g.n[0]}^3 Q1, "
                     f"{cfg.m_points} points), median of 3 = {dt:.2f} s wall; OpenMP element "
                     f"loop + numpy DLM",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if one_core:
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-one-core",
                            "--workload", next(k for k, v in __import__("fsi_workloads").CONFIGS.items()
                                               if v is cfg)],
                           env=env, capture_output=True, text=True, timeout=600)
        if r.returncode == 0 and r.stdout.strip():
            out["one_core"] = json.loads(r.stdout.strip().splitlines()[-1])
        else:
            out["one_core"] = {"error": (r.stderr or "")[-300:]}
    return out


NEWTON_MODES_C5 = ["plain_f64_st2", "plain_mixed_st2", "extrap_mixed_st2", "extrap_mixed_st2_ft", "nn_mixed_st2"]


def newton_block(workload="c5", train_end=20, eval_steps=2, epochs=20, modes=None, eta=5e-3, pc_reuse=True,
                 basis32=True):
    """Newton steps of the rotating-plates channel on the workload's grid (192^3 by default):
    the run is advanced train_end steps (mixed precision, Schur block-triangular preconditioner
    with two velocity steps); the warm-start network is trained on its steps 2..train_end with
    the library's kernels; then each of the next eval_steps steps is solved from the same state
    in every mode, all to the same absolute residual 1e-8 ||R(x_plain)||.  Modes: plain / extrap
    / nn guess, f64 / mixed inner precision, _ft the full Newton tangent (Picard otherwise).
    eta: the Newton forcing (relative tolerance of the linear solves before the last one), the
    same in every mode; 5e-3 gave the shortest steps of 1e-3 ... 2e-2 for plain FP64 and for
    mixed precision at 192^3 and 64^3.  pc_reuse: the preconditioner is built at the first Newton
    iterate of each step and reused (the same Krylov counts as rebuilding it at every iterate at
    192^3 and 64^3, without three of the four setups), in every mode.  basis32: the mixed modes
    keep the Krylov basis in FP32 (their inner solves stop at the FP32 level anyway; the FP64
    modes keep an FP64 basis)."""
    import statistics

    import fsi_workloads as W
    from paper_2601_08266_amd import experiments as ex
    from paper_2601_08266_amd.learned import LearnedWarmStart
    from paper_2601_08266_amd.stepper import ChannelRun

    modes = list(modes or NEWTON_MODES_C5)
    cfg = W.CONFIGS[workload]
    t0 = time.perf_counter()
    run = ChannelRun(cfg, precond="schur_tri", vel_steps=2, eta=eta, pc_reuse=pc_reuse, basis32=basis32)
    run.record_extrap = True
    for _ in range(train_end):
        run.step()
    sim_s = time.perf_counter() - t0
    lw, ks = None, list(range(1, train_end))
    if any(m.startswith("nn") for m in modes):
        lw = LearnedWarmStart(run, seed=0)
        lw.fit_normalisation(run.history, ks)
        lw.build_dataset(run.history, ks)
        lw.train(epochs=epochs, lr=1e-3, seed=0)
    rows = []
    for k in range(train_end, train_end + eval_steps):
        rows.append(ex._solve_modes(run, lw, k, modes))
        run.restore(k)
        run.step()

    def agg(m, key):
        return statistics.mean(r[m][key] for r in rows)

    g = cfg.grid
    out = {"workload": f"{g.n[0]}^3 Q1 channel, {cfg.m_points} points on three rotating plates, "
                       f"dt = {cfg.dt}, backward Euler; trained on steps 2-{train_end}, "
                       f"steps {train_end + 1}-{train_end + eval_steps} solved in every mode",
           "tol": "1e-8 * ||R(x_plain)||, the same absolute threshold in every mode",
           "precond": "Schur block-triangular, 2 velocity steps", "forcing_eta": eta,
           "precond_setup": "once per step" if pc_reuse else "every Newton iterate",
           "krylov_basis_mixed": "f32" if basis32 else "f64", "dof": 4 * g.num_nodes,
           "simulate_s": round(sim_s, 1)}
    if lw is not None:
        out.update({"train_ms": round(lw.train_ms, 1), "epochs": epochs, "train_samples": len(ks),
                    "final_train_loss": round(lw.losses[-1], 4) if lw.losses else None})
    for m in modes:
        out[m] = {"ms_per_step": round(agg(m, "ms_newton") + agg(m, "ms_guess"), 2),
                  "ms_guess": round(agg(m, "ms_guess"), 2),
                  "newton_iters": round(agg(m, "newton"), 2), "krylov_iters": round(agg(m, "krylov"), 1),
                  "phases_ms": [round(statistics.mean(r[m]["phases_ms"][i] for r in rows), 1) for i in range(3)]}
        if m != modes[0]:
            out[m]["max_rel_diff_vs_" + modes[0]] = max(r[m]["rel_diff_vs_" + modes[0]] for r in rows)
        if m.startswith(("nn", "extrap")):
            out[m]["guess_used"] = [str(r[m]["used_guess"]) for r in rows]
    base = out[modes[0]]["ms_per_step"]
    for m in modes[1:]:
        out["speedup_" + m + "_vs_" + modes[0]] = round(base / out[m]["ms_per_step"], 3)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-step block")
    ap.add_argument("--newton-epochs", type=int, default=20)
    ap.add_argument("--newton-eval-steps", type=int, default=2)
    ap.add_argument("--newton-train-end", type=int, default=20,
                    help="steps run before the measured ones (the network trains on 2..this)")
    ap.add_argument("--newton-modes", default=None, help="comma list of Newton modes (default: all)")
    ap.add_argument("--newton-eta", type=float, default=5e-3, help="Newton forcing of the linear solves")
    ap.add_argument("--newton-pc-rebuild", action="store_true",
                    help="rebuild the preconditioner at every Newton iterate (default: once per step)")
    ap.add_argument("--newton-basis64", action="store_true",
                    help="keep an FP64 Krylov basis in the mixed modes too (default: FP32 there)")
    ap.add_argument("--newton-probe", action="store_true",
                    help="also the short 64^3 Newton-step probe with block-Jacobi and Schur modes")
    ap.add_argument("--no-solid", action="store_true", help="skip the solid-block timings")
    ap.add_argument("--no-q2", action="store_true", help="skip the 96^3 Q2 apply row")
    ap.add_argument("--cpu-one-core", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--experiment", default=None,
                    choices=["warmstart", "c5", "netspeed", "c3", "probe", "solid", "solid_steps"],
                    help="run a Newton-step experiment instead of the apply benchmark")
    ap.add_argument("--exp-steps", type=int, default=200)
    ap.add_argument("--exp-modes", default=None,
                    help="comma list: c3 inner precisions (mixed,f64); c5/probe Newton modes "
                         "(plain|extrap|nn _ mixed|f64, suffix _st / _sd for the Schur preconditioner)")
    ap.add_argument("--exp-basis32", action="store_true",
                    help="solid_steps: FP32 inner solves keep their Krylov basis in FP32")
    ap.add_argument("--exp-precond", default="bjacobi", choices=["bjacobi", "schur_diag", "schur_tri"],
                    help="preconditioner of the c3 solve and of the warmstart run's Newton steps")
    ap.add_argument("--exp-restart", type=int, default=50, help="c3 FGMRES restart length")
    ap.add_argument("--exp-vel-steps", type=int, default=0,
                    help="c3 / warmstart: minimal-residual steps on the velocity block of the Schur preconditioner")
    ap.add_argument("--exp-integrator", default="be", choices=["be", "genalpha"],
                    help="time integrator of the probe / warmstart / c5 runs")
    ap.add_argument("--exp-rho-inf", type=float, default=0.5, help="generalized-alpha rho_inf")
    ap.add_argument("--exp-inflow", type=float, default=1.0, help="solid_steps: inflow velocity")
    ap.add_argument("--exp-gravity", type=float, default=0.0,
                    help="solid_steps: body force -g e_z per unit mass on the solid (0: none)")
    ap.add_argument("--exp-c-stiff", type=float, default=0.0,
                    help="solid / solid_steps: stiffness share of the preconditioners' per-point kappa")
    ap.add_argument("--exp-train-end", type=int, default=100)
    ap.add_argument("--exp-epochs", type=int, default=20)
    ap.add_argument("--exp-stride", type=int, default=1)
    ap.add_argument("--exp-save", default=None)
    ap.add_argument("--exp-load", default=None)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (for counter calibration)")
    args = ap.parse_args(argv)
    if args.cpu_one_core:
        return cpu_one_core_main(args.workload)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(how the apply would shard is described in the design notes)", file=sys.stderr)
        return 2

    import torch

    import fsi_workloads as W
    import paper_2601_08266_amd as fsi

    if args.experiment:
        return run_experiment(args)
    dev = torch.device("cuda:0")
    cfg = W.CONFIGS[args.workload]
    g = cfg.grid
    case64 = build_problem(cfg, torch.float64, dev)
    case32 = build_problem(cfg, torch.float32, dev)
    N = case64["N"]

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ms64, wall64, kern = time_applies(fsi, torch, case64, args.steps, args.warmup, profile=True)
    ms32, wall32, kern32 = time_applies(fsi, torch, case32, args.steps, args.warmup, profile=True)
    # the point-by-point DLM path (B, kappa, B^T corner sums in the node gather) instead of the
    # per-cell blocks folded into the cell kernel
    pw = dict(case64)
    p0 = case64["prob"]
    pw["prob"] = fsi.Problem(g, p0.prm, p0.a, p0.tables, p0.kappa, s=p0.s)
    pw["ws"] = torch.empty(pw["prob"].workspace_bytes(), dtype=torch.uint8, device=dev)
    ms_pw, _, kern_pw = time_applies(fsi, torch, pw, args.steps, args.warmup, profile=False)
    del pw
    blocks = {"f64": time_blocks(fsi, torch, case64, args.steps, args.warmup),
              "f32": time_blocks(fsi, torch, case32, args.steps, args.warmup)} if g.order == 1 else None

    resident = 4 * N * 8 * 4 < 256e6
    cold64 = time_cold(torch, case64) if resident else None
    gdofs64 = 4 * N / (ms64 * 1e-3) / 1e9
    gdofs32 = 4 * N / (ms32 * 1e-3) / 1e9
    cell_ms, launches = kern.get("vms_q1_cells", (0.0, 0))
    flops = q1_cell_flops() * g.num_cells + dlm_cell_flops() * case64["tab"].n_occ
    achieved_tf = flops / (cell_ms * 1e-3) / 1e12 if cell_ms > 0 else 0.0
    hbm_bytes = 96 * N          # x in, y out, a, s: 4*8 + 4*8 + 3*8 + 8 per node (FP64)
    hbm_gbs = hbm_bytes / (cell_ms * 1e-3) / 1e9 if cell_ms > 0 else 0.0

    out = {
        "metric": "GDOF/s of VMS+DLM Jacobian apply",
        "value": round(gdofs64, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{cfg.name}: {g.n[0]}x{g.n[1]}x{g.n[2]} Q{g.order}-Q{g.order} VMS+DLM "
                        f"Jacobian apply, {cfg.m_points} solid points ({cfg.solid})",
            "dof": 4 * N, "cells": g.num_cells, "points": cfg.m_points,
            "nu": cfg.nu, "dt": cfg.dt, "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu", "kernel": "vms_q1_cells<double>",
            "achieved": round(achieved_tf, 3), "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved_tf / PEAK_FP64_VALU_TFLOPS, 4),
            "traffic": cell_traffic_bytes(args.workload), "traffic_unit": "bytes/launch",
            "flops_per_launch": flops, "kernel_ms_avg": round(cell_ms, 6),
            "launches": launches,
            "hbm_algorithmic_GBs": round(hbm_gbs, 1),
            "hbm_frac": round(hbm_gbs / PEAK_HBM_GBS, 4),
            # vectors that fit the 256 MB Infinity Cache stay there between back-to-back applies
            # (then extra.cold_cache_* times applies after a 512 MiB overwrite)
            "infinity_cache_resident": resident,
        },
        "extra": {
            "fp32_gdofs": round(gdofs32, 4), "fp32_ms_per_step": round(ms32, 6),
            "host_wall_ms_per_step_f64": round(wall64, 6),
            "kernels_f64_ms": {k: round(v[0], 6) for k, v in kern.items()},
            "kernels_f32_ms": {k: round(v[0], 6) for k, v in kern32.items()},
            # the DLM block applied point by point (B, kappa, B^T) instead of through the per-cell
            # blocks, which are built once per point set (dlm_gram) and reused by every apply
            "pointwise_dlm_gdofs_f64": round(4 * N / (ms_pw * 1e-3) / 1e9, 4),
            "pointwise_dlm_ms_per_step_f64": round(ms_pw, 6),
            # the preconditioner's products with the velocity block F and the pressure-gradient
            # block G (velocity rows of J on (x_u, 0) and on (0, x_p))
            "block_products": blocks,
            "locate_ms": round(case64["locate_ms"], 3),
            "dlm_gram_ms": round(case64["gram_ms"], 3),
            "dlm_gram_in_applies": round(case64["gram_ms"] / ms64, 3),
            "n_occupied_cells": case64["tab"].n_occ,
            **time_dlm(fsi, torch, case64),
        },
    }
    if cold64 is not None:
        out["extra"]["cold_cache_ms_per_apply_f64"] = round(cold64, 6)
        out["extra"]["cold_cache_gdofs_f64"] = round(4 * N / (cold64 * 1e-3) / 1e9, 4)
    # free the apply benchmark's buffers before the Newton runs
    del case32
    torch.cuda.synchronize()
    if args.workload != "c1" and not args.no_solid:
        out["solid_block"] = time_solid(fsi, torch, cfg, cpu=not args.no_cpu_baseline)
    if not args.no_q2:
        out["q2_apply"] = time_q2_apply(fsi, torch)
    if not args.no_newton and args.workload in ("c2", "c5"):
        out["newton_step"] = newton_block("c5" if args.workload == "c5" else "c4",
                                          train_end=args.newton_train_end, epochs=args.newton_epochs,
                                          eval_steps=args.newton_eval_steps,
                                          modes=args.newton_modes.split(",") if args.newton_modes else None,
                                          eta=args.newton_eta, pc_reuse=not args.newton_pc_rebuild,
                                          basis32=not args.newton_basis64)
    if args.newton_probe:
        out["newton_probe_64cube"] = newton_step_probe()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, case64)
    print(json.dumps(out))
    return 0


def run_experiment(args):
    import torch

    from paper_2601_08266_amd import experiments as ex
    from paper_2601_08266_amd import warmstart as wsn

    if args.experiment == "netspeed":
        dims = (65, 65, 65)
        net = wsn.WarmStartNet(dims)
        V = 65 ** 3
        x = torch.zeros(V * 32, dtype=torch.int16, device="cuda")
        t = torch.zeros(V * 32, dtype=torch.float32, device="cuda")
        for _ in range(3):
            net.forward(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            net.forward(x)
        torch.cuda.synchronize()
        fwd = (time.perf_counter() - t0) / 10 * 1e3
        t0 = time.perf_counter()
        for _ in range(5):
            net.train_sample(x, t, want_loss=False)
        torch.cuda.synchronize()
        trn = (time.perf_counter() - t0) / 5 * 1e3
        flops = 2.0 * 27 * V * sum(l.cin * l.cout for l in net.layers)
        print(json.dumps({"experiment": "netspeed", "lattice": "65^3", "params": net.n_params,
                          "forward_ms": round(fwd, 3), "train_sample_ms": round(trn, 3),
                          "forward_padded_TFLOPs": round(flops / fwd / 1e9, 2)}))
        return 0
    modes = args.exp_modes.split(",") if args.exp_modes else None
    if args.experiment == "c3":
        print(json.dumps({"experiment": "solve_c3",
                          **ex.solve_c3(max_iters=args.exp_steps, modes=tuple(modes or ("mixed", "f64")),
                                        precond=args.exp_precond, restart=args.exp_restart,
                                        vel_steps=args.exp_vel_steps)}))
        return 0
    if args.experiment == "solid":
        print(json.dumps({"experiment": "solid_solve",
                          **ex.solid_solve(max_iters=args.exp_steps, precond=args.exp_precond,
                                           restart=args.exp_restart, vel_steps=args.exp_vel_steps,
                                           workload=args.workload, c_stiff=args.exp_c_stiff)}))
        return 0
    if args.experiment == "solid_steps":
        print(json.dumps({"experiment": "solid_steps",
                          **ex.solid_steps(steps=args.exp_steps, precond=args.exp_precond,
                                           vel_steps=args.exp_vel_steps, workload=args.workload,
                                           c_stiff=args.exp_c_stiff, integrator=args.exp_integrator,
                                           rho_inf=args.exp_rho_inf, inflow=args.exp_inflow,
                                           gravity=(0.0, 0.0, -args.exp_gravity) if args.exp_gravity else None,
                                           basis32=args.exp_basis32)}))
        return 0
    if args.experiment == "probe":
        print(json.dumps({"experiment": "newton_probe",
                          **newton_step_probe(modes=modes, integrator=args.exp_integrator,
                                              rho_inf=args.exp_rho_inf)}))
        return 0
    if args.experiment == "warmstart":
        # --workload c5: the 192^3 run trained on its own first steps
        key = "c5" if args.workload == "c5" else "c4"
        summary, lw = ex.warmstart(key, steps=args.exp_steps, train_end=args.exp_train_end,
                                   epochs=args.exp_epochs, eval_stride=args.exp_stride,
                                   save_path=args.exp_save, precond=args.exp_precond,
                                   integrator=args.exp_integrator, rho_inf=args.exp_rho_inf,
                                   vel_steps=args.exp_vel_steps)
        print(json.dumps({"experiment": "warmstart_" + key, **summary}))
        return 0
    summary = ex.large_c5(state_path=args.exp_load, modes=modes, integrator=args.exp_integrator,
                          rho_inf=args.exp_rho_inf)
    print(json.dumps({"experiment": "large_c5", **summary}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
