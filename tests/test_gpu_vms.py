"""GPU parity of fsi_vms_apply against the FP64 oracle (section 2.1 operator).

Bar: max over fields of the relative 2-norm error <= 1e-12 (FP64) and
<= 1e-5 (FP32, inputs rounded to FP32 before both sides see them).
"""
import numpy as np
import pytest

import fsi_workloads as W
from oracle import dlm as odlm
from oracle import vms as ovms

from helpers import field_rel_err, points_for, rows_field_rel_err, sample_rows

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _torch():
    import torch
    return torch


def setup_case(cfg, dtype, with_s=True, with_mask=False, grid=None):
    torch = _torch()
    import paper_2601_08266_amd as fsi
    g = grid or cfg.grid
    N = g.num_nodes
    a = W.advection_field(g, cfg.seed_fields)
    x = W.random_vector(4 * N, cfg.seed_vectors)
    s = None
    if with_s:
        X, _ = points_for(cfg)
        cell, _ = odlm.locate(g, X)
        s = odlm.s_field(g, cell, cfg.s_max)
    mask = W.channel_dirichlet_mask(g) if with_mask else None
    npdt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    # both sides see the same (possibly FP32-rounded) values
    a = a.astype(npdt).astype(np.float64)
    x = x.astype(npdt).astype(np.float64)
    if s is not None:
        s = s.astype(npdt).astype(np.float64)
    dev = "cuda"
    t = dict(
        a=torch.tensor(a.ravel(), dtype=tdt, device=dev),
        x=torch.tensor(x, dtype=tdt, device=dev),
        s=None if s is None else torch.tensor(s, dtype=tdt, device=dev),
        mask=None if mask is None else torch.tensor(W.mask_to_bits(mask).view(np.int32), device=dev),
    )
    prm_o = ovms.params_array(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    prm_g = fsi.make_params(cfg.nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    return g, a, x, s, mask, t, prm_o, prm_g


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("with_s,with_mask", [(False, False), (True, False), (True, True)])
def test_vms_q1_c1_full(dtype, with_s, with_mask):
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    g, a, x, s, mask, t, prm_o, prm_g = setup_case(cfg, dtype, with_s, with_mask)
    y = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=t["s"], mask=t["mask"]).cpu().numpy()
    ref = ovms.apply(g, prm_o, a, x, s=s, mask=mask)
    err = field_rel_err(y, ref, 4)
    print(f"c1 {dtype} s={with_s} mask={with_mask}: rel err {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(11, 9, 6), (1, 1, 1), (17, 3, 9), (8, 8, 4)])
def test_vms_q1_ragged_grids(dtype, n):
    """Several bricks with ragged tails, a single cell, and exactly one brick."""
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    grid = W.Grid(n, 1, x0=(0.1, -0.2, 0.05), h=(0.07, 0.09, 0.11))
    g, a, x, s, mask, t, prm_o, prm_g = setup_case(cfg, dtype, with_s=False, with_mask=True,
                                                   grid=grid)
    rng = np.random.default_rng(sum(n))
    s = rng.uniform(1.0, 100.0, size=grid.num_nodes)
    if dtype == "f32":
        s = s.astype(np.float32).astype(np.float64)
    torch = _torch()
    ts = torch.tensor(s, dtype=t["x"].dtype, device="cuda")
    y = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=ts, mask=t["mask"]).cpu().numpy()
    ref = ovms.apply(g, prm_o, a, x, s=s, mask=mask)
    err = field_rel_err(y, ref, 4)
    print(f"grid {n} {dtype}: rel err {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vms_q1_weak_viscous_form(dtype):
    """The operator without the strong viscous term in the stabilisation residuals
    (visc_strong = 0, the kernel's other compiled variant) on a ragged multi-brick grid with s
    and Dirichlet rows."""
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c1"]
    grid = W.Grid((11, 9, 6), 1, x0=(0.1, -0.2, 0.05), h=(0.07, 0.09, 0.11))
    g, a, x, s, mask, t, prm_o, _ = setup_case(cfg, dtype, with_s=False, with_mask=True, grid=grid)
    rng = np.random.default_rng(23)
    s = rng.uniform(1.0, 100.0, size=grid.num_nodes)
    if dtype == "f32":
        s = s.astype(np.float32).astype(np.float64)
    torch = _torch()
    ts = torch.tensor(s, dtype=t["x"].dtype, device="cuda")
    # a viscosity at which the strong viscous term matters (nu / h^2 comparable to c_m)
    nu = 0.5
    prm_o = ovms.params_array(nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I)
    prm_w = fsi.make_params(nu, cfg.c_m, cfg.dt, cfg.C_T, cfg.C_I, visc_strong=False)
    y = fsi.vms_apply(g, prm_w, t["a"], t["x"], s=ts, mask=t["mask"]).cpu().numpy()
    ref = ovms.apply(g, prm_o, a, x, s=s, mask=mask, visc_strong=False)
    err = field_rel_err(y, ref, 4)
    # not vacuous: the strong form differs by far more than the bar
    ref_s = ovms.apply(g, prm_o, a, x, s=s, mask=mask, visc_strong=True)
    diff = field_rel_err(ref_s, ref, 4)
    print(f"weak viscous form {dtype}: rel err {err:.3e} (strong vs weak {diff:.2e})")
    assert err <= TOL[dtype]
    assert diff > 100 * TOL["f32"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vms_q1_c2_sampled_rows(dtype):
    """Full 64^3 size, bench launch configuration; oracle recomputes sampled rows."""
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c2"]
    g, a, x, s, mask, t, prm_o, prm_g = setup_case(cfg, dtype, with_s=True, with_mask=False)
    y = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=t["s"]).cpu().numpy()
    rows = sample_rows(g, 3000, seed=1)
    ref = ovms.apply_rows(g, prm_o, a, x, rows, s=s)
    err = rows_field_rel_err(y[rows], ref, rows, g.num_nodes)
    print(f"c2 {dtype} sampled rows: rel err {err:.3e}")
    assert err <= TOL[dtype]
    # bitwise determinism over repeated applies
    y2 = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=t["s"]).cpu().numpy()
    assert np.array_equal(y.view(np.uint8), y2.view(np.uint8))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [(3, 2, 2), (5, 4, 6), (4, 4, 4), (1, 1, 1), (9, 3, 5)])
def test_vms_q2_small_grids(dtype, n):
    """Q2: one brick, several bricks with ragged tails, a single cell; s with jumps."""
    import paper_2601_08266_amd as fsi
    torch = _torch()
    cfg = W.CONFIGS["c1"]
    grid = W.Grid(n, 2, x0=(0.1, -0.2, 0.05), h=(0.13, 0.09, 0.11))
    g, a, x, s, mask, t, prm_o, prm_g = setup_case(cfg, dtype, with_s=False, with_mask=True,
                                                   grid=grid)
    rng = np.random.default_rng(sum(n) + 7)
    s = np.where(rng.uniform(size=grid.num_nodes) < 0.3, 100.0, 1.0)
    ts = torch.tensor(s, dtype=t["x"].dtype, device="cuda")
    y = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=ts, mask=t["mask"]).cpu().numpy()
    ref = ovms.apply(g, prm_o, a, x, s=s, mask=mask)
    err = field_rel_err(y, ref, 4)
    print(f"q2 grid {n} {dtype}: rel err {err:.3e}")
    assert err <= TOL[dtype]
    y2 = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=ts, mask=t["mask"]).cpu().numpy()
    assert np.array_equal(y, y2)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_vms_q2_c3_sampled_rows(dtype):
    """96^3 Q2 (28.8M DOF): sampled rows recomputed by the oracle, brick faces included."""
    import paper_2601_08266_amd as fsi
    cfg = W.CONFIGS["c3"]
    g, a, x, s, mask, t, prm_o, prm_g = setup_case(cfg, dtype, with_s=True, with_mask=True)
    y = fsi.vms_apply(g, prm_g, t["a"], t["x"], s=t["s"], mask=t["mask"]).cpu().numpy()
    rows = sample_rows(g, 400, seed=3, brick=(4, 4, 4))
    ref = ovms.apply_rows(g, prm_o, a, x, rows, s=s, mask=mask)
    err = rows_field_rel_err(y[rows], ref, rows, g.num_nodes)
    print(f"c3 {dtype} sampled rows: rel err {err:.3e}")
    assert err <= TOL[dtype]
