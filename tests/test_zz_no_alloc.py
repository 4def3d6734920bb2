"""fsi_dlm_BT_noalloc (the B^T entry point without a workspace, for callers that cannot
allocate) against fsi_dlm_BT through the C ABI: the same kernels, so the results must be
bitwise equal; two calls in a row, the second on a smaller point set, in FP64 and FP32 and on a
Q2 grid; sizes beyond the library's scratch array are rejected before any device work."""
import ctypes

import numpy as np
import pytest

import fsi_workloads as W

from helpers import points_for


def _grid(g):
    import paper_2601_08266_amd as fsi
    return fsi.grid_from(g)


def _bt_pair(g, X, kappa, dtype, seed):
    """(y from fsi_dlm_BT, y from fsi_dlm_BT_noalloc) for the same lam, kappa and y0."""
    import torch
    import paper_2601_08266_amd as fsi
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tab = fsi.dlm_locate(g, torch.tensor(np.ascontiguousarray(X).ravel(), dtype=torch.float64, device="cuda"),
                         dtype=tdt)
    N, m = g.num_nodes, X.shape[1]
    rng = np.random.default_rng(seed)
    lam = torch.tensor(rng.standard_normal(3 * m), dtype=tdt, device="cuda")
    kap = torch.tensor(kappa, dtype=tdt, device="cuda")
    y0 = torch.tensor(rng.standard_normal(3 * N), dtype=tdt, device="cuda")
    gs = _grid(g)
    code = fsi.dtype_code(tdt)
    ws = torch.empty(int(lib.fsi_dlm_BT_workspace(ctypes.byref(gs), tab.n_occ, code)), dtype=torch.uint8,
                     device="cuda")
    y_ref = y0.clone()
    rc = lib.fsi_dlm_BT(ctypes.byref(gs), code, m, tab.cell.data_ptr(), tab.xi.data_ptr(), tab.perm.data_ptr(),
                        tab.occ_cell.data_ptr(), tab.occ_start.data_ptr(), tab.occ_index.data_ptr(), tab.n_occ,
                        lam.data_ptr(), kap.data_ptr(), y_ref.data_ptr(), ws.data_ptr(), ws.numel(), None)
    assert rc == 0, lib.fsi_last_error()
    y = y0.clone()
    rc = lib.fsi_dlm_BT_noalloc(ctypes.byref(gs), code, m, tab.perm.data_ptr(), tab.xi.data_ptr(),
                                tab.occ_cell.data_ptr(), tab.occ_start.data_ptr(), tab.occ_index.data_ptr(),
                                tab.n_occ, lam.data_ptr(), kap.data_ptr(), y.data_ptr(), None)
    assert rc == 0, lib.fsi_last_error()
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y.cpu().numpy(), tab.n_occ


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_BT_matches_BT_on_two_calls(dtype):
    cases = []
    for key in ("c5", "c1"):          # the second call is on a smaller input
        cfg = W.CONFIGS[key]
        X, kappa = points_for(cfg)
        cases.append((cfg.grid, X, kappa))
    g = W.Grid((9, 7, 8), 2)
    X = np.random.default_rng(1).uniform(0.0, 1.0, (3, 4000))
    cases.append((g, X, np.random.default_rng(2).uniform(0.5, 2.0, 4000)))
    for i, (g, X, kappa) in enumerate(cases):
        y_ref, y, n_occ = _bt_pair(g, X, kappa, dtype, seed=10 + i)
        print(f"noalloc {dtype} call {i}: grid {g.n} Q{g.order}, {X.shape[1]} points, {n_occ} occupied cells, "
              f"equal {np.array_equal(y_ref, y)}", flush=True)
        assert np.array_equal(y_ref, y)


def test_noalloc_rejects_sizes_beyond_the_scratch_array():
    """Host-side check (no device work): more occupied cells than the array holds."""
    import paper_2601_08266_amd._lib as L
    lib = L.lib()
    cap = int(lib.fsi_dlm_BT_noalloc_max_bytes())
    assert cap == 32 << 20
    g = _grid(W.Grid((400, 400, 400), 1))
    n_occ = cap // (8 * 3 * 8) + 1                 # FP64 Q1: 192 B of corner sums per cell
    rc = lib.fsi_dlm_BT_noalloc(ctypes.byref(g), 0, n_occ, None, None, None, None, None, n_occ, None,
                                None, None, None)
    assert rc == L.FSI_ERR_WORKSPACE
    assert b"scratch" in lib.fsi_last_error()
    # at the limit it passes the size check and stops at the missing pointers
    rc = lib.fsi_dlm_BT_noalloc(ctypes.byref(g), 0, n_occ - 1, None, None, None, None, None, n_occ - 1, None,
                                None, None, None)
    assert rc == L.FSI_ERR_ARG
