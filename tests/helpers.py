"""Shared test helpers: seeded problem setup and the norm-wise parity measure."""
import numpy as np

import fsi_workloads as W


def field_rel_err(got, ref, nfields):
    """max over fields of ||got_f - ref_f||_2 / ||ref_f||_2 (flat arrays, field-major)."""
    got = np.asarray(got, dtype=np.float64).reshape(nfields, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(nfields, -1)
    errs = []
    for f in range(nfields):
        den = np.linalg.norm(ref[f])
        num = np.linalg.norm(got[f] - ref[f])
        errs.append(num / den if den > 0 else num)
    return max(errs)


def rows_field_rel_err(got, ref, rows, n):
    """Sampled rows (flat indices f*n + node) grouped by field f = row // n: the maximum over
    fields of ||got_f - ref_f|| / ||ref_f|| (the per-field measure of the full-grid checks)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fields = np.asarray(rows) // n
    errs = []
    for f in np.unique(fields):
        sel = fields == f
        den = np.linalg.norm(ref[sel])
        num = np.linalg.norm(got[sel] - ref[sel])
        errs.append(num / den if den > 0 else num)
    return max(errs)


def points_for(cfg):
    if cfg.solid == "sphere":
        X = W.sphere_points()
        vol = W.sphere_volume()
    else:
        X = W.plate_points(cfg.m_points, cfg.seed_fields)
        vol = W.plate_volume()
    kappa = W.kappa_weights(X.shape[1], vol, cfg.c_m, cfg.alpha)
    return X, kappa


def sample_rows(grid, n, seed=0, brick=(8, 8, 4)):
    """Random flat row indices (f*N + node) plus rows on brick faces and the domain boundary."""
    rng = np.random.default_rng(seed)
    N = grid.num_nodes
    nx, ny, nz = grid.nodes_per_axis
    rows = list(rng.choice(4 * N, n, replace=False))
    p = grid.order
    for k in range(min(nz, 3 * brick[2] * p + 2)):
        for j in (0, brick[1] * p, ny - 1):
            for i in (0, brick[0] * p, nx - 1):
                if j < ny and i < nx:
                    node = i + nx * (j + ny * k)
                    rows.extend(f * N + node for f in range(4))
    return np.unique(np.array(rows, dtype=np.int64))
