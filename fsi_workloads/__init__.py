"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module only *synthesises inputs*: grid geometry, a smooth advection field,
solid point clouds, per-point penalty weights, random vectors and Dirichlet
masks. It contains none of the method's arithmetic (no shape functions, no
stabilisation parameters, no point location), so both the CPU oracle and the
HIP path can consume the very same arrays without sharing any computation.

Workload recipe (stated once here, repeated in the design notes):

* Domain [0,1]^3, uniform hex cells, equal-order Q1 or Q2 for (u, v, w, p).
* Advection field a = sum_{m=1..3} A_m sin(2 pi k_m . x + phi_m) with integer
  wave vectors k_m in {-2..2}^3 \\ {0}, amplitudes A_m orthogonal to k_m (so a
  is pointwise divergence free), phases uniform in [0, 2 pi), rescaled so the
  RMS of |a| over the nodes is 1 (the paper's flows have |v| ~ 1 in these
  units; section 2.1 evaluates tau with the fluid velocity).
* Solids: a sphere of radius 0.25 (4 radial shells x 128 Fibonacci points) for
  the 8^3 case, and three thin curved plates (a hemispherical cup of radius
  0.3 and thickness 0.02 cut into three 116-degree sectors) for the larger
  cases; this stands in for the immersed thin leaflets of section 4.5.
* Per-point weight kappa_B = alpha * c_m * V_B with alpha = 100 and
  V_B = solid volume / M (stand-in for the solid block of the reduced system,
  section 2.4).
* Solid mesh (for the hyperelastic solid block): the same three plates meshed by
  structured trilinear hexahedra, two node layers through the thickness, polar
  angle 10-90 degrees; its nodes are the solid points.  Solid state: a finite
  rigid rotation plus a small smooth displacement field (seeded).
* Seeds: configuration k uses 1000 + k for fields and geometry and 2000 + k for
  random vectors.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Grid", "Config", "CONFIGS", "get_config", "node_coords", "advection_field",
    "sphere_points", "plate_points", "plate_volume", "sphere_volume",
    "kappa_weights", "random_vector", "channel_dirichlet_mask", "mask_to_bits",
    "rotating_plate_points", "smooth_fourier_field", "channel_inflow_pattern", "channel_inflow_value",
]


@dataclasses.dataclass(frozen=True)
class Grid:
    """Structured hex grid: n cells per axis, Lagrange order, origin, cell size."""

    n: tuple
    order: int = 1
    x0: tuple = (0.0, 0.0, 0.0)
    h: tuple = None

    def __post_init__(self):
        if self.h is None:
            object.__setattr__(self, "h", tuple(1.0 / float(v) for v in self.n))

    @property
    def nodes_per_axis(self):
        return tuple(self.order * v + 1 for v in self.n)

    @property
    def num_nodes(self):
        a, b, c = self.nodes_per_axis
        return a * b * c

    @property
    def num_cells(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def ndof(self):
        return 4 * self.num_nodes


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    grid: Grid
    m_points: int
    solid: str            # "sphere" | "plates"
    seed_fields: int
    seed_vectors: int
    nu: float = 1.0e-2
    dt: float = 1.0e-3
    C_T: float = 4.0
    C_I: float = 36.0
    s_max: float = 100.0
    alpha: float = 100.0

    @property
    def c_m(self):
        return 1.0 / self.dt


CONFIGS = {
    "c1": Config("c1_8cube_q1", Grid((8, 8, 8), 1), 512, "sphere", 1001, 2001),
    "c2": Config("c2_64cube_q1", Grid((64, 64, 64), 1), 200_000, "plates", 1002, 2002),
    "c3": Config("c3_96cube_q2", Grid((96, 96, 96), 2), 500_000, "plates", 1003, 2003),
    "c4": Config("c4_64cube_q1_rotating", Grid((64, 64, 64), 1), 200_000, "plates", 1004, 2004),
    "c5": Config("c5_192cube_q1", Grid((192, 192, 192), 1), 2_000_000, "plates", 1005, 2005),
}


def get_config(key: str) -> Config:
    return CONFIGS[key]


def node_coords(grid: Grid):
    """Node coordinates as three flat arrays, node id = i + Nx*(j + Ny*k)."""
    nx, ny, nz = grid.nodes_per_axis
    p = grid.order
    xs = grid.x0[0] + np.arange(nx) * (grid.h[0] / p)
    ys = grid.x0[1] + np.arange(ny) * (grid.h[1] / p)
    zs = grid.x0[2] + np.arange(nz) * (grid.h[2] / p)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def advection_field(grid: Grid, seed: int, n_modes: int = 3, rms: float = 1.0):
    """Divergence-free sum of random Fourier modes sampled at the nodes, SoA [3][N]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y, Z = node_coords(grid)
    a = np.zeros((3, X.size))
    for _ in range(n_modes):
        while True:
            k = rng.integers(-2, 3, size=3)
            if np.any(k != 0):
                break
        k = k.astype(np.float64)
        v = rng.standard_normal(3)
        v -= (v @ k) / (k @ k) * k          # amplitude orthogonal to k
        phi = rng.uniform(0.0, 2.0 * math.pi)
        arg = 2.0 * math.pi * (k[0] * X + k[1] * Y + k[2] * Z) + phi
        a += np.outer(v, np.sin(arg))
    scale = rms / math.sqrt(np.mean(np.sum(a * a, axis=0)))
    return np.ascontiguousarray(a * scale)


def smooth_fourier_field(grid: Grid, seed: int, channels: int = 4, n_modes: int = 3):
    """Smooth seeded field with `channels` components (right-hand sides)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y, Z = node_coords(grid)
    out = np.zeros((channels, X.size))
    for c in range(channels):
        for _ in range(n_modes):
            k = rng.integers(0, 3, size=3).astype(np.float64)
            amp = rng.standard_normal()
            phi = rng.uniform(0.0, 2.0 * math.pi, size=3)
            out[c] += amp * (np.cos(math.pi * k[0] * X + phi[0])
                             * np.cos(math.pi * k[1] * Y + phi[1])
                             * np.cos(math.pi * k[2] * Z + phi[2]))
    return out


def sphere_volume(radius: float = 0.25) -> float:
    return 4.0 / 3.0 * math.pi * radius ** 3


def sphere_points(n_layers: int = 4, per_layer: int = 128, radius: float = 0.25,
                  center=(0.5, 0.5, 0.5)):
    """Radial shells r = radius*(l+1)/n_layers, Fibonacci points on each shell. [3][M]."""
    golden = math.pi * (3.0 - math.sqrt(5.0))
    i = np.arange(per_layer, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / per_layer
    rad = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = golden * i
    unit = np.stack([rad * np.cos(th), rad * np.sin(th), z])
    pts = []
    for layer in range(n_layers):
        r = radius * (layer + 1) / n_layers
        pts.append(np.asarray(center)[:, None] + r * unit)
    return np.ascontiguousarray(np.concatenate(pts, axis=1))


PLATE_R = (0.29, 0.31)
PLATE_MARGIN_DEG = 2.0


def plate_volume() -> float:
    """Total volume of the three cup sectors (thickness 0.02, radius 0.3)."""
    r0, r1 = PLATE_R
    dphi = math.radians(120.0 - 2.0 * PLATE_MARGIN_DEG)
    return 3.0 * (r1 ** 3 - r0 ** 3) / 3.0 * 1.0 * dphi


def plate_points(m: int, seed: int, center=(0.5, 0.5, 0.5), rotation_deg: float = 0.0):
    """Three thin cup-shaped plates (hemispherical cup cut into 120-degree sectors). [3][M].

    Plate k: X = c + r (cos t, sin t cos f, sin t sin f) with r ~ U[0.29,0.31],
    cos t ~ U[0,1], f ~ U[120k+2, 120(k+1)-2] degrees. The rim lies in the plane
    x = 0.5. An optional rigid rotation about the x axis through c is applied.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = [m // 3 + (1 if k < m % 3 else 0) for k in range(3)]
    out = []
    for k, cnt in enumerate(counts):
        r = rng.uniform(PLATE_R[0], PLATE_R[1], size=cnt)
        ct = rng.uniform(0.0, 1.0, size=cnt)
        st = np.sqrt(1.0 - ct * ct)
        lo = math.radians(120.0 * k + PLATE_MARGIN_DEG)
        hi = math.radians(120.0 * (k + 1) - PLATE_MARGIN_DEG)
        f = rng.uniform(lo, hi, size=cnt)
        out.append(np.stack([r * ct, r * st * np.cos(f), r * st * np.sin(f)]))
    rel = np.concatenate(out, axis=1)
    if rotation_deg != 0.0:
        th = math.radians(rotation_deg)
        c, s = math.cos(th), math.sin(th)
        y = c * rel[1] - s * rel[2]
        z = s * rel[1] + c * rel[2]
        rel = np.stack([rel[0], y, z])
    return np.ascontiguousarray(np.asarray(center)[:, None] + rel)


def rotating_plate_points(m: int, seed: int, t: float, period: float = 0.8,
                          amp_deg: float = 20.0, center=(0.5, 0.5, 0.5)):
    """Plates rotated rigidly about the x axis by theta(t) = amp sin(2 pi t / period).

    Returns (X [3][M], g [3][M]) with g the rigid-body velocity theta' e_x x (X - c).
    """
    th = amp_deg * math.sin(2.0 * math.pi * t / period)
    X = plate_points(m, seed, center=center, rotation_deg=th)
    thdot = math.radians(amp_deg) * (2.0 * math.pi / period) * math.cos(2.0 * math.pi * t / period)
    rel = X - np.asarray(center)[:, None]
    g = np.stack([np.zeros_like(rel[0]), -thdot * rel[2], thdot * rel[1]])
    return X, np.ascontiguousarray(g)


PLATE_T_DEG = (10.0, 90.0)


# Solid material of the hyperelastic block: shear modulus C0 with the bulk-to-shear
# ratio kappa_s = C0 / 10 of the paper's oscillating-leaflet case (section 4.3), the
# falling sphere's density ratio rho_s0 / rho_f = 1.5 (section 4.4), and mu_f = nu rho_f
# of the fluid settings (nu = 1e-2).
SOLID_MATERIAL = dict(C0=1.0e5, kappa_s=1.0e4, rho_s0=1.5, rho_f=1.0, mu_f=0.01)


def plate_solid_mesh(n_t: int, n_f: int, n_r: int = 2, center=(0.5, 0.5, 0.5),
                     rotation_deg: float = 0.0):
    """Structured trilinear-hex mesh of the three plates; its nodes are the solid points.

    Plate k spans r in [0.29, 0.31] (n_r nodes), polar angle t in [10, 90] degrees (n_t
    nodes; the pole is left out so no element degenerates) and azimuth f in
    [120k + 2, 120(k+1) - 2] degrees (n_f nodes), all uniformly spaced:
    X = c + r (cos t, sin t cos f, sin t sin f), then an optional rigid rotation about the
    x axis through c.  Node (k, i_r, j_t, l_f) has index ((k n_f + l_f) n_t + j_t) n_r + i_r.
    Element corner a + 2b + 4c sits at offsets (a, b, c) along (r, t, f), a right-handed
    order (positive volume).

    Returns (X [3][M] float64, conn [E][8] int32).
    """
    assert n_r >= 2 and n_t >= 2 and n_f >= 2
    out, conns = [], []
    r = np.linspace(PLATE_R[0], PLATE_R[1], n_r)
    t = np.radians(np.linspace(PLATE_T_DEG[0], PLATE_T_DEG[1], n_t))
    for k in range(3):
        f = np.radians(np.linspace(120.0 * k + PLATE_MARGIN_DEG, 120.0 * (k + 1) - PLATE_MARGIN_DEG, n_f))
        F, T, R = np.meshgrid(f, t, r, indexing="ij")          # [n_f][n_t][n_r]
        out.append(np.stack([R * np.cos(T), R * np.sin(T) * np.cos(F), R * np.sin(T) * np.sin(F)]).reshape(3, -1))
        base = k * n_f * n_t * n_r
        lf, jt, ir = np.meshgrid(np.arange(n_f - 1), np.arange(n_t - 1), np.arange(n_r - 1), indexing="ij")
        lf, jt, ir = lf.ravel(), jt.ravel(), ir.ravel()
        corners = []
        for cidx in range(8):
            a, b, c = cidx & 1, (cidx >> 1) & 1, cidx >> 2
            corners.append(base + ((lf + c) * n_t + (jt + b)) * n_r + (ir + a))
        conns.append(np.stack(corners, axis=1))
    rel = np.concatenate(out, axis=1)
    if rotation_deg != 0.0:
        th = math.radians(rotation_deg)
        cs, sn = math.cos(th), math.sin(th)
        rel = np.stack([rel[0], cs * rel[1] - sn * rel[2], sn * rel[1] + cs * rel[2]])
    X = np.ascontiguousarray(np.asarray(center, dtype=np.float64)[:, None] + rel)
    return X, np.ascontiguousarray(np.concatenate(conns).astype(np.int32))


def solid_mesh_size(m_target: int):
    """(n_t, n_f) of a two-layer plate mesh with about m_target nodes (3 plates x 2 x n_t x n_f)."""
    per = max(m_target / 6.0, 4.0)
    n_t = max(2, int(round(math.sqrt(per / 1.48))))
    n_f = max(2, int(round(per / n_t)))
    return n_t, n_f


def solid_displacement(X, seed: int, rotation_deg: float = 10.0, amp: float = 0.002,
                       center=(0.5, 0.5, 0.5)):
    """Synthetic solid state: U = (R - I)(X - c) + amp * d(X), [3][M].

    R is a rigid rotation about the x axis by rotation_deg (a finite rotation) and d a
    smooth field sum_{m=1..3} A_m sin(2 pi k_m . X + phi_m) with integer k_m in {-3..3}^3,
    A_m ~ N(0, I) and phases uniform in [0, 2 pi) (small strains on top of the rotation).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rel = X - np.asarray(center, dtype=np.float64)[:, None]
    th = math.radians(rotation_deg)
    cs, sn = math.cos(th), math.sin(th)
    U = np.stack([np.zeros_like(rel[0]), (cs - 1.0) * rel[1] - sn * rel[2], sn * rel[1] + (cs - 1.0) * rel[2]])
    for _ in range(3):
        kv = rng.integers(-3, 4, size=3)
        while not kv.any():
            kv = rng.integers(-3, 4, size=3)
        A = rng.standard_normal(3)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        U += amp * A[:, None] * np.sin(2.0 * math.pi * (kv @ X) + ph)[None, :]
    return np.ascontiguousarray(U)


def kappa_weights(m: int, solid_volume: float, c_m: float, alpha: float = 100.0):
    """Per-point penalty weight kappa_B = alpha c_m V_B, V_B = V_solid / M."""
    return np.full(m, alpha * c_m * solid_volume / m)


def random_vector(n: int, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)


def channel_dirichlet_mask(grid: Grid):
    """Boolean [3][N]: velocity Dirichlet DOFs of the channel problem.

    Inflow x = 0 (all three components prescribed), no-slip on the four y and z
    faces; x = 1 is traction free (no Dirichlet DOFs, which also fixes the
    pressure level).
    """
    nx, ny, nz = grid.nodes_per_axis
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    node = (i == 0) | (j == 0) | (j == ny - 1) | (k == 0) | (k == nz - 1)
    return np.stack([node, node, node])


def channel_inflow_pattern(grid: Grid):
    """[3][N] Dirichlet data of the channel's inflow for a unit inflow speed: u_x = 1 on the
    x = 0 face, zero elsewhere (no-slip wins on the face's edges)."""
    nx, ny, nz = grid.nodes_per_axis
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inflow = ((i == 0) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)).ravel()
    pat = np.zeros((3, grid.num_nodes))
    pat[0][inflow] = 1.0
    return pat


def channel_inflow_value(t: float, period: float = 0.8):
    """Inflow speed of the channel workloads at time t: sin(2 pi t / period)."""
    return math.sin(2.0 * math.pi * t / period)


def mask_to_bits(mask3):
    """Pack a boolean [3][N] mask into uint32 words, bit (f*N + node) of the stream."""
    flat = np.asarray(mask3, dtype=bool).reshape(-1)
    nwords = (flat.size + 31) // 32
    padded = np.zeros(nwords * 32, dtype=bool)
    padded[: flat.size] = flat
    return np.ascontiguousarray(np.packbits(padded, bitorder="little").view("<u4"))
