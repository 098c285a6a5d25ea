"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module draws random parameters and evaluates closed-form initial data
(Maxwellians, sums of two Maxwellians, the 3D BKW profile, Sod and blast
states).  It contains none of the collision operator's arithmetic: no Fourier
transforms, no kernel tables, no projection.  Everything is FP64 numpy on the
host; callers copy to the device themselves.

Parameter recipes follow the workloads of the paper's numerical section
(two-Maxwellian relaxation of Test 1.3, Sod tube of Part 2, the 3D flow of
Part 4) with the sizes of the configured workloads.
"""
from __future__ import annotations

import math
import numpy as np

BASE_SEED = 1608080090


def rng(offset: int = 0) -> np.random.Generator:
    """PCG64 generator seeded with ``BASE_SEED + offset``."""
    return np.random.Generator(np.random.PCG64(BASE_SEED + int(offset)))


def velocity_nodes(n: int, T: float) -> np.ndarray:
    """Node-based velocity grid v_j = -T + j*2T/n, j = 0..n-1 (FP64)."""
    return -T + np.arange(n, dtype=np.float64) * (2.0 * T / n)


def maxwellian(n: int, T: float, rho: float, u, theta: float) -> np.ndarray:
    """rho (2 pi theta)^{-3/2} exp(-|v-u|^2 / (2 theta)) on the n^3 grid, [x][y][z]."""
    v = velocity_nodes(n, T)
    gx = np.exp(-(v - u[0]) ** 2 / (2 * theta))
    gy = np.exp(-(v - u[1]) ** 2 / (2 * theta))
    gz = np.exp(-(v - u[2]) ** 2 / (2 * theta))
    c = rho / (2 * math.pi * theta) ** 1.5
    return c * gx[:, None, None] * gy[None, :, None] * gz[None, None, :]


def two_maxwellian_params(ncell: int, seed_offset: int = 2):
    """Per-cell parameters of a sum of two isotropic Maxwellians.

    rho ~ U[0.5, 2], theta ~ U[0.5, 2], bulk velocity ~ N(0, 0.5^2 I3) per
    component, independently for each of the two Maxwellians of each cell.
    Returns (rho[ncell,2], theta[ncell,2], u[ncell,2,3]).
    """
    g = rng(seed_offset)
    rho = g.uniform(0.5, 2.0, size=(ncell, 2))
    theta = g.uniform(0.5, 2.0, size=(ncell, 2))
    u = g.normal(0.0, 0.5, size=(ncell, 2, 3))
    return rho, theta, u


def two_maxwellian_cells(n: int, T: float, ncell: int, seed_offset: int = 2,
                         first: int = 0, count: int | None = None) -> np.ndarray:
    """f[count][n][n][n] (FP64): cells first..first+count-1 of the seeded batch."""
    rho, theta, u = two_maxwellian_params(ncell, seed_offset)
    if count is None:
        count = ncell - first
    out = np.empty((count, n, n, n), dtype=np.float64)
    for i in range(count):
        c = first + i
        out[i] = (maxwellian(n, T, rho[c, 0], u[c, 0], theta[c, 0])
                  + maxwellian(n, T, rho[c, 1], u[c, 1], theta[c, 1]))
    return out


def two_maxwellian_torch(n: int, T: float, ncell: int, device, seed_offset: int = 2,
                         dtype=None):
    """Same batch as :func:`two_maxwellian_cells`, evaluated with torch on ``device``.

    The parameters come from the same numpy stream; the Maxwellians are
    evaluated separably in FP64 (outer products of 1D Gaussians), which is the
    same arithmetic as the numpy path up to rounding order of the product.
    """
    import torch
    dtype = dtype or torch.float64
    rho, theta, u = two_maxwellian_params(ncell, seed_offset)
    v = torch.as_tensor(velocity_nodes(n, T), dtype=torch.float64, device=device)
    out = torch.zeros((ncell, n, n, n), dtype=torch.float64, device=device)
    rho_t = torch.as_tensor(rho, device=device)
    th_t = torch.as_tensor(theta, device=device)
    u_t = torch.as_tensor(u, device=device)
    for m in range(2):
        th = th_t[:, m].view(-1, 1)
        c = (rho_t[:, m] / (2 * math.pi * th_t[:, m]) ** 1.5).view(-1, 1, 1, 1)
        gx = torch.exp(-(v.view(1, -1) - u_t[:, m, 0:1]) ** 2 / (2 * th))
        gy = torch.exp(-(v.view(1, -1) - u_t[:, m, 1:2]) ** 2 / (2 * th))
        gz = torch.exp(-(v.view(1, -1) - u_t[:, m, 2:3]) ** 2 / (2 * th))
        out += c * gx[:, :, None, None] * gy[:, None, :, None] * gz[:, None, None, :]
    return out.to(dtype)


def random_positive_cells(n: int, ncell: int, seed_offset: int = 7) -> np.ndarray:
    """Rough positive data U[0.1, 1) per node: exercises every Fourier mode."""
    g = rng(seed_offset)
    return g.uniform(0.1, 1.0, size=(ncell, n, n, n))


def bkw3d(n: int, T: float, t: float) -> np.ndarray:
    """3D BKW profile for Maxwell molecules with unit density and temperature.

    f(v,t) = exp(-|v|^2/2K) / (2 (2 pi K)^{3/2}) * [(5K-3)/K + (1-K)|v|^2/K^2],
    K = 1 - exp(-t/6).  The 3D counterpart of the 2D formula of Test 1.1
    (eq. Jngb); nonnegative for t >= 6 ln(5/2).
    """
    v = velocity_nodes(n, T)
    v2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    K = 1.0 - math.exp(-t / 6.0)
    return bkw3d_K(v2, K)


def bkw3d_K(v2: np.ndarray, K: float) -> np.ndarray:
    """BKW profile as a function of |v|^2 and the similarity parameter K."""
    return (np.exp(-v2 / (2 * K)) / (2 * (2 * math.pi * K) ** 1.5)
            * ((5 * K - 3) / K + (1 - K) * v2 / K ** 2))


def sod_states(nx: int):
    """1D Sod tube on [0,1]: (rho, theta) per cell centre, zero bulk velocity.

    Left (rho=1, theta=1) for x < 1/2, right (rho=0.125, theta=0.8).
    """
    xc = (np.arange(nx) + 0.5) / nx
    rho = np.where(xc < 0.5, 1.0, 0.125)
    theta = np.where(xc < 0.5, 1.0, 0.8)
    return xc, rho, theta


def blast_density(nc: int, x0=(0.5, 0.5, 0.5)) -> np.ndarray:
    """rho = 1 + 0.5 exp(-|x - x0|^2 / 0.01) on an nc^3 periodic unit cube, [z][y][x]."""
    xc = (np.arange(nc) + 0.5) / nc
    dz = (xc - x0[2])[:, None, None] ** 2
    dy = (xc - x0[1])[None, :, None] ** 2
    dx = (xc - x0[0])[None, None, :] ** 2
    return 1.0 + 0.5 * np.exp(-(dx + dy + dz) / 0.01)


# ---------------------------------------------------------------- two velocity dimensions

def maxwellian2(n: int, T: float, rho: float, u, theta: float) -> np.ndarray:
    """rho (2 pi theta)^{-1} exp(-|v-u|^2 / (2 theta)) on the n^2 grid, [x][y]."""
    v = velocity_nodes(n, T)
    gx = np.exp(-(v - u[0]) ** 2 / (2 * theta))
    gy = np.exp(-(v - u[1]) ** 2 / (2 * theta))
    return rho / (2 * math.pi * theta) * gx[:, None] * gy[None, :]


def two_maxwellian_cells_2d(n: int, T: float, ncell: int, seed_offset: int = 20) -> np.ndarray:
    """f[ncell][n][n] (FP64): per cell a sum of two isotropic two-dimensional
    Maxwellians, rho ~ U[0.5, 2], theta ~ U[0.5, 2], u ~ N(0, 0.5^2 I2)
    (the two-Maxwellian shape of the paper's homogeneous tests, in 2D)."""
    g = rng(seed_offset)
    rho = g.uniform(0.5, 2.0, size=(ncell, 2))
    theta = g.uniform(0.5, 2.0, size=(ncell, 2))
    u = g.normal(0.0, 0.5, size=(ncell, 2, 2))
    out = np.empty((ncell, n, n), dtype=np.float64)
    for c in range(ncell):
        out[c] = (maxwellian2(n, T, rho[c, 0], u[c, 0], theta[c, 0])
                  + maxwellian2(n, T, rho[c, 1], u[c, 1], theta[c, 1]))
    return out


def bkw2d_initial(n: int, T: float, node_offset: float = 0.0) -> np.ndarray:
    """Initial datum of the two-dimensional BKW test: |v|^2/pi exp(-|v|^2) on the n^2 grid,
    sampled at v_j = -T + (j + node_offset) 2T/n (node_offset = 1/2: cell centres)."""
    v = velocity_nodes(n, T) + node_offset * (2.0 * T / n)
    v2 = v[:, None] ** 2 + v[None, :] ** 2
    return v2 / math.pi * np.exp(-v2)


# ---------------------------------------------------------------- full-size workload recipes

UNEVEN_N = (16, 24, 32, 48)
UNEVEN_SPLIT = {16: (4, 4), 32: (8, 4), 64: (8, 8)}     # M -> (polar, azimuthal) nodes
UNEVEN_GAMMA = (0.0, 0.5, 1.0)


def uneven_batch_draws(ncell: int = 2048, seed_offset: int = 3):
    """Per-cell (n, M, gamma) drawn uniformly from {16, 24, 32, 48} x {16, 32, 64}
    x {0, 0.5, 1} (the uneven-batch workload); returns three int/float arrays."""
    g = rng(seed_offset)
    n = np.array(UNEVEN_N)[g.integers(0, 4, size=ncell)]
    M = np.array((16, 32, 64))[g.integers(0, 3, size=ncell)]
    gamma = np.array(UNEVEN_GAMMA)[g.integers(0, 3, size=ncell)]
    return n, M, gamma


def blast_cell(n: int, T: float, rho: float, cell: int, seed_offset: int = 5) -> np.ndarray:
    """One cell of the 3D x 3D blast: rho times the unit Maxwellian times (1 + 0.01 xi),
    xi ~ N(0, 1) per velocity node, drawn from a generator seeded per cell."""
    g = rng(10_000_000 * seed_offset + cell)
    return maxwellian(n, T, rho, (0.0, 0.0, 0.0), 1.0) * (1.0 + 0.01 * g.normal(size=(n, n, n)))
