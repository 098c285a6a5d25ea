"""FP64 CPU oracle of the BGK relaxation operator with the conservative discrete
Maxwellian (test infrastructure; only tests, the smoke check and the bench's
CPU-baseline leg may use it, and it shares no code with the HIP library).

Q_BGK(f) = nu (E[U] - f) (Section 2, eq. ibgk), where U = C f are the discrete
moments of the cell and E[U] is the pointwise Maxwellian M[f] at the nodes
(Section 2, eq. i5 and the temperature relation below it) projected back onto
U with the minimisation of Section 3.2 (eq. minimMax), so that C E[U] = U.

Readings:
* the temperature is d_v rho theta = sum |v|^2 f dv^{d_v} - rho |u|^2 (eq. i5's
  relation with E = (1/2) int |v|^2 f);
* nu is either a constant (mu in Test 4.1) or nu = rho (Test 2.2), possibly scaled;
* the time step is the forward Euler step of eq. f_coll, or, as an option,
  the exact solution of d f/dt = nu (E - f) with E fixed (the moments, hence E,
  do not change during the collision step).
"""
from __future__ import annotations

import math

import numpy as np

from . import fks_oracle as O3
from . import fks_oracle2d as O2

__all__ = ["bgk_moments", "bgk_primitive", "bgk_maxwellian_pointwise", "bgk_equilibrium",
           "bgk_Q", "bgk_step"]


def bgk_moments(f: np.ndarray, n: int, T: float, dim: int) -> np.ndarray:
    """U = C f (rho, rho u, sum |v|^2 f dv^d) of one cell."""
    return (O2.moments2(f, n, T) if dim == 2 else O3.moments(f, n, T)).reshape(-1)


def bgk_primitive(U: np.ndarray, dim: int):
    """(rho, u, theta) with d rho theta = U_last - rho |u|^2."""
    rho = U[0]
    u = U[1:1 + dim] / rho
    theta = (U[1 + dim] / rho - float(u @ u)) / dim
    return rho, u, theta


def bgk_maxwellian_pointwise(U: np.ndarray, n: int, T: float, dim: int) -> np.ndarray:
    """rho (2 pi theta)^{-d/2} exp(-|v - u|^2 / (2 theta)) at the nodes (eq. i5)."""
    rho, u, theta = bgk_primitive(U, dim)
    v = O3.velocity_grid(n, T)
    axes = np.meshgrid(*([v] * dim), indexing="ij")
    r2 = sum((a - ua) ** 2 for a, ua in zip(axes, u))
    return rho / (2.0 * math.pi * theta) ** (dim / 2.0) * np.exp(-r2 / (2.0 * theta))


def bgk_equilibrium(f: np.ndarray, n: int, T: float, dim: int) -> np.ndarray:
    """E[U] = M~ + C^T (C C^T)^{-1} (U - C M~) with U = C f (eq. minimMax)."""
    U = bgk_moments(f, n, T, dim)
    Mt = bgk_maxwellian_pointwise(U, n, T, dim)
    if dim == 2:
        return O2.project2(Mt, U, n, T)
    return O3.project(Mt, U, n, T)


def bgk_Q(f: np.ndarray, n: int, T: float, dim: int, nu: float, nu_rho: bool = False) -> np.ndarray:
    """Q_BGK = nu' (E[U] - f) with nu' = nu, or nu * rho if ``nu_rho`` (eq. ibgk)."""
    E = bgk_equilibrium(f, n, T, dim)
    rho = bgk_moments(f, n, T, dim)[0]
    return (nu * rho if nu_rho else nu) * (E - f)


def bgk_step(f: np.ndarray, n: int, T: float, dim: int, nu: float, dt_over_tau: float,
             nu_rho: bool = False, exact: bool = False) -> np.ndarray:
    """One collision step: f + (dt/tau) Q_BGK (eq. f_coll) or, if ``exact``,
    E + exp(-nu' dt/tau) (f - E)."""
    E = bgk_equilibrium(f, n, T, dim)
    rho = bgk_moments(f, n, T, dim)[0]
    nup = nu * rho if nu_rho else nu
    if exact:
        return E + math.exp(-nup * dt_over_tau) * (f - E)
    return f + dt_over_tau * nup * (E - f)
