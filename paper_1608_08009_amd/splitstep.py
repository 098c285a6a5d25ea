"""FKS split step on the GPU: exact transport shift, then the collision update.

One step (Section 3.1, eqs. transport/collision splitting, f_bar and f_coll):
    f*      = transport_shift(f)                      (fks_transport_shift)
    f^{n+1} = f* + (dt/tau) Q_c(f*)                   (fks_collide_batch)
where Q_c is the fast spectral operator after the conservation projection.
Variants (the paper names higher-order splittings and other collision
integrators as possible; Section 3.1):
  * scheme="strang": half a transport step, the collision step, half a
    transport step (the transport shift is exact for any dt);
  * collision="rk2": the midpoint rule for the collision ODE,
    f^{n+1} = f* + (dt/tau) Q_c(f* + (dt/2tau) Q_c(f*)), as two calls of
    fks_collide_batch (the second with f_base = f*);
  * collision="exp": the exponential Euler step for stiff collisions (small
    tau; the paper defers to the integrators of its references).  With Q split
    as [Q + mu (f - M)] - mu (f - M), M the local Maxwellian, the step is
    f^{n+1} = f* + ((1 - exp(-mu dt/tau)) / mu) Q_c(f*): one call whose step
    never exceeds 1/mu.  mu bounds the loss frequency, e.g.
    4 pi C_gamma (2R)^gamma rho_max.
Every step runs in the HIP library; this module only sequences the calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import (BC_DIRICHLET, BC_PERIODIC, Plan, collide_batch, exp_euler_step, transport_shift,
               workspace_size)
from . import stable_dt as _stable_dt


@dataclass
class Space:
    nx: int
    ny: int
    nz: int
    dx: float
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz


def stable_dt(space: Space, T: float, tau: float, R: float, gamma: float, c_gamma: float,
              rho_max: float) -> float:
    """min(dx/T, tau/mu) with mu = 4 pi C_gamma (2R)^gamma rho_max (fks_stable_dt)."""
    return _stable_dt(space.dx, T, tau, R, gamma, c_gamma, rho_max)


class SplitStepper:
    """Owns the ping-pong buffers, the workspace and the transport offsets of one run."""

    def __init__(self, plan: Plan, space: Space, f, bc_f=None, scheme: str = "lie",
                 collision: str = "euler", mu: float = 0.0):
        import torch
        if scheme not in ("lie", "strang") or collision not in ("euler", "rk2", "exp"):
            raise ValueError("scheme must be 'lie' or 'strang', collision 'euler', 'rk2' or 'exp'")
        if collision == "exp" and not (mu > 0 and math.isfinite(mu)):
            raise ValueError("collision='exp' needs the penalization constant mu > 0")
        self.mu = mu
        self.plan = plan
        self.space = space
        self.n = plan.n
        self.T = plan.desc.T
        self.f = f
        self.tmp = torch.empty_like(f)
        self.mid = torch.empty_like(f) if collision == "rk2" else None
        self.bc_f = bc_f
        self.scheme = scheme
        self.collision = collision
        self.offsets = np.zeros((3, self.n), dtype=np.float64)
        seg = [(plan, self.tmp, None, self.f, space.ncell, 0.0)]
        self.ws = torch.empty(max(workspace_size(seg), 1), dtype=torch.uint8, device=f.device)
        self.steps = 0

    def _transport(self, src, dst, dt: float) -> None:
        sp = self.space
        transport_shift(src, dst, sp.nx, sp.ny, sp.nz, sp.dx, sp.bc, self.n, self.T, dt,
                        self.offsets, bc_f=self.bc_f)

    def _collide(self, src, dst, dt_over_tau: float) -> None:
        nc = self.space.ncell
        if self.collision == "exp":
            h = exp_euler_step(self.mu, dt_over_tau)
            collide_batch([(self.plan, src, None, dst, nc, h)], workspace=self.ws)
        elif self.collision == "euler":
            collide_batch([(self.plan, src, None, dst, nc, dt_over_tau)], workspace=self.ws)
        else:
            collide_batch([(self.plan, src, None, self.mid, nc, 0.5 * dt_over_tau)], workspace=self.ws)
            collide_batch([(self.plan, self.mid, None, dst, nc, dt_over_tau, src)], workspace=self.ws)

    def step(self, dt: float, tau: float) -> None:
        if self.scheme == "lie":
            self._transport(self.f, self.tmp, dt)
            self._collide(self.tmp, self.f, dt / tau)
        else:
            self._transport(self.f, self.tmp, 0.5 * dt)
            self._collide(self.tmp, self.f, dt / tau)
            self._transport(self.f, self.tmp, 0.5 * dt)
            self.f, self.tmp = self.tmp, self.f
        self.steps += 1
