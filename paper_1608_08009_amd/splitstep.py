"""FKS split step on the GPU: exact transport shift, then the collision update.

One step (Section 3.1, eqs. transport/collision splitting, f_bar and f_coll):
    f*      = transport_shift(f)                      (fks_transport_shift)
    f^{n+1} = f* + (dt/tau) Q_c(f*)                   (fks_collide_batch)
where Q_c is the fast spectral operator after the conservation projection.
Every step runs in the HIP library; this module only sequences the calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import (BC_DIRICHLET, BC_PERIODIC, Plan, collide_batch, transport_shift,
               workspace_size)


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
    """min(dx/T, tau/mu) with mu = 4 pi C_gamma (2R)^gamma rho_max (collision stability bound)."""
    mu = 4.0 * math.pi * c_gamma * (2.0 * R) ** gamma * rho_max
    return min(space.dx / T, tau / mu)


class SplitStepper:
    """Owns the ping-pong buffer, the workspace and the transport offsets of one run."""

    def __init__(self, plan: Plan, space: Space, f, bc_f=None):
        import torch
        self.plan = plan
        self.space = space
        self.n = plan.n
        self.T = plan.desc.T
        self.f = f
        self.tmp = torch.empty_like(f)
        self.bc_f = bc_f
        self.offsets = np.zeros((3, self.n), dtype=np.float64)
        seg = [(plan, self.tmp, None, self.f, space.ncell, 0.0)]
        self.ws = torch.empty(max(workspace_size(seg), 1), dtype=torch.uint8, device=f.device)
        self.steps = 0

    def step(self, dt: float, tau: float) -> None:
        sp = self.space
        transport_shift(self.f, self.tmp, sp.nx, sp.ny, sp.nz, sp.dx, sp.bc, self.n, self.T, dt,
                        self.offsets, bc_f=self.bc_f)
        collide_batch([(self.plan, self.tmp, None, self.f, sp.ncell, dt / tau)], workspace=self.ws)
        self.steps += 1
