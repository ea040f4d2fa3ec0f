"""FP64 oracle of one full step (test infrastructure only).

One step is the RK3 dycore followed by the column physics on the post-dycore
state, the order of the paper's ASUCA step (physics interface after the
dynamical core, section "The ASUCA Weather Prediction Model") and of the
reduced application's physics-then-dynamics alternation, here with the dycore
first so that physics sees the transported state.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import dycore, physics
from .mass import mass_sums
from .params import DEFAULT, Params


def step(state: dycore.State, inp, p: Params = DEFAULT, physics_on: bool = True,
         dt: Optional[float] = None) -> dycore.State:
    """Advance ``state`` by one step with the frozen winds and 2D fields of ``inp``."""
    dt = inp.dt if dt is None else dt
    k4 = p.k4(inp.dx, dt)
    s = dycore.rk3(state, inp.u, inp.v, inp.w, inp.dx, inp.dx, inp.dz, dt, k4)
    if not physics_on:
        return s
    out = physics.column_physics(s.rho, s.theta, s.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, dt, p)
    return dycore.State(s.rho, out.theta, out.q)


def run(inp, nsteps: int, p: Params = DEFAULT, physics_on: bool = True) -> dycore.State:
    """Run ``nsteps`` steps from the initial state held in ``inp``."""
    s = dycore.State(inp.rho.copy(), inp.theta.copy(), inp.q.copy())
    for _ in range(nsteps):
        s = step(s, inp, p, physics_on)
    return s


def masses(s: dycore.State, inp) -> np.ndarray:
    return mass_sums(s.rho, s.theta, s.q, inp.dx, inp.dx, inp.dz)
