"""Threaded driver of the oracle step over j-slabs (test infrastructure only).

A step of the weather oracle is local: each RK stage reads at most two cells
around a cell in i and j, so one step reads at most six, and the column
physics reads none.  ``run`` therefore advances the whole periodic grid by
applying ``step.step`` to periodic windows of the grid -- one j-slab each,
enlarged by six rows on either side -- and keeping each window's middle
rows.  Every value is the same arithmetic on the same operands as in
``step.run`` over the whole grid (the oracle has no reductions across
cells), so the result is equal bit for bit; a CPU test checks that.  The
windows are independent, so a thread pool runs them at once (NumPy releases
the interpreter lock inside its array loops).

This is how the tests and the benchmark's CPU baseline run the oracle on the
larger grids; it adds no arithmetic of its own.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import dycore, step
from .params import DEFAULT, Params

REACH = 6          # rows one step reads on either side (3 RK stages x 2 cells)


MAX_THREADS = 16   # a one-GPU share of a host's cores


def allowed_cores() -> int:
    """Cores this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:          # pragma: no cover - non-Linux
        return os.cpu_count() or 1


def default_threads() -> int:
    return max(1, min(allowed_cores(), MAX_THREADS))


def _window(a: np.ndarray, rows: np.ndarray) -> np.ndarray:
    return np.take(a, rows, axis=-2)


class _Grid:
    """The frozen fields of one problem and its j-slab windows."""

    def __init__(self, inp, slabs: int):
        self.inp = inp
        ny = inp.ny
        slabs = max(1, min(slabs, ny))
        edges = np.linspace(0, ny, slabs + 1).round().astype(int)
        self.parts = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]
        self.rows = []
        self.frozen = []
        for a, b in self.parts:
            rows = np.arange(a - REACH, b + REACH) % ny
            self.rows.append(rows)
            sub = _SubInputs(inp, rows)
            self.frozen.append(sub)


class _SubInputs:
    """The frozen inputs of one window (the fields ``step.step`` reads)."""

    def __init__(self, inp, rows):
        self.nx, self.ny, self.nz = inp.nx, len(rows), inp.nz
        self.dx, self.dt, self.dz = inp.dx, inp.dt, inp.dz
        for name in ("u", "v", "w", "theta_s", "q_s", "f0", "ch"):
            setattr(self, name, _window(getattr(inp, name), rows))


def run(inp, nsteps: int, threads: int = 0, slabs: int = 0, p: Params = DEFAULT,
        physics_on: bool = True) -> dycore.State:
    """``step.run(inp, nsteps)`` over j-slab windows on ``threads`` threads
    (0: the allowed cores, at most 16); ``slabs`` windows (0: one per thread)."""
    threads = threads or default_threads()
    slabs = slabs or threads
    g = _Grid(inp, slabs)
    s = dycore.State(inp.rho.copy(), inp.theta.copy(), inp.q.copy())

    def one(n):
        rows, sub = g.rows[n], g.frozen[n]
        win = dycore.State(*(_window(f, rows) for f in s))
        out = step.step(win, sub, p, physics_on)
        return tuple(f[:, REACH:REACH + (g.parts[n][1] - g.parts[n][0])] for f in out)

    with ThreadPoolExecutor(max_workers=threads) as pool:
        for _ in range(nsteps):
            pieces = list(pool.map(one, range(len(g.parts))))
            s = dycore.State(*(np.concatenate([pc[f] for pc in pieces], axis=1) for f in range(3)))
    return s
