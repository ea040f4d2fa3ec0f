"""Seeded synthetic inputs for the structured-grid weather step.

This module only *draws* inputs: the grid spacing profile, the frozen C-grid
winds, the initial prognostic fields, the 2D surface fields and the time step
fixed by the Courant limit.  It holds none of the step's own arithmetic (no
fluxes, no diffusion, no physics), so both the FP64 CPU oracle and the GPU path
may consume what it returns.

Every array is drawn in C order with shape ``(nz, ny, nx)`` (``(ny, nx)`` for
the 2D fields), so ``i`` is the fastest index, matching the i-fastest storage
order the paper prescribes for GPUs (section "Architecture-Dependent Storage
Order").  ``k = 0`` is the lowest level.

Random streams: ``numpy.random.Generator(PCG64(SeedSequence([seed, sid])))``
with stream ids psi=1, w=3, q=4, mode phases=5, C_h=6 (2 is unused).

Recipe (the paper gives only the problem class, a 2 km mesoscale C-grid with
58 stretched levels, section "The ASUCA Weather Prediction Model"; the numbers
below are this implementation's choices):

* ``dz_k = 50 * r**k`` with ``r = 20**(1/(nz-1))`` (50 m at the ground,
  1000 m at the top).
* Horizontal winds at C-grid faces (u at east faces ``x=(i+1)dx``, v at north
  faces ``y=(j+1)dy``) from a streamfunction psi at cell corners,
  ``u = -d(psi)/dy``, ``v = d(psi)/dx``: white psi noise scaled so that u and v
  are each N(0, 10^2) m/s, plus three 5 m/s sine modes with wave numbers (1,0),
  (0,1), (1,1) over the domain and uniform random phases.
* w at the ``nz+1`` face levels: N(0, 0.1^2) on interior faces with the mean of
  each face level removed, 0 at the ground and the lid.
* An irrotational correction ``grad(chi)`` (periodic Poisson solve per level)
  absorbs the vertical divergence of w, so the discrete 3D divergence of the
  frozen wind is zero to rounding.  Independent draws per face give a wind
  whose convergence zones compound density exponentially (the exact solution
  of the continuity equation under a frozen divergent wind is unbounded), so a
  multi-hundred-step run could not stay finite under any scheme.
* theta = 300 + 2 sin(2 pi x/Lx) sin(2 pi y/Ly) exp(-((z-3000)/3000)^2) K.
* q = min(0.02, lognormal(ln 0.006, 0.5)) kg/kg, independent per cell.
* rho = 1.2 exp(-z/8000) kg/m^3.
* theta_s = 301 + sin(2 pi j/ny) K, q_s = 0.015,
  F0 = 600 + 200 sin(2 pi i/nx) cos(2 pi j/ny) W/m^2, C_h ~ U(0.005, 0.02) m/s.
* dt = 0.3 / max over cells of the summed directional Courant rate.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

STREAM_PSI, STREAM_W, STREAM_Q, STREAM_PHASE, STREAM_CH = 1, 3, 4, 5, 6

# Named grid configurations (the paper's 1581x1301x58 production grid and
# smaller shares of it).
CONFIGS = {
    "tiny": dict(nx=64, ny=64, nz=16, seed=0),
    "share": dict(nx=400, ny=320, nz=58, seed=1),
    "full": dict(nx=1581, ny=1301, nz=58, seed=2),
    "crop": dict(nx=256, ny=256, nz=58, seed=3),
}

DX_DEFAULT = 2000.0
CFL_DEFAULT = 0.3


def _rng(seed: int, sid: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(sid)])))


def stretched_dz(nz: int, dz_bottom: float = 50.0, dz_top: float = 1000.0) -> np.ndarray:
    """Geometric level thicknesses from ``dz_bottom`` to ``dz_top`` (nz >= 2)."""
    if nz < 2:
        raise ValueError("nz must be >= 2")
    r = (dz_top / dz_bottom) ** (1.0 / (nz - 1))
    return dz_bottom * r ** np.arange(nz, dtype=np.float64)


def level_centres(dz: np.ndarray) -> np.ndarray:
    """Height of each cell centre above the ground."""
    return np.concatenate(([0.0], np.cumsum(dz)[:-1])) + 0.5 * dz


@dataclasses.dataclass
class Inputs:
    """One seeded problem: geometry, frozen winds, initial state, 2D fields."""

    nx: int
    ny: int
    nz: int
    dx: float
    dt: float
    dz: np.ndarray          # (nz,)
    u: np.ndarray           # (nz, ny, nx) east-face winds
    v: np.ndarray           # (nz, ny, nx) north-face winds
    w: np.ndarray           # (nz+1, ny, nx) face-level winds, w[0]=w[nz]=0
    rho: np.ndarray         # (nz, ny, nx)
    theta: np.ndarray       # (nz, ny, nx)
    q: np.ndarray           # (nz, ny, nx)
    theta_s: np.ndarray     # (ny, nx)
    q_s: np.ndarray         # (ny, nx)
    f0: np.ndarray          # (ny, nx)
    ch: np.ndarray          # (ny, nx)
    seed: int = 0

    def fields(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in
                ("u", "v", "w", "rho", "theta", "q", "theta_s", "q_s", "f0", "ch")}

    def copy(self) -> "Inputs":
        return dataclasses.replace(self, **{k: v.copy() for k, v in self.fields().items()},
                                   dz=self.dz.copy())

    def astype(self, dtype) -> "Inputs":
        """Round every field to ``dtype`` and back to float64 (same values both sides see)."""
        out = self.copy()
        for k, v in out.fields().items():
            setattr(out, k, v.astype(dtype).astype(np.float64))
        return out


def cfl_dt(u: np.ndarray, v: np.ndarray, w: np.ndarray, dx: float, dy: float,
           dz: np.ndarray, cfl: float = CFL_DEFAULT) -> float:
    """Time step at which the largest summed Courant rate equals ``cfl``.

    For each cell the rate is max|u| over its two x faces / dx + the same in y
    + max|w| over its two z faces / dz_k.  The faces of cell i in x are the
    east faces of cells i-1 and i (periodic).
    """
    au = np.abs(u)
    ax = np.maximum(au, np.roll(au, 1, axis=2)) / dx
    av = np.abs(v)
    ay = np.maximum(av, np.roll(av, 1, axis=1)) / dy
    aw = np.abs(w)
    az = np.maximum(aw[:-1], aw[1:]) / dz[:, None, None]
    rate = float(np.max(ax + ay + az))
    return cfl / rate


def generate(nx: int, ny: int, nz: int, seed: int = 0, dx: float = DX_DEFAULT,
             dz: Optional[np.ndarray] = None, dt: Optional[float] = None,
             cfl: float = CFL_DEFAULT) -> Inputs:
    """Draw one seeded problem of the given size (all float64)."""
    if dz is None:
        dz = stretched_dz(nz)
    dz = np.asarray(dz, dtype=np.float64)
    dy = dx
    lx, ly = nx * dx, ny * dy
    zc = level_centres(dz)

    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)

    # streamfunction at corners (x=(i+1)dx, y=(j+1)dy): noise plus three modes
    sig_psi = 10.0 * dy / np.sqrt(2.0)
    psi = _rng(seed, STREAM_PSI).normal(0.0, sig_psi, size=(nz, ny, nx))
    phases = _rng(seed, STREAM_PHASE).uniform(0.0, 2.0 * np.pi, size=3)
    xq, yq = (i + 1.0) * dx, (j + 1.0) * dy
    for (a, b), ph in zip(((1.0, 0.0), (0.0, 1.0), (1.0, 1.0)), phases):
        kmag = 2.0 * np.pi * np.hypot(a / lx, b / ly)
        psi += ((5.0 / kmag) * np.sin(2.0 * np.pi * (a * xq[None, :] / lx + b * yq[:, None] / ly)
                                      + ph))[None]
    u = -(psi - np.roll(psi, 1, axis=1)) / dy
    v = (psi - np.roll(psi, 1, axis=2)) / dx
    del psi

    w = np.zeros((nz + 1, ny, nx))
    if nz > 1:
        w[1:nz] = _rng(seed, STREAM_W).normal(0.0, 0.1, size=(nz - 1, ny, nx))
        w[1:nz] -= w[1:nz].mean(axis=(1, 2), keepdims=True)

    # irrotational part: (d2/dx2 + d2/dy2) chi = -(w_top - w_bottom)/dz per level
    src = -(w[1:] - w[:-1]) / dz[:, None, None]
    lam = (-(4.0 / dx ** 2) * np.sin(np.pi * np.arange(nx // 2 + 1) / nx) ** 2)[None, :] \
        + (-(4.0 / dy ** 2) * np.sin(np.pi * np.fft.fftfreq(ny)) ** 2)[:, None]
    lam[0, 0] = 1.0
    chat = np.fft.rfft2(src) / lam[None]
    chat[:, 0, 0] = 0.0
    chi = np.fft.irfft2(chat, s=(ny, nx))
    del chat, src
    u += (np.roll(chi, -1, axis=2) - chi) / dx
    v += (np.roll(chi, -1, axis=1) - chi) / dy
    del chi

    xc = (i + 0.5) * dx
    yc = (j + 0.5) * dy
    hpert = np.sin(2.0 * np.pi * yc / ly)[:, None] * np.sin(2.0 * np.pi * xc / lx)[None, :]
    vprof = np.exp(-((zc - 3000.0) / 3000.0) ** 2)
    theta = 300.0 + 2.0 * vprof[:, None, None] * hpert[None]
    q = np.minimum(0.02, np.exp(_rng(seed, STREAM_Q).normal(np.log(0.006), 0.5, size=(nz, ny, nx))))
    rho = np.broadcast_to(1.2 * np.exp(-zc / 8000.0)[:, None, None], (nz, ny, nx)).copy()

    theta_s = np.broadcast_to((301.0 + np.sin(2.0 * np.pi * j / ny))[:, None], (ny, nx)).copy()
    q_s = np.full((ny, nx), 0.015)
    f0 = 600.0 + 200.0 * np.cos(2.0 * np.pi * j / ny)[:, None] * np.sin(2.0 * np.pi * i / nx)[None, :]
    ch = _rng(seed, STREAM_CH).uniform(0.005, 0.02, size=(ny, nx))

    if dt is None:
        dt = cfl_dt(u, v, w, dx, dy, dz, cfl)
    return Inputs(nx=nx, ny=ny, nz=nz, dx=float(dx), dt=float(dt), dz=dz, u=u, v=v, w=w,
                  rho=rho, theta=theta, q=q, theta_s=theta_s, q_s=q_s, f0=f0, ch=ch, seed=seed)


def generate_config(name: str, **overrides) -> Inputs:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    return generate(**cfg)


def crop(inp: Inputs, i0: int, j0: int, cx: int, cy: int) -> Inputs:
    """Periodic window [i0, i0+cx) x [j0, j0+cy) of every field (indices wrap)."""
    ii = np.arange(i0, i0 + cx) % inp.nx
    jj = np.arange(j0, j0 + cy) % inp.ny

    def c3(a):
        return a[:, jj][:, :, ii]

    def c2(a):
        return a[jj][:, ii]

    return Inputs(nx=cx, ny=cy, nz=inp.nz, dx=inp.dx, dt=inp.dt, dz=inp.dz.copy(),
                  u=c3(inp.u), v=c3(inp.v), w=c3(inp.w), rho=c3(inp.rho), theta=c3(inp.theta),
                  q=c3(inp.q), theta_s=c2(inp.theta_s), q_s=c2(inp.q_s), f0=c2(inp.f0),
                  ch=c2(inp.ch), seed=inp.seed)
