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
with stream ids psi_z=1, psi_x=2, psi_y=3, q=4, mode phases=5, C_h=6.

Recipe (the paper gives only the problem class, a 2 km mesoscale C-grid with
58 stretched levels, section "The ASUCA Weather Prediction Model"; the numbers
below are this implementation's choices):

* ``dz_k = 50 * r**k`` with ``r = 20**(1/(nz-1))`` (50 m at the ground,
  1000 m at the top).
* Winds at C-grid faces (u at east faces ``x=(i+1)dx``, v at north faces
  ``y=(j+1)dy``, w at the ``nz+1`` face levels) are the discrete curl of an
  edge-staggered vector potential ``(psi_x, psi_y, psi_z)``:
  ``u = d(psi_z)/dy - d(psi_y)/dz``, ``v = d(psi_x)/dz - d(psi_z)/dx``,
  ``w = d(psi_y)/dx - d(psi_x)/dy``.  psi_z is white noise scaled so that its
  part of u and v is N(0, 10^2) m/s, plus three 5 m/s sine modes with wave
  numbers (1,0), (0,1), (1,1) over the domain and uniform random phases.
  psi_x, psi_y are white noise scaled so that w is N(0, 0.1^2) m/s, and zero
  on the ground and lid edges so that w vanishes there.  The discrete 3D
  divergence of such a wind is zero to rounding.  Independent draws per face
  would give a wind whose convergence zones compound density exponentially
  (the exact solution of the continuity equation under a frozen divergent
  wind is unbounded), so a multi-hundred-step run could not stay finite under
  any scheme.  The vertical part adds about 141/dz_k m/s rms to u and v.
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

STREAM_PSI_Z, STREAM_PSI_X, STREAM_PSI_Y, STREAM_Q, STREAM_PHASE, STREAM_CH = 1, 2, 3, 4, 5, 6

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
             cfl: float = CFL_DEFAULT, dtype=np.float64) -> Inputs:
    """Draw one seeded problem of the given size.

    Values are computed in float64 one k-plane at a time and stored as
    ``dtype`` (float64 by default; float32 halves the host memory of a
    full-size problem and gives the same values as rounding the float64 draw).
    """
    if dz is None:
        dz = stretched_dz(nz)
    dz = np.asarray(dz, dtype=np.float64)
    dy = dx
    lx, ly = nx * dx, ny * dy
    zc = level_centres(dz)
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)

    g_psi = _rng(seed, STREAM_PSI_Z)
    g_px = _rng(seed, STREAM_PSI_X)
    g_py = _rng(seed, STREAM_PSI_Y)
    g_q = _rng(seed, STREAM_Q)
    phases = _rng(seed, STREAM_PHASE).uniform(0.0, 2.0 * np.pi, size=3)

    # psi_z modes on vertical edges (x=(i+1)dx, y=(j+1)dy), same on every level
    xq, yq = (i + 1.0) * dx, (j + 1.0) * dy
    modes = np.zeros((ny, nx))
    for (a, b), ph in zip(((1.0, 0.0), (0.0, 1.0), (1.0, 1.0)), phases):
        kmag = 2.0 * np.pi * np.hypot(a / lx, b / ly)
        modes += (5.0 / kmag) * np.sin(2.0 * np.pi * (a * xq[None, :] / lx + b * yq[:, None] / ly) + ph)
    sig_psi = 10.0 * dy / np.sqrt(2.0)
    sig = 0.1 * dx / 2.0               # psi_x, psi_y: w ~ N(0, 0.1^2)

    u = np.empty((nz, ny, nx), dtype=dtype)
    v = np.empty((nz, ny, nx), dtype=dtype)
    w = np.zeros((nz + 1, ny, nx), dtype=dtype)
    theta = np.empty((nz, ny, nx), dtype=dtype)
    q = np.empty((nz, ny, nx), dtype=dtype)
    rho = np.empty((nz, ny, nx), dtype=dtype)

    def dj_(a):                        # a[j] - a[j-1], periodic
        return a - np.roll(a, 1, axis=0)

    def di_(a):                        # a[i] - a[i-1], periodic
        return a - np.roll(a, 1, axis=1)

    xc = (i + 0.5) * dx
    yc = (j + 0.5) * dy
    hpert = np.sin(2.0 * np.pi * yc / ly)[:, None] * np.sin(2.0 * np.pi * xc / lx)[None, :]
    vprof = np.exp(-((zc - 3000.0) / 3000.0) ** 2)

    zero = np.zeros((ny, nx))
    px_lo, py_lo = zero, zero          # psi_x, psi_y on the face below level k
    rate = 0.0
    for k in range(nz):
        psi = g_psi.normal(0.0, sig_psi, size=(ny, nx)) + modes
        if k + 1 < nz:
            px_hi = g_px.normal(0.0, sig, size=(ny, nx))
        else:
            px_hi = zero
        if k + 1 < nz:
            py_hi = g_py.normal(0.0, sig, size=(ny, nx))
        else:
            py_hi = zero
        uk = -dj_(psi) / dy - (py_hi - py_lo) / dz[k]
        vk = di_(psi) / dx + (px_hi - px_lo) / dz[k]
        if k + 1 < nz:
            w[k + 1] = di_(py_hi) / dx - dj_(px_hi) / dy
        u[k] = uk
        v[k] = vk
        theta[k] = 300.0 + 2.0 * vprof[k] * hpert
        q[k] = np.minimum(0.02, np.exp(g_q.normal(np.log(0.006), 0.5, size=(ny, nx))))
        rho[k] = 1.2 * np.exp(-zc[k] / 8000.0)
        # summed Courant rate of the cells of this level
        au = np.abs(u[k].astype(np.float64))
        av = np.abs(v[k].astype(np.float64))
        aw = np.maximum(np.abs(w[k].astype(np.float64)), np.abs(w[k + 1].astype(np.float64)))
        lvl = (np.maximum(au, np.roll(au, 1, axis=1)) / dx + np.maximum(av, np.roll(av, 1, axis=0)) / dy
               + aw / dz[k])
        rate = max(rate, float(lvl.max()))
        px_lo, py_lo = px_hi, py_hi

    theta_s = np.broadcast_to((301.0 + np.sin(2.0 * np.pi * j / ny))[:, None], (ny, nx)).astype(dtype)
    q_s = np.full((ny, nx), 0.015, dtype=dtype)
    f0 = (600.0 + 200.0 * np.cos(2.0 * np.pi * j / ny)[:, None]
          * np.sin(2.0 * np.pi * i / nx)[None, :]).astype(dtype)
    ch = _rng(seed, STREAM_CH).uniform(0.005, 0.02, size=(ny, nx)).astype(dtype)

    if dt is None:
        dt = cfl / rate
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


# ---- the paper's reduced weather application ------------------------------
# Its initial state and boundary values (section "Reduced Weather
# Application": a 300 box in a zero field, heat wells of 330 at the surface
# and 200 at the boundary layer).  The field is (nz, ny + 2, nx + 2) float64,
# i fastest, with a one-cell ring around the nx x ny interior.

RW_SURFACE = 330.0
RW_PBL = 200.0
RW_NU_DEFAULT = 0.1      # the diffusion number; the paper prints no value for it


def rw_shape(nx: int, ny: int, nz: int):
    """Array shape (k, j, i) of a reduced-application field, ring included."""
    return (nz, ny + 2, nx + 2)


def rw_box_init(nx: int, ny: int, nz: int) -> np.ndarray:
    """0 everywhere except 300 on the middle half of each dimension.

    A cell with 1-based interior indices (i, j, k) is inside when
    n/4 < index <= 3n/4 in every dimension; the ring (index 0 and n+1) is
    outside.
    """
    e = np.zeros(rw_shape(nx, ny, nz))

    def inside(n, idx):
        return (idx * 4 > n) & (idx * 4 <= 3 * n)

    ii = inside(nx, np.arange(nx + 2))
    jj = inside(ny, np.arange(ny + 2))
    kk = inside(nz, np.arange(1, nz + 1))
    e[np.ix_(kk, jj, ii)] = 300.0
    return e


def rw_boundary_fields(nx: int, ny: int):
    """Surface and boundary-layer values over the (ny + 2) x (nx + 2) columns."""
    return np.full((ny + 2, nx + 2), RW_SURFACE), np.full((ny + 2, nx + 2), RW_PBL)


# ---- fast modes (HEVI short steps) ----------------------------------------
# Perturbation fields of the linear acoustic-gravity system about a resting
# state: u, v at east / north faces and pi at cell centres (nz, ny, nx); w and
# b on the nz + 1 level faces, zero at the ground and lid.  White noise plus a
# smooth large-scale part, so that both the grid-scale and the long waves are
# present:  u, v ~ N(0, 1) m/s + 2 m/s modes;  w ~ N(0, 0.05) m/s;
# b ~ N(0, 0.005) m/s^2;  pi ~ N(0, 5) m^2/s^2 + a 20 m^2/s^2 mode.  Stream ids
# 11-15.  The short step defaults to 2 s, a horizontal sound Courant number
# c tau / dx = 0.34 at 2 km.

HEVI_TAU_DEFAULT = 2.0
HEVI_C_SOUND = 340.0
HEVI_N_BV = 0.01


@dataclasses.dataclass
class FastFields:
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    b: np.ndarray
    pi: np.ndarray
    dz: np.ndarray
    dx: float

    def astype(self, dtype) -> "FastFields":
        """Values rounded to ``dtype`` (stored back as float64)."""
        c = lambda a: a.astype(dtype).astype(np.float64)  # noqa: E731
        return FastFields(c(self.u), c(self.v), c(self.w), c(self.b), c(self.pi), self.dz.copy(), self.dx)


def hevi_fields(nx: int, ny: int, nz: int, seed: int = 0, dx: float = DX_DEFAULT,
                dz: Optional[np.ndarray] = None) -> FastFields:
    dz = stretched_dz(nz) if dz is None else np.asarray(dz, dtype=np.float64)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    ph = _rng(seed, 15).uniform(0.0, 2.0 * np.pi, 3)
    mode = np.sin(2.0 * np.pi * x[None, :] + ph[0]) * np.cos(2.0 * np.pi * y[:, None] + ph[1])
    zc = level_centres(dz)
    vert = np.cos(np.pi * zc / (np.sum(dz)))[:, None, None]
    u = _rng(seed, 11).normal(0.0, 1.0, (nz, ny, nx)) + 2.0 * vert * mode[None]
    v = _rng(seed, 12).normal(0.0, 1.0, (nz, ny, nx)) - 2.0 * vert * mode[None]
    w = np.zeros((nz + 1, ny, nx))
    w[1:nz] = _rng(seed, 13).normal(0.0, 0.05, (nz - 1, ny, nx))
    b = np.zeros((nz + 1, ny, nx))
    b[1:nz] = _rng(seed, 14).normal(0.0, 0.005, (nz - 1, ny, nx))
    pi = _rng(seed, 15).normal(0.0, 5.0, (nz, ny, nx)) + 20.0 * vert * mode[None]
    return FastFields(u, v, w, b, pi, dz, dx)
