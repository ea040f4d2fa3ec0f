"""FP64 oracle of the HEVI fast-mode short step (test infrastructure only).

What the paper fixes (section "The ASUCA Weather Prediction Model"): sound
and gravity waves are integrated separately from the long Runge-Kutta step,
with a second-order Runge-Kutta scheme in shorter steps, horizontally
explicit and vertically implicit (HEVI); section "Hybrid ASUCA Strong Scaling
GPU Results" names these fast modes as the largest cost of the model.  It
prints no equations; the readings taken here (R-hevi) are:

* The fast modes are the linear acoustic-gravity system about a resting
  state, with kinematic pressure pi (pressure perturbation over the reference
  density) and buoyancy b:
      du/dt = -dpi/dx,  dv/dt = -dpi/dy,  dw/dt = -dpi/dz + b,
      db/dt = -N^2 w,   dpi/dt = -c^2 (du/dx + dv/dy + dw/dz),
  sound speed c (340 m/s by default) and buoyancy frequency N (0.01 1/s).
* C-grid placement as the dycore's winds: u on east faces, v on north faces,
  pi at cell centres; w and b on the nz + 1 vertical faces (b with w, so the
  buoyancy coupling is local), w = b = 0 on the ground and lid faces.
  Differences: dpi/dx at face i+1/2 is (pi_{i+1} - pi_i)/dx and du/dx at
  cell i is (u_{i+1/2} - u_{i-1/2})/dx (periodic); dpi/dz at face k+1/2 is
  (pi_{k+1} - pi_k)/dz_{k+1/2} with dz_{k+1/2} = (dz_k + dz_{k+1})/2 and
  dw/dz at cell k is (w_{k+1/2} - w_{k-1/2})/dz_k.
* One short step of length tau is a two-stage (midpoint) Runge-Kutta step:
  stage s in {1, 2} with h = tau/2, tau starts from the step's base state X
  and uses the previous stage's pi (stage 0 = the base) in the horizontal:
      u' = u - h dpi_prev/dx,  v' = v - h dpi_prev/dy       (explicit)
      D  = du'/dx + dv'/dy                                    (forward-backward)
  then the vertical terms are trapezoidal (implicit) over the stage, with
  wm = (w' + w)/2 the stage's mean vertical wind:
      wm - w = (h/2) (-dpi_m/dz + b_m),  b_m = b - (h/2) N^2 wm,
      pi_m = pi - (h/2) c^2 (D + dwm/dz),
  a tridiagonal system for wm on the interior faces of every column (the
  same matrix in every column); then w' = 2 wm - w, b' = b - h N^2 wm,
  pi' = pi - h c^2 (D + dwm/dz).

Array conventions: u, v, pi are (nz, ny, nx); w, b are (nz + 1, ny, nx) with
index f the face below level f.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np
from scipy.linalg import solve_banded

C_SOUND = 340.0       # m/s
N_BV = 0.01           # 1/s
AX_K, AX_J, AX_I = 0, 1, 2


class Fast(NamedTuple):
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    b: np.ndarray
    pi: np.ndarray


def face_spacing(dz: np.ndarray) -> np.ndarray:
    """dz_{k+1/2} for the nz - 1 interior faces."""
    return (dz[:-1] + dz[1:]) / 2.0


def horizontal(base: Fast, pi_prev: np.ndarray, dx: float, dy: float, h: float):
    """Stage winds u' = u - h dpi/dx, v' = v - h dpi/dy and their divergence D."""
    u = base.u - h * (np.roll(pi_prev, -1, axis=AX_I) - pi_prev) / dx
    v = base.v - h * (np.roll(pi_prev, -1, axis=AX_J) - pi_prev) / dy
    d = (u - np.roll(u, 1, axis=AX_I)) / dx + (v - np.roll(v, 1, axis=AX_J)) / dy
    return u, v, d


def implicit_matrix(dz: np.ndarray, h: float, c: float, n: float) -> np.ndarray:
    """Banded form (for solve_banded, one sub- and one super-diagonal) of the
    interior-face system  (1 + h^2 N^2/4) wm_f - (h^2 c^2/4) d/dz(d wm/dz)_f."""
    nz = dz.shape[0]
    dzf = face_spacing(dz)                    # faces 1 .. nz-1 (index f-1)
    a = h * h * c * c / 4.0
    lo = a / (dzf * dz[:-1])                  # couples face f to face f-1 (through cell f-1)
    hi = a / (dzf * dz[1:])                   # couples face f to face f+1 (through cell f)
    ab = np.zeros((3, nz - 1))
    ab[1] = 1.0 + h * h * n * n / 4.0 + lo + hi
    ab[0, 1:] = -hi[:-1]                      # super-diagonal
    ab[2, :-1] = -lo[1:]                      # sub-diagonal
    return ab


def vertical(base: Fast, d: np.ndarray, dz: np.ndarray, h: float, c: float, n: float):
    """Trapezoidal vertical part of a stage: (w', b', pi') from the base and D."""
    nz = dz.shape[0]
    dzf = face_spacing(dz)[:, None, None]
    dzc = dz[:, None, None]
    w, b, pi = base.w, base.b, base.pi
    rhs = (w[1:nz] + (h / 2.0) * (-(pi[1:] - pi[:-1]) / dzf + b[1:nz])
           + (h * h * c * c / 4.0) * (d[1:] - d[:-1]) / dzf)
    wm = np.zeros_like(w)
    if nz > 1:
        ab = implicit_matrix(dz, h, c, n)
        shape = rhs.shape
        wm[1:nz] = solve_banded((1, 1), ab, rhs.reshape(nz - 1, -1)).reshape(shape)
    w_new = 2.0 * wm - w
    b_new = b - h * n * n * wm
    b_new[0] = 0.0
    b_new[nz] = 0.0
    w_new[0] = 0.0
    w_new[nz] = 0.0
    pi_new = pi - h * c * c * (d + (wm[1:] - wm[:-1]) / dzc)
    return w_new, b_new, pi_new


def stage(base: Fast, pi_prev: np.ndarray, dx: float, dy: float, dz: np.ndarray, h: float,
          c: float = C_SOUND, n: float = N_BV) -> Fast:
    u, v, d = horizontal(base, pi_prev, dx, dy, h)
    w, b, pi = vertical(base, d, dz, h, c, n)
    return Fast(u, v, w, b, pi)


def short_step(x: Fast, dx: float, dy: float, dz: np.ndarray, tau: float, c: float = C_SOUND,
               n: float = N_BV) -> Fast:
    """One RK2 (midpoint) HEVI short step of length tau."""
    s1 = stage(x, x.pi, dx, dy, dz, tau / 2.0, c, n)
    return stage(x, s1.pi, dx, dy, dz, tau, c, n)


def run(x: Fast, nsteps: int, dx: float, dy: float, dz: np.ndarray, tau: float, c: float = C_SOUND,
        n: float = N_BV) -> Fast:
    for _ in range(nsteps):
        x = short_step(x, dx, dy, dz, tau, c, n)
    return x


def energy(x: Fast, dx: float, dy: float, dz: np.ndarray, c: float = C_SOUND, n: float = N_BV) -> float:
    """Kinetic + available potential + elastic energy of the discrete state:
    (u^2 + v^2)/2 and pi^2/(2 c^2) per cell volume, (w^2 + b^2/N^2)/2 per
    interior-face volume dx dy dz_{k+1/2}."""
    nz = dz.shape[0]
    vc = dx * dy * dz[:, None, None]
    vf = dx * dy * face_spacing(dz)[:, None, None]
    e = 0.5 * np.sum((x.u ** 2 + x.v ** 2) * vc) + 0.5 * np.sum(x.pi ** 2 * vc) / (c * c)
    e += 0.5 * np.sum(x.w[1:nz] ** 2 * vf) + 0.5 * np.sum(x.b[1:nz] ** 2 * vf) / (n * n)
    return float(e)
