"""FP64 oracle of the kinematic finite-volume dycore (test infrastructure only).

What the paper fixes (section "The ASUCA Weather Prediction Model"): a
structured C-grid, finite volumes in three dimensions with I and J
interchangeable horizontal directions and K treated separately, and a
third-order Runge-Kutta long step (the Wicker-Skamarock scheme the paper
cites).  It prints no equations; the readings taken here are:

* Kinematic transport: winds u, v, w are frozen at C-grid faces; the
  prognostic fields are density rho and the mixing ratios theta and q.
* Face values are third-order upwind-biased, with the coefficients taken in
  index space.  In k the two faces next to the ground and the lid use the
  centred average; the ground and lid faces carry no flux.
* The tracer update is written in increment (mixing-ratio) form, which is the
  conservative update rearranged so that a constant field gives exactly zero
  increment.
* Horizontal biharmonic diffusion acts on theta and q (not rho), as a
  density-weighted flux of the gradient of the 5-point Laplacian, with
  ``K4 = gamma4 dx^4 / dt``.
* RK3 stages use h = dt/3, dt/2, dt, each relative to the step's base state.

Array conventions: cell fields are ``(nz, ny, nx)`` float64, i fastest; u is
the east face of each cell, v the north face; w is ``(nz+1, ny, nx)`` with
``w[k]`` the face below level k.  Horizontal boundaries are periodic.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np

AX_K, AX_J, AX_I = 0, 1, 2


class State(NamedTuple):
    rho: np.ndarray
    theta: np.ndarray
    q: np.ndarray


def nb(a: np.ndarray, d: int, axis: int) -> np.ndarray:
    """Periodic neighbour: element ``index + d`` along ``axis``."""
    return np.roll(a, -d, axis=axis)


def upwind3_face(phi: np.ndarray, vel: np.ndarray, axis: int) -> np.ndarray:
    """Third-order upwind face value at ``index + 1/2`` along a periodic axis.

    Velocity >= 0 takes the stencil (i-1, i, i+1) with weights (-1, 5, 2)/6;
    velocity < 0 the mirror image (2, 5, -1)/6 on (i, i+1, i+2).  Written in
    increment form so that the weights act on differences:
    phi_i + (2 (phi_{i+1} - phi_i) + (phi_i - phi_{i-1})) / 6.
    """
    pm1, p0, p1, p2 = nb(phi, -1, axis), phi, nb(phi, 1, axis), nb(phi, 2, axis)
    pos = p0 + (2.0 * (p1 - p0) + (p0 - pm1)) / 6.0
    neg = p1 + (2.0 * (p0 - p1) + (p1 - p2)) / 6.0
    return np.where(vel >= 0.0, pos, neg)


def vertical_faces(phi: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Face values at the nz+1 face levels; index f is the face below level f.

    Faces 0 and nz (ground, lid) are set to 0 and never carry flux.  Faces 1
    and nz-1 (next to them) take the centred average; faces 2..nz-2 take the
    third-order upwind value with the sign of w at that face.
    """
    nz = phi.shape[0]
    out = np.zeros((nz + 1,) + phi.shape[1:])
    for f in range(1, nz):
        lo, hi = f - 1, f          # the face lies between levels lo and hi
        if f == 1 or f == nz - 1:
            out[f] = phi[lo] + (phi[hi] - phi[lo]) / 2.0
        else:
            pos = phi[lo] + (2.0 * (phi[hi] - phi[lo]) + (phi[lo] - phi[lo - 1])) / 6.0
            neg = phi[hi] + (2.0 * (phi[lo] - phi[hi]) + (phi[hi] - phi[hi + 1])) / 6.0
            out[f] = np.where(w[f] >= 0.0, pos, neg)
    return out


def vertical_flux(w: np.ndarray, rho_face: np.ndarray) -> np.ndarray:
    """Mass flux w * rho_f at the nz+1 face levels, zero at the ground and lid."""
    F = w * rho_face
    F[0] = 0.0
    F[-1] = 0.0
    return F


def laplacian5(phi: np.ndarray, dx: float, dy: float) -> np.ndarray:
    """Horizontal 5-point Laplacian."""
    return ((nb(phi, 1, AX_I) - 2.0 * phi + nb(phi, -1, AX_I)) / dx ** 2
            + (nb(phi, 1, AX_J) - 2.0 * phi + nb(phi, -1, AX_J)) / dy ** 2)


def biharmonic_tendency(phi: np.ndarray, rho: np.ndarray, k4: float, dx: float,
                        dy: float) -> np.ndarray:
    """Density-weighted biharmonic tendency B of d(rho phi)/dt.

    Lambda = Laplacian(phi);  G_{i+1/2} = K4 (rho_i + rho_{i+1})/2 (Lambda_{i+1} - Lambda_i)/dx;
    B = -[(G_{i+1/2} - G_{i-1/2})/dx + (G_{j+1/2} - G_{j-1/2})/dy].
    """
    lam = laplacian5(phi, dx, dy)
    gx = k4 * ((rho + nb(rho, 1, AX_I)) / 2.0) * (nb(lam, 1, AX_I) - lam) / dx
    gy = k4 * ((rho + nb(rho, 1, AX_J)) / 2.0) * (nb(lam, 1, AX_J) - lam) / dy
    return -((gx - nb(gx, -1, AX_I)) / dx + (gy - nb(gy, -1, AX_J)) / dy)


def stage(base: State, star: State, u: np.ndarray, v: np.ndarray, w: np.ndarray,
          dx: float, dy: float, dz: np.ndarray, h: float, k4: float) -> State:
    """One RK stage: new = base + h * L(star), in increment form.

    rho_new = rho_n - h D(rho),  D = divergence of the mass fluxes
    F = (u rho*_f, v rho*_f, w rho*_f).  For phi in (theta, q):
      A = -[ F_{+}(phi*_f+ - phi_n) - F_{-}(phi*_f- - phi_n) ] per direction / spacing
      phi_new = phi_n + h (A + B(phi*)) / rho_new.
    """
    dzc = dz[:, None, None]
    rf_x = upwind3_face(star.rho, u, AX_I)
    rf_y = upwind3_face(star.rho, v, AX_J)
    rf_z = vertical_faces(star.rho, w)
    fx = u * rf_x                       # east-face flux of each cell
    fy = v * rf_y                       # north-face flux
    fz = vertical_flux(w, rf_z)         # (nz+1) faces
    fx_w = nb(fx, -1, AX_I)             # west face of cell i = east face of i-1
    fy_s = nb(fy, -1, AX_J)
    div = (fx - fx_w) / dx + (fy - fy_s) / dy + (fz[1:] - fz[:-1]) / dzc
    rho_new = base.rho - h * div

    out = [rho_new]
    for name in ("theta", "q"):
        ps = getattr(star, name)
        pn = getattr(base, name)
        px = upwind3_face(ps, u, AX_I)
        py = upwind3_face(ps, v, AX_J)
        pz = vertical_faces(ps, w)
        ax = (fx * (px - pn) - fx_w * (nb(px, -1, AX_I) - pn)) / dx
        ay = (fy * (py - pn) - fy_s * (nb(py, -1, AX_J) - pn)) / dy
        az = (fz[1:] * (pz[1:] - pn) - fz[:-1] * (pz[:-1] - pn)) / dzc
        a = -(ax + ay + az)
        b = biharmonic_tendency(ps, star.rho, k4, dx, dy)
        out.append(pn + h * (a + b) / rho_new)
    return State(*out)


def rk3(s: State, u, v, w, dx: float, dy: float, dz: np.ndarray, dt: float,
        k4: float) -> State:
    """Wicker-Skamarock RK3: stages h = dt/3, dt/2, dt from the base state."""
    s1 = stage(s, s, u, v, w, dx, dy, dz, dt / 3.0, k4)
    s2 = stage(s, s1, u, v, w, dx, dy, dz, dt / 2.0, k4)
    return stage(s, s2, u, v, w, dx, dy, dz, dt, k4)
