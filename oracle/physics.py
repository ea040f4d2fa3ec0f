"""FP64 oracle of the column physics (test infrastructure only).

What the paper fixes: physics runs after the dynamical core, column by column,
with no interaction between columns until the next dycore call (section
"Architecture-Dependant Parallelization Granularity"); the K direction is
sequential because of loop-carried dependencies (section "The ASUCA Weather
Prediction Model"); radiation is a per-column loop over k and the boundary
exchange relaxes the lowest level toward a boundary value with a transfer
velocity (the reduced application's radiation and heat-exchange routines,
appendix "Reduced Weather: Radiation" / "Heat Exchange").  The processes are
boundary-layer mixing and radiation (section "Hybrid ASUCA Strong Scaling GPU
Results").

Readings taken (the paper prints no equations for them):

* Parallel split: diffusion and radiation both start from the post-dycore
  state (rho+, theta+, q+).
* K_z at interface k+1/2 from the shear of the cell-centred winds:
  K = K_min + l^2 |dU/dz|; alpha = dt rho_{k+1/2} K / dz_{k+1/2}; m_k = rho_k dz_k.
* Implicit (backward Euler) vertical diffusion in delta form with a Robin
  surface condition (beta = dt rho_0 C_h toward the surface value) and a
  zero-flux lid; theta and q share the matrix.
* Transmissivity: dtau_k = kappa_q rho_k max(q_k, 0) dz_k, tau the suffix sum
  from the lid down, T = exp(-tau), F = F0 T at interfaces, heating
  H_k = (F_{k+1/2} - F_{k-1/2}) / (c_p m_k).
* theta = theta+ + delta_theta + dt H, q = q+ + delta_q; the tendencies are
  delta_theta/dt + H and delta_q/dt.
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np

from .params import DEFAULT, Params


def thomas(a: np.ndarray, b: np.ndarray, c: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Solve a tridiagonal system by the Thomas algorithm (no pivoting).

    Row k:  a[k] x[k-1] + b[k] x[k] + c[k] x[k+1] = d[k]  (a[0], c[-1] unused).
    The leading axis is k; any trailing axes are independent columns.
    Forward elimination runs k = 0 .. n-1, back substitution n-1 .. 0.
    """
    n = b.shape[0]
    cp = np.empty_like(b)
    dp = np.empty_like(d)
    cp[0] = c[0] / b[0]
    dp[0] = d[0] / b[0]
    for k in range(1, n):
        den = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / den
        dp[k] = (d[k] - a[k] * dp[k - 1]) / den
    x = np.empty_like(d)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


class Coeffs(NamedTuple):
    alpha: np.ndarray     # (nz+1, ...) interface exchange, alpha[k] below level k; 0 at ground/lid
    m: np.ndarray         # (nz, ...) layer mass per area
    beta: np.ndarray      # (...) surface exchange


def centred_winds(u: np.ndarray, v: np.ndarray):
    """Cell-centre winds: mean of the two C-grid faces of each cell."""
    ub = (np.roll(u, 1, axis=2) + u) / 2.0
    vb = (np.roll(v, 1, axis=1) + v) / 2.0
    return ub, vb


def diffusion_coeffs(rho: np.ndarray, u: np.ndarray, v: np.ndarray, ch: np.ndarray,
                     dz: np.ndarray, dt: float, p: Params = DEFAULT) -> Coeffs:
    """Interface exchange alpha, layer mass m and surface exchange beta."""
    nz = rho.shape[0]
    dzc = dz.reshape((nz,) + (1,) * (rho.ndim - 1))
    ub, vb = centred_winds(u, v)
    dzi = (dzc[:-1] + dzc[1:]) / 2.0                   # interface spacing k+1/2
    shear = np.sqrt((ub[1:] - ub[:-1]) ** 2 + (vb[1:] - vb[:-1]) ** 2) / dzi
    kz = p.k_min + p.mix_len ** 2 * shear
    rho_i = (rho[:-1] + rho[1:]) / 2.0
    alpha = np.zeros((nz + 1,) + rho.shape[1:])
    alpha[1:nz] = dt * rho_i * kz / dzi
    m = rho * dzc
    beta = dt * rho[0] * ch
    return Coeffs(alpha, m, beta)


def dominance_ratio(cf: Coeffs) -> np.ndarray:
    """Per-column max_k (alpha_{k-1/2} + alpha_{k+1/2}) / m_k."""
    r = (cf.alpha[:-1] + cf.alpha[1:]) / cf.m
    return r.max(axis=0)


def implicit_diffusion(phi: np.ndarray, phi_s: np.ndarray, cf: Coeffs) -> np.ndarray:
    """Delta of one backward-Euler vertical diffusion step (delta form).

    Row k: -a_{k-1/2} d_{k-1} + (m_k + a_{k-1/2} + a_{k+1/2} + beta[k=0]) d_k - a_{k+1/2} d_{k+1}
           = a_{k+1/2}(phi_{k+1} - phi_k) - a_{k-1/2}(phi_k - phi_{k-1}) + beta[k=0](phi_s - phi_0)
    """
    nz = phi.shape[0]
    al, ah = cf.alpha[:-1], cf.alpha[1:]          # below / above each level
    sub = -al
    sup = -ah
    diag = cf.m + al + ah
    diag = diag.copy()
    diag[0] = diag[0] + cf.beta
    up = np.zeros_like(phi)
    dn = np.zeros_like(phi)
    up[:-1] = phi[1:] - phi[:-1]                  # phi_{k+1} - phi_k
    dn[1:] = phi[1:] - phi[:-1]                   # phi_k - phi_{k-1}
    rhs = ah * up - al * dn
    rhs = rhs.copy()
    rhs[0] = rhs[0] + cf.beta * (phi_s - phi[0])
    return thomas(sub, diag, sup, rhs)


def radiation(rho: np.ndarray, q: np.ndarray, f0: np.ndarray, dz: np.ndarray,
              p: Params = DEFAULT):
    """Heating rate H (nz, ...) and interface transmissivity T (nz+1, ...).

    T[f] is the transmissivity of the face below level f (T[nz] = 1 at the lid),
    tau[f] = sum of dtau over the levels at and above f, accumulated from the lid.
    """
    nz = rho.shape[0]
    dzc = dz.reshape((nz,) + (1,) * (rho.ndim - 1))
    dtau = p.kappa_q * rho * np.maximum(q, 0.0) * dzc
    tau = np.zeros((nz + 1,) + rho.shape[1:])
    for f in range(nz - 1, -1, -1):
        tau[f] = tau[f + 1] + dtau[f]
    trans = np.exp(-tau)
    flux = f0 * trans
    m = rho * dzc
    heat = (flux[1:] - flux[:-1]) / (p.cp * m)
    return heat, trans


class PhysicsOut(NamedTuple):
    theta: np.ndarray
    q: np.ndarray
    t_theta: np.ndarray     # tendency of theta [K/s]
    t_q: np.ndarray         # tendency of q [1/s]
    ratio: np.ndarray       # per-column dominance ratio max_k r_k


def column_physics(rho, theta, q, u, v, theta_s, q_s, f0, ch, dz, dt: float,
                   p: Params = DEFAULT) -> PhysicsOut:
    """Implicit vertical diffusion of theta and q plus radiative heating."""
    cf = diffusion_coeffs(rho, u, v, ch, dz, dt, p)
    d_theta = implicit_diffusion(theta, theta_s, cf)
    d_q = implicit_diffusion(q, q_s, cf)
    heat, _ = radiation(rho, q, f0, dz, p)
    theta_new = theta + d_theta + dt * heat
    q_new = q + d_q
    return PhysicsOut(theta_new, q_new, d_theta / dt + heat, d_q / dt, dominance_ratio(cf))
