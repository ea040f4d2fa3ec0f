"""Small builders shared by the tests (no method arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_1802_05839_amd.inputs import Inputs, stretched_dz


def uniform_inputs(nx=16, ny=12, nz=8, dx=2000.0, dt=5.0, dz=None, u0=0.0, v0=0.0,
                   rho0=1.0, theta0=300.0, q0=0.01, theta_s=None, q_s=None, f0=0.0,
                   ch=0.0) -> Inputs:
    """Horizontally and vertically uniform fields with w = 0."""
    if dz is None:
        dz = stretched_dz(nz)
    dz = np.asarray(dz, dtype=np.float64)
    sh = (nz, ny, nx)
    return Inputs(nx=nx, ny=ny, nz=nz, dx=dx, dt=dt, dz=dz,
                  u=np.full(sh, u0), v=np.full(sh, v0), w=np.zeros((nz + 1, ny, nx)),
                  rho=np.full(sh, rho0), theta=np.full(sh, theta0), q=np.full(sh, q0),
                  theta_s=np.full((ny, nx), theta0 if theta_s is None else theta_s),
                  q_s=np.full((ny, nx), q0 if q_s is None else q_s),
                  f0=np.full((ny, nx), f0), ch=np.full((ny, nx), ch))


def nmax(a, ref):
    """Normalized max error max|a - ref| / max|ref|."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / (den if den > 0 else 1.0))
