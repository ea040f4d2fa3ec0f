"""Global mass sums (test infrastructure only).

Totals M_rho = sum rho V, M_theta = sum rho theta V, M_q = sum rho q V with
V = dx dy dz_k, summed exactly rounded by ``math.fsum``.  The paper reduces
with an OpenACC ``reduction(+:...)`` clause (appendix "Parallel Region
Construct"); this is the plain definition of the same global sum.
"""
from __future__ import annotations

import math

import numpy as np


def mass_sums(rho: np.ndarray, theta: np.ndarray, q: np.ndarray, dx: float, dy: float,
              dz: np.ndarray) -> np.ndarray:
    vol = (dx * dy * np.asarray(dz, dtype=np.float64))[:, None, None]
    m = rho * vol
    return np.array([math.fsum(m.ravel()),
                     math.fsum((m * theta).ravel()),
                     math.fsum((m * q).ravel())])
