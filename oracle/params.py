"""Constants of the oracle (test infrastructure only).

The paper names the processes but prints no coefficients for them: a C-grid
finite-volume dycore with a third-order Runge-Kutta long step (section "The
ASUCA Weather Prediction Model"), and radiation and boundary-layer physics
after MSM0705 (the comparison table in section "Comparison to Previous Work";
module impact in section "Hybrid ASUCA Strong Scaling GPU Results").  The
values below are the readings this implementation adopts.  The GPU library
holds its own copy and reports it back; a test asserts the two agree.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass(frozen=True)
class Params:
    gamma4: float = 2.0 ** -8     # biharmonic strength: K4 = gamma4 * dx^4 / dt
    k_min: float = 0.1            # background vertical diffusivity [m^2/s]
    mix_len: float = 50.0         # mixing length l in K = K_min + l^2 |dU/dz| [m]
    kappa_q: float = 0.02         # absorber mass extinction coefficient [m^2/kg]
    cp: float = 1004.0            # heat capacity of air [J/(kg K)]
    t_dd: float = 64.0            # weak-dominance threshold for the FP64 elimination

    def k4(self, dx: float, dt: float) -> float:
        return self.gamma4 * dx ** 4 / dt


DEFAULT = Params()
