"""Integrity of the long-horizon oracle fixtures (CPU): the sample index is
the generator's seeded draw, the stored statistics bound the samples, and
the short-horizon end of the same recipe reproduces the oracle exactly (the
fixture script's problem and sampling, run for 2 steps on the crop grid,
equal a direct oracle run at the same cells)."""
import os

import numpy as np
import pytest

from oracle import step
from tests.golden import make_long_horizon as mk

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("cfg", sorted(mk.CASES))
def test_fixture_is_consistent(cfg):
    fx = np.load(os.path.join(HERE, f"long_horizon_{cfg}.npz"), allow_pickle=False)
    assert int(fx["nsteps"]) == mk.CASES[cfg]
    idx = fx["index"]
    from paper_1802_05839_amd import inputs
    c = inputs.CONFIGS[cfg]
    shape = (c["nz"], c["ny"], c["nx"])
    np.testing.assert_array_equal(idx, mk.sample_index(shape))
    assert idx.size == mk.NSAMPLE and np.all(np.diff(idx) > 0)
    for name in ("rho", "theta", "q"):
        smp = fx[f"{name}_sample"]
        norm, amax, vmax, vmin = fx[f"{name}_stats"]
        assert np.all(np.isfinite(smp))
        assert np.max(np.abs(smp)) <= amax and np.max(smp) <= vmax and np.min(smp) >= vmin
        assert np.linalg.norm(smp) <= norm and vmax > vmin


def test_fixture_recipe_matches_oracle_on_a_short_run():
    # the recipe's problem, 2 steps by the whole-grid oracle and by the j-slab
    # driver the fixture script uses
    from oracle import slabs
    inp = mk.f32_problem("crop")
    ref = step.run(inp, 2)
    idx = mk.sample_index(ref.rho.shape)
    got = slabs.run(inp, 2)
    for a, b in zip((ref.rho, ref.theta, ref.q), (got.rho, got.theta, got.q)):
        np.testing.assert_array_equal(a.ravel()[idx], b.ravel()[idx])
