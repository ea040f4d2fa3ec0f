"""The threaded j-slab driver of the oracle equals the plain whole-grid run
bit for bit (CPU only)."""
import numpy as np
import pytest

from oracle import slabs, step
from paper_1802_05839_amd import inputs


@pytest.mark.parametrize("nx,ny,nz,nslab,threads", [(24, 20, 6, 3, 2), (17, 13, 5, 13, 4), (16, 31, 4, 1, 1),
                                                    (20, 9, 5, 2, 3)])
def test_slab_run_equals_whole_grid_bitwise(nx, ny, nz, nslab, threads):
    inp = inputs.generate(nx, ny, nz, seed=nx + ny)
    want = step.run(inp, 3)
    got = slabs.run(inp, 3, threads=threads, slabs=nslab)
    for a, b in zip(want, got):
        np.testing.assert_array_equal(a, b)


def test_slab_run_dycore_only_bitwise():
    inp = inputs.generate(18, 14, 5, seed=5)
    want = step.run(inp, 2, physics_on=False)
    got = slabs.run(inp, 2, threads=2, slabs=4, physics_on=False)
    for a, b in zip(want, got):
        np.testing.assert_array_equal(a, b)
