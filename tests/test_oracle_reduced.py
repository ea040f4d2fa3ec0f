"""Pins of the reduced weather application oracle (CPU only).

Each pin fixes the rules of the paper's printed reduced application by a
value that follows from them independently of the oracle's code: a constant
field is a fixed point, single-cell impulses give the stencil weights and
which cells each rule reaches (including the corner columns, which take the
ring-column rule), a quadratic field gives the exact discrete Laplacian, and
the physics relaxes the boundary levels to the closed-form fixed point.
Dyadic values (nu = 1/8, integer fields) make the expected values exact.
"""
import numpy as np
import pytest

from oracle import reduced as rw
from paper_1802_05839_amd import inputs

NU = 0.125


def _impulse(nx, ny, nz, k, j, i):
    e = np.zeros(rw.shape(nx, ny, nz))
    e[k, j, i] = 1.0
    return e


def _nonzero(a):
    return {tuple(int(v) for v in idx): a[tuple(idx)] for idx in np.argwhere(a != 0)}


@pytest.mark.parametrize("nx,ny,nz", [(5, 4, 2), (6, 7, 3), (9, 5, 6)])
def test_constant_field_is_a_fixed_point_of_diffusion(nx, ny, nz):
    e = np.full(rw.shape(nx, ny, nz), 256.0)
    np.testing.assert_array_equal(rw.diffuse(e, NU), e)


def test_interior_impulse_gives_the_seven_point_weights():
    nx, ny, nz = 8, 7, 6
    out = rw.diffuse(_impulse(nx, ny, nz, 3, 4, 5), NU)
    want = {(3, 4, 5): 1 - 6 * NU, (3, 4, 4): NU, (3, 4, 6): NU, (3, 3, 5): NU, (3, 5, 5): NU,
            (2, 4, 5): NU, (4, 4, 5): NU}
    assert _nonzero(out) == want


def test_bottom_and_top_levels_use_five_neighbours():
    nx, ny, nz = 6, 6, 4
    out = rw.diffuse(_impulse(nx, ny, nz, 0, 3, 3), NU)
    assert _nonzero(out) == {(0, 3, 3): 1 - 5 * NU, (0, 3, 2): NU, (0, 3, 4): NU, (0, 2, 3): NU,
                             (0, 4, 3): NU, (1, 3, 3): NU}
    out = rw.diffuse(_impulse(nx, ny, nz, nz - 1, 2, 5), NU)
    assert _nonzero(out) == {(nz - 1, 2, 5): 1 - 5 * NU, (nz - 1, 2, 4): NU, (nz - 1, 2, 6): NU,
                             (nz - 1, 1, 5): NU, (nz - 1, 3, 5): NU, (nz - 2, 2, 5): NU}


def test_two_level_columns():
    # nz = 2: both levels take the five-neighbour rule, each other's vertical neighbour
    nx, ny = 4, 3
    out = rw.diffuse(_impulse(nx, ny, 2, 1, 2, 2), NU)
    assert out[1, 2, 2] == 1 - 5 * NU and out[0, 2, 2] == NU


def test_ring_row_reaches_the_opposite_row_and_not_the_corner_rule():
    nx, ny, nz = 5, 4, 3
    # a cell of ring row j = 0 at an interior i: itself, the opposite ring row,
    # and the interior cell above it (its j-1 neighbour)
    out = rw.diffuse(_impulse(nx, ny, nz, 1, 0, 2), NU)
    assert _nonzero(out) == {(1, 0, 2): 1 - 2 * NU, (1, ny + 1, 2): NU, (1, 1, 2): NU}


def test_corner_columns_take_the_ring_column_rule():
    nx, ny, nz = 5, 4, 3
    # corner (j = 0, i = 0): the column rule pairs it with (0, nx+1) only; the
    # row rule (written first, then overwritten) would have reached (ny+1, 0)
    out = rw.diffuse(_impulse(nx, ny, nz, 2, 0, 0), NU)
    assert _nonzero(out) == {(2, 0, 0): 1 - 2 * NU, (2, 0, nx + 1): NU}
    assert out[2, ny + 1, 0] == 0.0
    # a ring-column cell at an interior j reaches the opposite column and the
    # interior cell to its right
    out = rw.diffuse(_impulse(nx, ny, nz, 0, 2, nx + 1), NU)
    assert _nonzero(out) == {(0, 2, nx + 1): 1 - 2 * NU, (0, 2, 0): NU, (0, 2, nx): NU}


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_quadratic_field_gives_the_exact_laplacian(axis):
    # interior levels of interior columns: E + nu (sum of neighbours - 6 E)
    # and a quadratic along one axis has second difference 2
    nx, ny, nz = 7, 6, 7
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    e = ((k, j, i)[axis] ** 2).astype(np.float64)
    out = rw.diffuse(e, NU)
    inner = (slice(1, nz - 1), slice(1, ny + 1), slice(1, nx + 1))
    np.testing.assert_array_equal(out[inner], e[inner] + 2 * NU)


def test_physics_closed_forms():
    nx, ny, nz = 3, 2, 5
    e = np.full(rw.shape(nx, ny, nz), 300.0)
    surf, pbl = inputs.rw_boundary_fields(nx, ny)
    out = rw.run_physics(e, surf, pbl)
    np.testing.assert_array_equal(out[1:nz - 1], 300.0 + 0.1)
    b = 300.0 + 0.1
    np.testing.assert_allclose(out[0], b - 0.01 * (b - 330.0), rtol=1e-15)
    np.testing.assert_allclose(out[nz - 1], b - 0.01 * (b - 200.0), rtol=1e-15)
    assert out[0, 0, 0] > b > out[nz - 1, 0, 0]


def test_boundary_levels_relax_to_the_heat_well_fixed_point():
    # without diffusion the bottom level obeys e <- 0.99 (e + 0.1) + 0.01 * 330,
    # whose fixed point is 330 + 0.1 * 0.99 / 0.01 = 339.9 (and 209.9 on top)
    nx, ny, nz = 2, 2, 3
    e = np.zeros(rw.shape(nx, ny, nz))
    surf, pbl = inputs.rw_boundary_fields(nx, ny)
    for _ in range(6000):
        e = rw.run_physics(e, surf, pbl)
    np.testing.assert_allclose(e[0], 339.9, rtol=1e-9)
    np.testing.assert_allclose(e[nz - 1], 209.9, rtol=1e-9)
    np.testing.assert_allclose(e[1], 600.0, rtol=1e-9)   # 6000 steps of +0.1


def test_box_init_covers_the_middle_half():
    e = inputs.rw_box_init(8, 12, 4)
    assert e.shape == (4, 14, 10)
    assert set(np.unique(e)) == {0.0, 300.0}
    # 1-based interior indices 3..6 of 8, 4..9 of 12, 2..3 of 4; ring and outside are 0
    box = np.zeros_like(e, dtype=bool)
    box[1:3, 4:10, 3:7] = True
    np.testing.assert_array_equal(e == 300.0, box)


def test_step_is_physics_then_diffusion_and_rejects_flat_columns():
    nx, ny, nz = 6, 5, 4
    e = inputs.rw_box_init(nx, ny, nz)
    surf, pbl = inputs.rw_boundary_fields(nx, ny)
    np.testing.assert_array_equal(rw.step(e, surf, pbl, NU), rw.diffuse(rw.run_physics(e, surf, pbl), NU))
    with pytest.raises(ValueError):
        rw.diffuse(np.zeros(rw.shape(nx, ny, 1)), NU)


def _rule(i, j, k, nx, ny, nz, nu):
    """(centre weight, ordered neighbour list) of cell (i, j, k) by its class.

    The rules of the diffusion as mathematics, looked up per cell:
      ring column (i = 0 or nx + 1; the corner columns included):
          weight 1 - 2 nu; neighbours: the inner column, the opposite ring column
      ring row (j = 0 or ny + 1, i interior):
          weight 1 - 2 nu; neighbours: the inner row, the opposite ring row
      interior column, bottom or top level:
          weight 1 - 5 nu; neighbours i-1, i+1, j-1, j+1, the one level inside
      interior column, other levels:
          weight 1 - 6 nu; neighbours i-1, i+1, j-1, j+1, k-1, k+1
    """
    if i in (0, nx + 1):
        inner, opposite = (1, nx + 1) if i == 0 else (nx, 0)
        return 1.0 - 2.0 * nu, [(k, j, inner), (k, j, opposite)]
    if j in (0, ny + 1):
        inner, opposite = (1, ny + 1) if j == 0 else (ny, 0)
        return 1.0 - 2.0 * nu, [(k, inner, i), (k, opposite, i)]
    horizontal = [(k, j, i - 1), (k, j, i + 1), (k, j - 1, i), (k, j + 1, i)]
    if k == 0:
        return 1.0 - 5.0 * nu, horizontal + [(1, j, i)]
    if k == nz - 1:
        return 1.0 - 5.0 * nu, horizontal + [(nz - 2, j, i)]
    return 1.0 - 6.0 * nu, horizontal + [(k - 1, j, i), (k + 1, j, i)]


def _diffuse_by_rules(e, nu, rng):
    """Every cell from its rule, visited in a random order."""
    nz, nyp, nxp = e.shape
    ny, nx = nyp - 2, nxp - 2
    out = np.full_like(e, np.nan)
    for flat in rng.permutation(e.size):
        k, j, i = np.unravel_index(flat, e.shape)
        w, nbs = _rule(int(i), int(j), int(k), nx, ny, nz, nu)
        s = e[nbs[0]]
        for nb in nbs[1:]:
            s = s + e[nb]
        out[k, j, i] = e[k, j, i] * w + nu * s
    return out


@pytest.mark.parametrize("nx,ny,nz", [(3, 2, 2), (4, 5, 3), (6, 3, 5)])
def test_diffusion_equals_per_cell_rules_bitwise(nx, ny, nz):
    # brute force on tiny grids with random values and a non-dyadic nu: the
    # vectorised oracle equals every cell's rule (looked up from its class,
    # cells visited in random order) to the last bit
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    e = rng.uniform(-50.0, 400.0, rw.shape(nx, ny, nz))
    np.testing.assert_array_equal(rw.diffuse(e, 0.137), _diffuse_by_rules(e, 0.137, rng))


def test_physics_equals_per_cell_rule_bitwise():
    # each cell from the physics rule of its level, cells in random order:
    #   x = E + 0.1;  bottom level: x - 0.01 (x - surface);  top level: x - 0.01 (x - boundary layer)
    rng = np.random.default_rng(3)
    nx, ny, nz = 4, 3, 5
    e = rng.uniform(0.0, 400.0, rw.shape(nx, ny, nz))
    surf = rng.uniform(280.0, 340.0, (ny + 2, nx + 2))
    pbl = rng.uniform(180.0, 240.0, (ny + 2, nx + 2))
    want = np.full_like(e, np.nan)
    for flat in rng.permutation(e.size):
        k, j, i = np.unravel_index(flat, e.shape)
        x = e[k, j, i] + 0.1
        if k == 0:
            x = x - 0.01 * (x - surf[j, i])
        if k == nz - 1:
            x = x - 0.01 * (x - pbl[j, i])
        want[k, j, i] = x
    np.testing.assert_array_equal(rw.run_physics(e, surf, pbl), want)
