"""Properties of the seeded input generators (CPU only)."""
import numpy as np

from paper_1802_05839_amd import inputs


def test_shapes_and_reproducibility():
    a = inputs.generate(20, 12, 7, seed=4)
    b = inputs.generate(20, 12, 7, seed=4)
    c = inputs.generate(20, 12, 7, seed=5)
    for name, arr in a.fields().items():
        np.testing.assert_array_equal(arr, getattr(b, name))
    assert not np.array_equal(a.u, c.u)
    assert a.u.shape == (7, 12, 20) and a.w.shape == (8, 12, 20) and a.f0.shape == (12, 20)
    assert a.dt == b.dt


def test_winds_are_discretely_nondivergent():
    inp = inputs.generate(48, 40, 12, seed=1)
    dz = inp.dz[:, None, None]
    div = ((inp.u - np.roll(inp.u, 1, axis=2)) / inp.dx + (inp.v - np.roll(inp.v, 1, axis=1)) / inp.dx
           + (inp.w[1:] - inp.w[:-1]) / dz)
    assert np.max(np.abs(div)) < 1e-15
    assert np.all(inp.w[0] == 0.0) and np.all(inp.w[-1] == 0.0)


def test_marginal_statistics():
    inp = inputs.generate(128, 128, 16, seed=2)
    assert 9.5 < inp.u.std() < 12.5 and 9.5 < inp.v.std() < 12.5
    assert 0.09 < inp.w[1:-1].std() < 0.11
    assert inp.q.max() <= 0.02 and inp.q.min() > 0.0
    assert abs(np.median(inp.q) - 0.006) < 0.0003
    assert np.all(inp.ch >= 0.005) and np.all(inp.ch < 0.02)
    np.testing.assert_allclose(inp.dz[0], 50.0)
    np.testing.assert_allclose(inp.dz[-1], 1000.0)
    assert 2.0 < inp.dt < 20.0


def test_crop_wraps_periodically():
    inp = inputs.generate(16, 10, 4, seed=3)
    c = inputs.crop(inp, 14, 8, 6, 5)
    np.testing.assert_array_equal(c.theta[:, 0, 0], inp.theta[:, 8, 14])
    np.testing.assert_array_equal(c.theta[:, 4, 5], inp.theta[:, (8 + 4) % 10, (14 + 5) % 16])
