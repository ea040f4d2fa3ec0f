"""Pins of the surrogate oracle (CPU only)."""
import numpy as np
import pytest

from oracle import mlp


def test_splitmix64_reference_sequence():
    # The generator's output for state increments 0, 1, 2 of the golden gamma
    # (seed 0): the published reference values of SplitMix64.
    gamma = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = mlp.splitmix64(np.arange(3, dtype=np.uint64) * gamma)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_bf16_round_to_nearest_even():
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6,
             1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7, -(1 + 2 ** -7 + 2 ** -9): -(1 + 2 ** -7),
             2 ** -130: 2 ** -130, 0.0: 0.0}
    for x, want in cases.items():
        assert mlp.bf16(x) == want, (x, mlp.bf16(x), want)
    r = np.random.default_rng(0).normal(size=10000)
    b = mlp.bf16(r)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2.0 ** -8)
    assert np.all(mlp.bf16(b) == b)


def test_he_uniform_bounds_and_zero_bias():
    p = mlp.init_params(7, n_in=40, n_hid=64, n_out=10)
    for k, fan in (("W1", 40), ("W2", 64), ("W3", 64)):
        bound = np.float32(np.sqrt(6.0 / fan))
        assert np.all(np.abs(p[k]) <= bound)
        assert abs(p[k].mean()) < 0.1 * bound
        assert np.std(p[k]) == pytest.approx(bound / np.sqrt(3.0), rel=0.1)
    assert all(np.all(p[b] == 0) for b in ("b1", "b2", "b3"))
    q = mlp.init_params(8, n_in=40, n_hid=64, n_out=10)
    assert not np.array_equal(p["W1"], q["W1"])
    np.testing.assert_array_equal(p["W2"], mlp.init_params(7, n_in=40, n_hid=64, n_out=10)["W2"])


def test_gradients_match_central_differences():
    # P10: the analytic gradient (no BF16 rounding) against central finite
    # differences of the loss, every parameter of a small network.
    rng = np.random.default_rng(1)
    n_in, n_hid, n_out, b = 7, 9, 5, 6
    p = {"W1": rng.normal(size=(n_hid, n_in)), "b1": rng.normal(size=n_hid) * 0.1,
         "W2": rng.normal(size=(n_hid, n_hid)), "b2": rng.normal(size=n_hid) * 0.1,
         "W3": rng.normal(size=(n_out, n_hid)), "b3": rng.normal(size=n_out) * 0.1}
    x = rng.normal(size=(b, n_in))
    t = rng.normal(size=(b, n_out))
    y, cache = mlp.forward(p, x, bf=False)
    g = mlp.backward(cache, y, t, bf=False)
    h = 1e-6
    worst = 0.0
    for k, a in p.items():
        num = np.zeros_like(a)
        for idx in np.ndindex(a.shape):
            old = a[idx]
            a[idx] = old + h
            lp = mlp.loss(mlp.forward(p, x, bf=False)[0], t)
            a[idx] = old - h
            lm = mlp.loss(mlp.forward(p, x, bf=False)[0], t)
            a[idx] = old
            num[idx] = (lp - lm) / (2 * h)
        worst = max(worst, np.max(np.abs(num - g[k])) / max(np.max(np.abs(g[k])), 1e-12))
    assert worst <= 1e-6, worst


def test_adam_closed_form_two_parameters():
    # P11: from zero moments, one step moves each parameter by
    # lr * g / (|g| + eps); a second step with gradient g2 by
    # lr * m2hat / (sqrt(v2hat) + eps) with the moments written out.
    p = {"w": np.array([0.5, -2.0])}
    g1 = {"w": np.array([0.2, -4.0])}
    st = mlp.adam_init(p)
    p1, st = mlp.adam_step(p, g1, st, lr=0.01)
    np.testing.assert_allclose(p1["w"], [0.5 - 0.01 * 0.2 / (0.2 + 1e-8), -2.0 + 0.01 * 4.0 / (4.0 + 1e-8)],
                               rtol=1e-15)
    g2 = {"w": np.array([-0.1, 1.0])}
    p2, st = mlp.adam_step(p1, g2, st, lr=0.01)
    m2 = 0.9 * 0.1 * np.array([0.2, -4.0]) + 0.1 * np.array([-0.1, 1.0])
    v2 = 0.999 * 0.001 * np.array([0.04, 16.0]) + 0.001 * np.array([0.01, 1.0])
    step2 = 0.01 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(p2["w"], p1["w"] - step2, rtol=1e-13)


def test_bf16_forward_close_to_exact_forward():
    rng = np.random.default_rng(2)
    p = mlp.init_params(3, n_in=32, n_hid=48, n_out=8)
    x = rng.normal(size=(20, 32))
    y1, _ = mlp.forward(p, x, bf=True)
    y0, _ = mlp.forward(p, x, bf=False)
    assert np.linalg.norm(y1 - y0) / np.linalg.norm(y0) < 2e-2


def test_feature_layout():
    nz, ny, nx = 3, 2, 4
    a = np.arange(nz * ny * nx, dtype=float).reshape(nz, ny, nx)
    u = np.zeros((nz, ny, nx))
    u[1, 1, 2] = 4.0                         # east face of cell (i=2, j=1): centre mean 2 at i=2 and i=3
    f = mlp.features(a + 100, a + 200, a + 300, u, np.zeros_like(u), np.full((ny, nx), 1.0),
                      np.full((ny, nx), 2.0), np.arange(8.0).reshape(ny, nx), np.full((ny, nx), 4.0))
    assert f.shape == (8, 5 * nz + 4)
    c = 2 + nx * 1                           # column i=2, j=1
    np.testing.assert_array_equal(f[c, 0:3], a[:, 1, 2] + 200 - 300)  # theta - 300 K
    np.testing.assert_array_equal(f[c, 3:6], a[:, 1, 2] + 300)      # q
    np.testing.assert_array_equal(f[c, 6:9], a[:, 1, 2] + 100)      # rho
    assert f[c, 9 + 1] == 2.0 and f[c + 1, 9 + 1] == 2.0 and f[c - 1, 9 + 1] == 0.0
    np.testing.assert_array_equal(f[:, 5 * nz + 2], np.arange(8.0))  # F0, column order i + nx j


def test_norm_stats_constant_feature():
    x = np.column_stack([np.full(10, 3.0), np.arange(10.0)])
    y = np.column_stack([np.arange(10.0), 2 * np.arange(10.0)])
    n = mlp.norm_stats(x, y)
    assert n.x_std[0] == 1.0 and n.x_mean[0] == 3.0
    assert n.sigma_theta == pytest.approx(np.arange(10.0).std())
    assert n.sigma_q == pytest.approx(2 * np.arange(10.0).std())


def test_sample_mask_and_judge():
    m = mlp.sample_mask(123, 5, 200000)
    assert 0.008 < m.mean() < 0.012
    assert not np.array_equal(m, mlp.sample_mask(123, 6, 200000))
    nz = 4
    ref = np.zeros((10, 2 * nz))
    hat = ref.copy()
    hat[:, :nz] = 0.3                       # constant error 0.3 in theta, 0 in q
    mask = np.zeros(10, bool)
    mask[[1, 4]] = True
    r_t, r_q, fb = mlp.judge(hat, ref, mask, sigma_theta=6.0, sigma_q=1.0)
    assert r_t == pytest.approx(0.3) and r_q == 0.0
    assert fb is False                      # 0.3 == 0.05 * 6 is not strictly greater
    assert mlp.judge(hat, ref, mask, sigma_theta=5.9, sigma_q=1.0)[2] is True
