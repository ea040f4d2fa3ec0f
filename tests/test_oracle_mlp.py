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


def _feature_state(seed, nz=6, ny=3, nx=5):
    rng = np.random.default_rng(seed)
    sh = (nz, ny, nx)
    return (np.full(sh, 1.1), 300 + rng.normal(0, 2, sh), rng.uniform(0, 0.02, sh),
            rng.normal(0, 10, sh), rng.normal(0, 10, sh), 300 + rng.normal(0, 1, (ny, nx)),
            rng.uniform(0, 0.02, (ny, nx)), np.arange(float(ny * nx)).reshape(ny, nx),
            np.full((ny, nx), 4.0))


def test_feature_profiles_reconstruct_theta_and_q():
    """Cumulative sums of profiles 1 and 2 give theta - 300 K and q back."""
    rho, th, q, u, v, ts, qs, f0, ch = _feature_state(1)
    nz = th.shape[0]
    f = mlp.features(rho, th, q, u, v, ts, qs, f0, ch)
    assert f.shape == (th[0].size, 5 * nz + 4)
    np.testing.assert_allclose(np.cumsum(f[:, :nz], axis=1), (th - 300).reshape(nz, -1).T, atol=1e-12)
    np.testing.assert_allclose(np.cumsum(f[:, nz:2 * nz], axis=1), q.reshape(nz, -1).T, atol=1e-15)
    np.testing.assert_array_equal(f[:, 5 * nz + 2], f0.ravel())          # column order i + nx j
    np.testing.assert_allclose(f[:, 5 * nz], (ts - 300).ravel(), atol=1e-12)
    np.testing.assert_array_equal(f[:, 5 * nz + 3], 4.0)


def test_feature_shear_closed_form_and_invariances():
    """Linear wind profiles: speed at k = 0 and a constant shear |(a, b)|;
    a uniform wind added to every level changes only the k = 0 speed; a
    uniform theta shift changes only the first feature; profiles 4 and 5 are
    the shear times the theta and q differences."""
    rho, th, q, _, _, ts, qs, f0, ch = _feature_state(2)
    nz, ny, nx = th.shape
    k = np.arange(nz, dtype=float)[:, None, None] * np.ones((1, ny, nx))
    a, b, c, d = 3.0, -4.0, 6.0, 8.0
    u, v = a * k + c, b * k + d                 # uniform in i, j: face and centre values agree
    f = mlp.features(rho, th, q, u, v, ts, qs, f0, ch)
    sp = f[:, 2 * nz:3 * nz]
    np.testing.assert_allclose(sp[:, 0], 10.0, rtol=1e-15)          # |(6, 8)|
    np.testing.assert_allclose(sp[:, 1:], 5.0, rtol=1e-15)          # |(3, -4)|
    g = mlp.features(rho, th + 7.5, q, u + 20.0, v - 3.0, ts, qs, f0, ch)
    same = np.ones(f.shape[1], bool)
    same[[0, 2 * nz]] = False                   # theta'_0 and the k = 0 speed
    np.testing.assert_allclose(g[:, same], f[:, same], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g[:, 2 * nz], np.hypot(c + 20.0, d - 3.0), rtol=1e-15)
    np.testing.assert_allclose(g[:, 0], f[:, 0] + 7.5, rtol=1e-15)
    np.testing.assert_allclose(f[:, 3 * nz + 1:4 * nz], sp[:, 1:] * f[:, 1:nz], rtol=1e-14)
    np.testing.assert_allclose(f[:, 4 * nz + 1:5 * nz], sp[:, 1:] * f[:, nz + 1:2 * nz], rtol=1e-14)
    assert np.all(f[:, 3 * nz] == 0) and np.all(f[:, 4 * nz] == 0)


def test_feature_face_staggering():
    """An east-face u perturbation of cell (i, j) at level k moves the
    cell-centred wind of cells i and i + 1 only, so only their speed/shear
    features at levels k and k + 1 change."""
    rho, th, q, u, v, ts, qs, f0, ch = _feature_state(3)
    nz, ny, nx = th.shape
    kk, jj, ii = 2, 1, nx - 1                   # the east face of the last cell wraps to i = 0
    u2 = u.copy()
    u2[kk, jj, ii] += 5.0
    f = mlp.features(rho, th, q, u, v, ts, qs, f0, ch)
    g = mlp.features(rho, th, q, u2, v, ts, qs, f0, ch)
    changed = np.argwhere(np.abs(g - f) > 0)
    cols = {ii + nx * jj, 0 + nx * jj}
    assert {int(c) for c in changed[:, 0]} == cols
    levels = {int(x) % nz for x in changed[:, 1]}
    assert levels == {kk, kk + 1}
    assert all(2 * nz <= x < 5 * nz for x in changed[:, 1])


def test_norm_stats_constant_feature():
    x = np.column_stack([np.full(10, 3.0), np.arange(10.0)])
    y = np.column_stack([np.arange(10.0), 2 * np.arange(10.0)])
    n = mlp.norm_stats(x, y)
    assert n.x_std[0] == 1.0 and n.x_mean[0] == 3.0
    assert n.sigma_theta == pytest.approx(np.arange(10.0).std())
    assert n.sigma_q == pytest.approx(2 * np.arange(10.0).std())


def test_norm_stats_pooled_target_scale():
    """Targets share the pooled std of their variable: the std of the whole
    theta block (all rows and levels), not the per-output std."""
    rng = np.random.default_rng(4)
    y = np.concatenate([rng.normal(0, 1, (500, 3)) * [1, 2, 3], rng.normal(5, 1e-3, (500, 3))], 1)
    n = mlp.norm_stats(rng.normal(size=(500, 2)), y)
    np.testing.assert_allclose(n.y_std[:3], np.std(y[:, :3].ravel()), rtol=1e-12)
    np.testing.assert_allclose(n.y_std[3:], np.std(y[:, 3:].ravel()), rtol=1e-12)
    np.testing.assert_allclose(n.y_mean, y.mean(0), rtol=1e-12)


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


def test_judge_columns_hand_built():
    """Four sampled columns (nz = 2) with column RMSE 1, 2, 3, 4 in theta and
    4, 3, 2, 1 in q; a fifth, unsampled column with a huge error is ignored."""
    nz = 2
    ref = np.zeros((5, 2 * nz))
    hat = np.zeros((5, 2 * nz))
    for c, (a, b) in enumerate([(1, 4), (2, 3), (3, 2), (4, 1)]):
        hat[c, :nz] = a          # RMSE over the two levels is a
        hat[c, nz:] = b
    hat[4] = 1e9
    mask = np.array([True, True, True, True, False])
    ft, fq = mlp.judge_columns(hat, ref, mask, sigma_theta=50.0, sigma_q=50.0, rel=0.05)   # bound 2.5
    assert (ft, fq) == (0.5, 0.5)
    ft, fq = mlp.judge_columns(hat, ref, mask, sigma_theta=60.0, sigma_q=20.0, rel=0.05)   # bounds 3, 1
    assert (ft, fq) == (0.25, 0.75)
    assert mlp.judge_columns(hat, ref, np.zeros(5, bool), 1.0, 1.0) == (0.0, 0.0)

