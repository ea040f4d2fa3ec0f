"""GPU parity of the surrogate: BF16 MFMA network, training step, features.

Weights, batches and gradients given to the GPU are drawn on the host (or
by the oracle); the oracle sees the same values.  Tolerances: forward outputs
<= 1e-3 relative (Frobenius), every gradient tensor <= 2e-3 relative
(Frobenius), against the oracle with BF16 rounding at the same points.
"""
import sys

import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import physics
from paper_1802_05839_amd import inputs, wx

pytestmark = pytest.mark.gpu

KIN, NOUTP, NIN, NOUT = wx.MLP_KIN, wx.MLP_NOUTP, wx.MLP_NIN, wx.MLP_NOUT


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _host_params(seed, scale=1.0):
    """FP32-representable weights (unpadded shapes) and small biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.uniform(-1, 1, (512, NIN)) * np.sqrt(6 / NIN) * scale,
         "b1": rng.normal(0, 0.05, 512),
         "W2": rng.uniform(-1, 1, (512, 512)) * np.sqrt(6 / 512) * scale,
         "b2": rng.normal(0, 0.05, 512),
         "W3": rng.uniform(-1, 1, (NOUT, 512)) * np.sqrt(6 / 512) * scale,
         "b3": rng.normal(0, 0.05, NOUT)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def _bf16_rows(rng, n):
    x = np.zeros((n, KIN))
    x[:, :NIN] = omlp.bf16(rng.normal(0, 1, (n, NIN)))
    return x


def _to_bf16_tensor(x):
    """Host float array of BF16-representable values -> device int16 bit patterns."""
    torch = _torch()
    bits = (x.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return torch.from_numpy(np.ascontiguousarray(bits)).cuda()


def _upload(mlp, p):
    mlp.set_params({k: v.astype(np.float32) for k, v in p.items()})


def test_init_matches_oracle_bitwise():
    _say("case: He-uniform init seed 5")
    m = wx.Mlp()
    m.init(5)
    ref = omlp.init_params(5)
    torch = _torch()
    torch.cuda.synchronize()
    w1 = m.param("W1").cpu().numpy()
    w2 = m.param("W2").cpu().numpy()
    w3 = m.param("W3").cpu().numpy()
    np.testing.assert_array_equal(w1[:, :NIN], ref["W1"].astype(np.float32))
    assert np.all(w1[:, NIN:] == 0)
    np.testing.assert_array_equal(w2, ref["W2"].astype(np.float32))
    np.testing.assert_array_equal(w3[:NOUT], ref["W3"].astype(np.float32))
    assert np.all(w3[NOUT:] == 0)
    for b in ("b1", "b2", "b3"):
        assert np.all(m.param(b).cpu().numpy() == 0)
    # BF16 copies and the transposes
    w2b = wx.bf16_bits_to_float(m._sec("W2_bf16", torch.int16, (512, 512))).cpu().numpy()
    np.testing.assert_array_equal(w2b, omlp.bf16(ref["W2"]))
    w3t = wx.bf16_bits_to_float(m._sec("W3T_bf16", torch.int16, (512, 128))).cpu().numpy()
    np.testing.assert_array_equal(w3t[:, :NOUT], omlp.bf16(ref["W3"]).T)


@pytest.mark.parametrize("n", [1000, 64, 7])
def test_forward_matches_oracle(n):
    _say(f"case: forward n={n}")
    rng = np.random.default_rng(10 + n)
    p = _host_params(3)
    m = wx.Mlp()
    m.init(1)
    _upload(m, p)
    x = _bf16_rows(rng, n)
    y = m.infer(_to_bf16_tensor(x)).cpu().numpy()
    ref, _ = omlp.forward(p, x[:, :NIN], bf=True)
    e = _rel(y[:, :NOUT], ref)
    _say(f"forward rel err {e:.3e}")
    assert e <= 1e-3
    assert np.all(y[:, NOUT:] == 0)


@pytest.mark.parametrize("n,m", [(1, 1), (7, 7), (1000, 1000), (2048000, 2048000), (5000, 4096)])
def test_device_shuffle_is_a_seeded_permutation(n, m):
    # wx_mlp_shuffle: the first m values of a permutation of 0..n-1, the same
    # for the same (seed, epoch), another for the next epoch; m > n is refused
    _say(f"case: shuffle n={n} m={m}")
    torch = _torch()
    a = torch.empty(m, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    c = torch.empty(n, dtype=torch.int32, device="cuda")
    wx.shuffle(5, 3, n, a)
    wx.shuffle(5, 3, n, b)
    wx.shuffle(5, 4, n, c)
    torch.cuda.synchronize()
    a, b, c = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(np.sort(c), np.arange(n))
    assert np.unique(a).size == m and a.min() >= 0 and a.max() < n
    if m == n:
        np.testing.assert_array_equal(np.sort(a), np.arange(n))
    if n >= 1000:
        assert not np.array_equal(a[:m], c[:m])
        # a shuffle, not a near-identity: few fixed points
        assert np.sum(a == np.arange(m)) < max(10, m // 100)
    if m > 1:
        with pytest.raises(wx.WxError):
            wx.shuffle(5, 3, m - 1, torch.empty(m, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("batch", [1, 257])
def test_training_step_stays_inside_its_workspace(batch):
    # the workspace of wx_mlp_forward_backward is exactly wx_mlp_work_bytes;
    # a guard band after it (batches whose last 64-row tile ends with a
    # 32-row group past the batch) must come back untouched
    _say(f"case: workspace bounds batch={batch}")
    torch = _torch()
    rng = np.random.default_rng(90 + batch)
    m = wx.Mlp()
    m.init(3)
    nbytes = int(m.lib.wx_mlp_work_bytes(batch))
    guard = 1 << 16
    buf = torch.full((nbytes + guard,), 0xA5, dtype=torch.uint8, device="cuda")
    m._work, m._work_batch = buf[:nbytes], batch
    nrows = batch + 5
    x = _bf16_rows(rng, nrows)
    t = np.zeros((nrows, NOUTP), dtype=np.float32)
    t[:, :NOUT] = rng.normal(0, 1, (nrows, NOUT))
    rows = rng.permutation(nrows)[:batch].astype(np.int32)
    m.forward_backward(_to_bf16_tensor(x), torch.from_numpy(t).cuda(), torch.from_numpy(rows).cuda())
    m.train_step(_to_bf16_tensor(x), torch.from_numpy(t).cuda(), torch.from_numpy(rows).cuda(), 1e-3, 1)
    torch.cuda.synchronize()
    tail = buf[nbytes:].cpu().numpy()
    assert np.all(tail == 0xA5), f"{int(np.sum(tail != 0xA5))} guard bytes written"


@pytest.mark.parametrize("batch", [1, 257, 300, 4096])
def test_gradients_match_oracle(batch):
    _say(f"case: gradients batch={batch}")
    torch = _torch()
    rng = np.random.default_rng(20 + batch)
    p = _host_params(4)
    m = wx.Mlp()
    m.init(1)
    _upload(m, p)
    nrows = batch + 77
    x = _bf16_rows(rng, nrows)
    t = np.zeros((nrows, NOUTP))
    t[:, :NOUT] = rng.normal(0, 1, (nrows, NOUT)).astype(np.float32)
    rows = rng.permutation(nrows)[:batch].astype(np.int32)
    m.forward_backward(_to_bf16_tensor(x), torch.from_numpy(t.astype(np.float32)).cuda(),
                       torch.from_numpy(rows).cuda())
    loss_sum = m.last_loss_sum()
    yb, cache = omlp.forward(p, x[rows, :NIN], bf=True)
    g = omlp.backward(cache, yb, t[rows, :NOUT], bf=True)
    ref_loss = float(np.sum((yb - t[rows, :NOUT]) ** 2))
    assert abs(loss_sum - ref_loss) / ref_loss <= 1e-3
    errs = {}
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        gg = m.param(name, "grad").cpu().numpy()
        if name == "W1":
            assert np.all(gg[:, NIN:] == 0)
            gg = gg[:, :NIN]
        if name == "W3":
            assert np.all(gg[NOUT:] == 0)
            gg = gg[:NOUT]
        if name == "b3":
            gg = gg[:NOUT]
        errs[name] = _rel(gg, g[name])
    _say(f"gradient rel errors {errs}")
    assert max(errs.values()) <= 2e-3, errs


def test_adam_matches_oracle():
    _say("case: Adam two steps")
    torch = _torch()
    rng = np.random.default_rng(30)
    p = _host_params(5)
    m = wx.Mlp()
    m.init(1)
    _upload(m, p)
    st = omlp.adam_init(p)
    cur = p
    for t in (1, 2):
        g = {k: rng.normal(0, 1e-2, v.shape).astype(np.float32).astype(np.float64) for k, v in p.items()}
        for name, arr in g.items():
            full = np.zeros(wx.MLP_PARAM_SHAPES[name], np.float32)
            full[tuple(slice(0, s) for s in arr.shape)] = arr
            m.param(name, "grad").copy_(torch.from_numpy(full))
        m.adam(1e-3, t)
        cur, st = omlp.adam_step(cur, g, st, lr=1e-3)
    torch.cuda.synchronize()
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        got = m.param(name).cpu().numpy()
        sl = tuple(slice(0, s) for s in cur[name].shape)
        np.testing.assert_allclose(got[sl], cur[name], rtol=0, atol=2e-7 + 1e-6 * np.abs(cur[name]).max())
    # the transposed BF16 copy is the transpose of the BF16 copy
    w3b = wx.bf16_bits_to_float(m._sec("W3_bf16", torch.int16, (128, 512))).cpu().numpy()
    w3t = wx.bf16_bits_to_float(m._sec("W3T_bf16", torch.int16, (512, 128))).cpu().numpy()
    np.testing.assert_array_equal(w3t, w3b.T)
    _check_fragment_copies(m)


def test_train_step_equals_forward_backward_then_adam():
    # the train step applies Adam inside the launch that forms the gradients;
    # it must equal the separate calls bit for bit, including the BF16 copies
    _say("case: fused train step vs forward_backward + adam, 3 steps")
    torch = _torch()
    rng = np.random.default_rng(31)
    nrows, batch = 1500, 300
    x = _to_bf16_tensor(_bf16_rows(rng, nrows))
    t = np.zeros((nrows, NOUTP), np.float32)
    t[:, :NOUT] = rng.normal(0, 1, (nrows, NOUT))
    y = torch.from_numpy(t).cuda()
    a, b = wx.Mlp(), wx.Mlp()
    a.init(2)
    b.init(2)
    for step in (1, 2, 3):
        rows = torch.from_numpy(rng.permutation(nrows)[:batch].astype(np.int32)).cuda()
        a.train_step(x, y, rows, 1e-3, step)
        b.forward_backward(x, y, rows)
        b.adam(1e-3, step)
    torch.cuda.synchronize()
    assert torch.equal(a.blob, b.blob)


def _fragment_order(w):
    """[N][K] -> matrix-core fragment order: block (R, S) of 32 rows x 16 k,
    lane l = row % 32 + 32 * (k % 16 // 8) holding its 8 consecutive k."""
    n, k = w.shape
    return w.reshape(n // 32, 32, k // 16, 2, 8).transpose(0, 2, 3, 1, 4).reshape(-1)


def _check_fragment_copies(m):
    torch = _torch()
    packed = m._sec("wpack_bf16", torch.int16, (512 * KIN + 512 * 512 + NOUTP * 512,)).cpu().numpy()
    off = 0
    for name, shape in (("W1_bf16", (512, KIN)), ("W2_bf16", (512, 512)), ("W3_bf16", (NOUTP, 512))):
        w = m._sec(name, torch.int16, shape).cpu().numpy()
        n = shape[0] * shape[1]
        np.testing.assert_array_equal(packed[off:off + n], _fragment_order(w), err_msg=name)
        off += n


def test_fragment_order_copies_follow_init_and_upload():
    _say("case: fragment-order weight copies after init and upload")
    m = wx.Mlp()
    m.init(3)
    _check_fragment_copies(m)
    _upload(m, _host_params(9))
    _check_fragment_copies(m)


def _state32(nx, ny, seed):
    inp = inputs.generate(nx, ny, 58, seed=seed)
    i32 = inp.astype(np.float32)
    i32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    i32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    return i32


def test_features_and_targets_match_oracle():
    _say("case: features and plain-physics targets 96x40x58")
    inp = _state32(96, 40, 41)
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    x_raw, y_raw = st.dataset()
    xr = x_raw.cpu().numpy().astype(np.float64)
    yr = y_raw.cpu().numpy().astype(np.float64)
    st.close()
    fx = omlp.features(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s, inp.f0, inp.ch)
    assert np.all(xr[:, NIN:] == 0)
    # FP32 differences, square roots and products against FP64: a few FP32
    # ulps of each value, or of the feature's scale where it cancels
    scale = np.max(np.abs(fx), axis=0)
    assert np.all(np.abs(xr[:, :NIN] - fx) <= 1e-6 * np.abs(fx) + 1e-6 * scale)
    out = physics.column_physics(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, inp.dt)
    ty = omlp.targets(out.t_theta, out.t_q)
    assert np.all(yr[:, NOUT:] == 0)
    # the FP32 stencil bar of the plain step's tendencies
    for blk in (slice(0, 58), slice(58, 116)):
        e = np.max(np.abs(yr[:, blk] - ty[:, blk])) / np.max(np.abs(ty[:, blk]))
        _say(f"target block {blk}: normalised max error {e:.3e}")
        assert e <= 1e-5, e


def test_fit_norm_and_normalize_match_oracle():
    _say("case: normalisation statistics")
    torch = _torch()
    rng = np.random.default_rng(50)
    n = 5000
    x = np.zeros((n, KIN), np.float32)
    x[:, :NIN] = rng.normal(3.0, 2.0, (n, NIN)) * rng.uniform(0.1, 10, NIN)
    x[:, 5] = 0.015                           # a constant feature
    y = np.zeros((n, NOUTP), np.float32)
    y[:, :NOUT] = rng.normal(0, 1e-3, (n, NOUT)) + rng.uniform(-1e-3, 1e-3, NOUT)
    m = wx.Mlp()
    m.init(1)
    xt = torch.from_numpy(x).cuda()
    yt = torch.from_numpy(y).cuda()
    m.fit_norm(xt, yt)
    ref = omlp.norm_stats(x[:, :NIN].astype(np.float64), y[:, :NOUT].astype(np.float64))
    xm = m._sec("x_mean", torch.float32, (KIN,)).cpu().numpy()
    xis = m._sec("x_invstd", torch.float32, (KIN,)).cpu().numpy()
    ym = m._sec("y_mean", torch.float32, (NOUTP,)).cpu().numpy()
    ys = m._sec("y_std", torch.float32, (NOUTP,)).cpu().numpy()
    np.testing.assert_allclose(xm[:NIN], ref.x_mean, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(1.0 / xis[:NIN], ref.x_std, rtol=1e-6)
    np.testing.assert_allclose(ym[:NOUT], ref.y_mean, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(ys[:NOUT], ref.y_std, rtol=1e-6)
    assert np.all(xis[NIN:] == 0)
    sig = m.sigma().cpu().numpy()
    np.testing.assert_allclose(sig, [ref.sigma_theta, ref.sigma_q], rtol=1e-9)
    xo, yo = m.normalize(xt, yt)
    xn = wx.bf16_bits_to_float(xo).cpu().numpy().astype(np.float64)
    want = omlp.bf16((x[:, :NIN] - ref.x_mean) / ref.x_std)
    # one BF16 step allowed where FP32 statistics move a value across a rounding
    # boundary; values that cancel to ~0 differ by the FP32 statistics' rounding
    excess = float(np.max(np.abs(xn[:, :NIN] - want) - 2.0 ** -7 * np.abs(want)))
    _say(f"normalised features: worst excess over one BF16 step {excess:.3e}")
    assert excess <= 1e-5
    assert np.mean(xn[:, :NIN] == want) > 0.99
    np.testing.assert_allclose(yo.cpu().numpy()[:, :NOUT], (y[:, :NOUT] - ref.y_mean) / ref.y_std,
                               rtol=1e-5, atol=1e-5)


def test_training_reduces_loss_and_is_reproducible():
    _say("case: training 64x64x58 dataset, 150 steps x2")
    torch = _torch()
    inp = _state32(64, 64, 42)
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    x_raw, y_raw = st.dataset()
    st.close()
    finals = []
    for _ in range(2):
        m = wx.Mlp()
        m.init(7)
        m.fit_norm(x_raw, y_raw)
        xn, yn = m.normalize(x_raw, y_raw)
        rng = np.random.default_rng(3)
        losses = []
        for t in range(1, 151):
            rows = torch.from_numpy(rng.permutation(4096)[:1024].astype(np.int32)).cuda()
            m.train_step(xn, yn, rows, 1e-3, t)
            if t in (1, 150):
                losses.append(m.last_loss_sum() / (1024 * NOUT))
        _say(f"loss {losses}")
        assert losses[1] < 0.5 * losses[0]
        finals.append(m.blob.cpu().numpy().copy())
    np.testing.assert_array_equal(finals[0], finals[1])
