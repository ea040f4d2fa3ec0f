"""What training buys: the trained surrogate against the same network untrained
and against leaving the physics out (zero tendencies), on held-out states.

A short run of the library's own training (the BF16 forward/backward kernels
and Adam) on plain-physics columns of 192 x 160 x 58 states; the full-size
recipe is the benchmark's.  Sizes keep the test to a few seconds.
"""
import sys

import numpy as np
import pytest

from bench import tendency_rmse
from paper_1802_05839_amd import inputs, surrogate, wx

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_training_beats_untrained_and_no_physics():
    import torch
    _say("case: short surrogate training, 192x160x58 states")
    x, y = surrogate.build_dataset(seeds=(200, 201), snapshots=(20, 60, 120), nx=192, ny=160)
    held = surrogate.held_out(nx=192, ny=160, seed=202, steps=(40,))[40]
    untrained = wx.Mlp()
    untrained.init(1)
    untrained.fit_norm(x, y)
    r_untrained = tendency_rmse(untrained, *held)
    trained = wx.Mlp()
    hist, secs = surrogate.fit(trained, x, y, epochs=30)
    r = tendency_rmse(trained, *held)
    _say(f"trained {secs:.1f}s, loss {hist[0]:.4f} -> {hist[-1]:.4f}; held-out rmse/sigma "
         f"theta {r['rmse_theta'] / r['sigma_theta']:.4f} q {r['rmse_q'] / r['sigma_q']:.4f}; "
         f"untrained {r_untrained['rmse_theta'] / r['sigma_theta']:.3f} "
         f"{r_untrained['rmse_q'] / r['sigma_q']:.3f}; zero-physics "
         f"{r['rmse_zero_theta'] / r['sigma_theta']:.3f} {r['rmse_zero_q'] / r['sigma_q']:.3f}")
    assert hist[-1] < 0.5 * hist[0]
    for v in ("theta", "q"):
        assert r[f"rmse_{v}"] < 0.25 * r[f"rmse_zero_{v}"]
        assert r[f"rmse_{v}"] < 0.25 * r_untrained[f"rmse_{v}"]
    # the judge of a coupled step sees the same gain
    inp = inputs.generate(192, 160, 58, seed=202, dtype=np.float32)
    rm = {}
    for name, m in (("trained", trained), ("untrained", untrained)):
        st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
        st.step(39)
        st.attach_mlp(m)
        st.set_phys_mode(wx.WX_PHYS_JUDGED)
        st.step(1)
        rm[name] = st.judge()
        st.close()
    _say(f"judge rmse trained {rm['trained'][:2]} untrained {rm['untrained'][:2]}")
    assert rm["trained"][0] < 0.25 * rm["untrained"][0] and rm["trained"][1] < 0.25 * rm["untrained"][1]
    assert rm["untrained"][2]                     # the untrained network is rejected
    del x, y
    torch.cuda.empty_cache()
