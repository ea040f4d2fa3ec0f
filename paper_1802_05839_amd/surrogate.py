"""Training and evaluation driver of the physics surrogate (host orchestration).

Every numerical step runs in libwx: the dataset rows come from
``wx_dataset`` (features and plain-physics tendencies of a state), the
statistics from ``wx_mlp_fit_norm``, the training steps from
``wx_mlp_train_step`` (BF16 MFMA forward/backward + Adam).  This module only
decides which states to sample, the seeded batch order and the bookkeeping.

Recipe: rows are the columns of post-dycore states -- the state that the
physics of step n sees inside a coupled step -- of plain-method runs on
400 x 320 x 58 grids (one GPU's share of the 1581 x 1301 x 58 grid) with
seeds 100..103 at n = 25, 100, 200 and 300: 16 snapshots x 128,000 columns =
2,048,000 rows, labelled with the plain-physics tendencies of that state.
The first steps are left out on purpose: the implicit diffusion removes the
initial white-noise layering of q within a few steps, with q tendencies a
hundred times those of the settled flow, and a training set holding them
would set the q scale (and the judge's bound) by that transient.  Those
steps are the judge's to reject.  The held-out states are seed 104 after 10
(transient), 50 and 300 steps.  120 epochs of batch 4096, Adam with the
learning rate 1e-3 decayed per epoch by a half cosine, shuffle seeded per
epoch.
"""
from __future__ import annotations

import time
from typing import List, Sequence

import numpy as np

from . import inputs, wx

TRAIN_SEEDS = (100, 101, 102, 103)
SNAPSHOTS = (25, 100, 200, 300)
HELD_OUT_SEED = 104
HELD_OUT_STEPS = (10, 50, 300)
EPOCHS = 120


def _post_dycore_rows(inp, steps: Sequence[int]):
    """(features, targets) of the state that the physics of step n sees, for
    each n in steps: n - 1 plain steps, then the dycore of step n alone."""
    import torch
    out = []
    for n in steps:
        st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
        if n > 1:
            st.step(n - 1)
        st.set_phys_mode(wx.WX_PHYS_OFF)
        st.step(1)
        out.append(st.dataset())
        torch.cuda.synchronize()
        st.close()
    return out


def build_dataset(seeds: Sequence[int] = TRAIN_SEEDS, snapshots: Sequence[int] = SNAPSHOTS,
                  nx: int = 400, ny: int = 320, log=None):
    """Raw (features, targets) device tensors over all seeds and snapshots:
    the post-dycore state of step n and its plain-physics tendencies, which
    is what the surrogate replaces inside a coupled step."""
    import torch
    xs, ys = [], []
    for seed in seeds:
        inp = inputs.generate(nx, ny, 58, seed=seed, dtype=np.float32)
        for x, y in _post_dycore_rows(inp, snapshots):
            xs.append(x)
            ys.append(y)
        if log:
            log(f"dataset seed {seed}: {len(snapshots)} snapshots")
    return torch.cat(xs), torch.cat(ys)


def train(mlp: "wx.Mlp", x, y, epochs: int = EPOCHS, batch: int = 4096, lr: float = 1e-3,
          shuffle_seed: int = 0, log=None) -> List[float]:
    """Adam over seeded shuffles, learning rate lr * (1 + cos(pi e / epochs)) / 2
    in epoch e; returns the last-batch training loss of each epoch."""
    import torch
    n = int(x.shape[0])
    nb = n // batch
    t = 0
    dev = x.device
    stream = torch.cuda.current_stream(dev)
    # each epoch's row order is drawn on the device (wx_mlp_shuffle), in
    # stream order before the epoch's steps; the per-epoch losses stay on the
    # device until the end, so the host never waits for the GPU
    rows = torch.empty(nb * batch, dtype=torch.int32, device=dev)
    losses = torch.zeros(epochs, dtype=torch.float32, device=dev)
    for ep in range(epochs):
        wx.shuffle(shuffle_seed, ep, n, rows, stream)
        lr_ep = lr * 0.5 * (1.0 + np.cos(np.pi * ep / epochs))
        for b in range(nb):
            t += 1
            mlp.train_step(x, y, rows[b * batch:(b + 1) * batch], lr_ep, t)
        losses[ep:ep + 1].copy_(mlp._loss)
    hist = (losses / float(batch * wx.MLP_NOUT)).cpu().tolist()
    if log:
        for ep, last in enumerate(hist):
            log(f"epoch {ep + 1}: last-batch loss {last:.5f}")
    return hist


def held_out(nx: int = 400, ny: int = 320, seed: int = HELD_OUT_SEED, steps: Sequence[int] = HELD_OUT_STEPS):
    """{step n: (raw features, targets)} of one held-out run, post-dycore states."""
    inp = inputs.generate(nx, ny, 58, seed=seed, dtype=np.float32)
    return dict(zip(steps, _post_dycore_rows(inp, steps)))


def fit(mlp: "wx.Mlp", x_raw, y_raw, epochs: int = EPOCHS, batch: int = 4096, lr: float = 1e-3,
        init_seed: int = 1, log=None):
    """Initialise, normalise and train; returns (loss history, seconds of training)."""
    import torch
    mlp.init(init_seed)
    mlp.fit_norm(x_raw, y_raw)
    xn, yn = mlp.normalize(x_raw, y_raw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(mlp, xn, yn, epochs=epochs, batch=batch, lr=lr, log=log)
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0
