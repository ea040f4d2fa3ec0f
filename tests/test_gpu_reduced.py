"""GPU parity of the paper's reduced weather application against the oracle.

The kernel does the printed FP64 operations in the printed order with no
fused multiply-add, so every comparison here is bit for bit.  Small grids
are compared whole over several steps (ragged tiles, more than one level
chunk, two-level columns, the ring and its corners); the paper's largest
shape (256 x 256 x 512) is compared on sampled columns, each recomputed by
the oracle on a crop wide enough to hold the sample's dependency cone.
"""
import sys

import numpy as np
import pytest

from oracle import reduced as rw
from paper_1802_05839_amd import inputs, wx

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _random_case(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    e = rng.uniform(0.0, 400.0, rw.shape(nx, ny, nz))
    surf = rng.uniform(280.0, 340.0, (ny + 2, nx + 2))
    pbl = rng.uniform(180.0, 240.0, (ny + 2, nx + 2))
    return e, surf, pbl


@pytest.mark.parametrize("nx,ny,nz,nsteps,nu", [(5, 4, 2, 3, 0.1), (37, 29, 11, 7, 0.1), (70, 9, 17, 5, 0.137),
                                                (130, 66, 40, 4, 0.1), (1, 1, 3, 6, 0.15), (64, 4, 16, 3, 0.05)])
def test_random_fields_bitwise(nx, ny, nz, nsteps, nu):
    _say(f"case: reduced app {nx}x{ny}x{nz} random fields, {nsteps} steps, nu={nu}")
    e, surf, pbl = _random_case(nx, ny, nz, seed=nx * 1000 + nz)
    app = wx.ReducedApp(e, surf, pbl, nu)
    app.run(nsteps)
    got = app.download()
    want = rw.simulate(e, surf, pbl, nsteps, nu)
    np.testing.assert_array_equal(got, want)


def test_paper_initial_state_128_cubed_bitwise():
    _say("case: reduced app 128^3 from the paper's box, 20 steps")
    n = 128
    e = inputs.rw_box_init(n, n, n)
    surf, pbl = inputs.rw_boundary_fields(n, n)
    app = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT)
    app.run(20)
    np.testing.assert_array_equal(app.download(), rw.simulate(e, surf, pbl, 20))


def test_single_step_entry_point_and_zero_steps():
    _say("case: reduced app wx_rw_step vs wx_rw_run, nsteps = 0")
    e, surf, pbl = _random_case(33, 12, 9, seed=5)
    a = wx.ReducedApp(e, surf, pbl, 0.1)
    a.run(0)
    assert a.cur == 0
    np.testing.assert_array_equal(a.download(), e)
    for _ in range(3):
        a.step_into()
    b = wx.ReducedApp(e, surf, pbl, 0.1)
    b.run(3)
    assert a.cur == b.cur == 1
    np.testing.assert_array_equal(a.download(), b.download())


def test_paper_largest_shape_sampled_columns():
    # 256 x 256 x 512, 20 steps: each sampled interior column is recomputed
    # by the oracle on a crop of half-width 21 around it (a step moves
    # information one cell, so the crop's own edge cannot reach the centre)
    nx, ny, nz, nsteps = 256, 256, 512, 20
    _say(f"case: reduced app {nx}x{ny}x{nz}, {nsteps} steps, sampled columns")
    e = inputs.rw_box_init(nx, ny, nz)
    surf, pbl = inputs.rw_boundary_fields(nx, ny)
    app = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT)
    app.run(nsteps)
    got = app.download()
    h = nsteps + 1
    rng = np.random.default_rng(7)
    # samples on the box edges (where the field varies) and at random
    pts = [(65, 65), (64, 192), (128, 65), (192, 192)] + [tuple(rng.integers(h + 1, 257 - h, 2)) for _ in range(4)]
    for j, i in pts:
        crop = e[:, j - h:j + h + 1, i - h:i + h + 1]
        cs = surf[j - h:j + h + 1, i - h:i + h + 1]
        cp = pbl[j - h:j + h + 1, i - h:i + h + 1]
        ref = rw.simulate(crop, cs, cp, nsteps)
        np.testing.assert_array_equal(got[:, j, i], ref[:, h, h], err_msg=f"column ({i}, {j})")


@pytest.mark.parametrize("nx,ny,nz,nsteps", [(5, 4, 2, 3), (70, 9, 17, 4), (1, 1, 3, 5)])
def test_kij_order_bitwise(nx, ny, nz, nsteps):
    _say(f"case: reduced app KIJ order {nx}x{ny}x{nz}, {nsteps} steps")
    e, surf, pbl = _random_case(nx, ny, nz, seed=nx * 7 + nz)
    app = wx.ReducedApp(e, surf, pbl, 0.1, order="kij")
    app.run(nsteps)
    np.testing.assert_array_equal(app.download(), rw.simulate(e, surf, pbl, nsteps, 0.1))


def test_kij_order_equals_ijk_order_128_cubed():
    _say("case: reduced app KIJ vs IJK order, 128^3 box, 10 steps")
    n = 128
    e = inputs.rw_box_init(n, n, n)
    surf, pbl = inputs.rw_boundary_fields(n, n)
    a = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT)
    b = wx.ReducedApp(e, surf, pbl, inputs.RW_NU_DEFAULT, order="kij")
    a.run(10)
    b.run(10)
    np.testing.assert_array_equal(a.download(), b.download())


@pytest.mark.parametrize("block", [(32, 16), (128, 1), (64, 4), (128, 4)])
def test_block_shapes_bitwise(block):
    # the block-size ablation: every shape does the printed arithmetic per
    # cell, so each equals the oracle bit for bit (ragged tiles in i and j,
    # two level chunks)
    _say(f"case: reduced app block {block[0]}x{block[1]}, 70x37x20, 4 steps")
    e, surf, pbl = _random_case(70, 37, 20, seed=77)
    app = wx.ReducedApp(e, surf, pbl, 0.1, block=block)
    app.run(4)
    np.testing.assert_array_equal(app.download(), rw.simulate(e, surf, pbl, 4, 0.1))


def test_unsupported_block_shape_is_rejected():
    _say("case: reduced app unsupported block shape")
    e, surf, pbl = _random_case(8, 8, 4, seed=78)
    app = wx.ReducedApp(e, surf, pbl, 0.1, block=(16, 16))
    with pytest.raises(wx.WxError, match="not one of"):
        app.run(1)
