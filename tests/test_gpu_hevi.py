"""GPU parity of the HEVI fast-mode short steps (wx_hevi_run) against the
FP64 oracle.

Tolerances (normalized max error max|gpu - oracle| / max|oracle| per field):
FP64 <= 1e-12 after several steps; FP32 from identical FP32-representable
inputs <= 2e-5 after 3 steps: pi' = pi - h c^2 (D + dwm/dz) carries
h c^2 D ~ 5x the size of pi itself at these amplitudes (c = 340 m/s), so
the few FP32 roundings of D (6e-8 relative each, ~10 of them between u and
D) reach pi at about 5 x 10 x 6e-8 = 3e-6 per step, and three steps stay
below 1e-5; w, b and the winds are smaller sums.  Bitwise checks: rest,
translation, run-to-run, periodic halo ring.
"""
import hashlib
import sys

import numpy as np
import pytest

from oracle import hevi
from paper_1802_05839_amd import inputs, wx
from tests._util import nmax

pytestmark = pytest.mark.gpu

NAMES = ("u", "v", "w", "b", "pi")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle(f, nsteps, tau):
    x = hevi.Fast(f.u, f.v, f.w, f.b, f.pi)
    return hevi.run(x, nsteps, f.dx, f.dx, f.dz, tau)


def _errors(got, ref):
    return {n: nmax(got[n], getattr(ref, n)) for n in NAMES}


@pytest.mark.parametrize("nx,ny,nz,nsteps", [(70, 37, 12, 6), (67, 9, 5, 5), (4, 4, 2, 3), (130, 66, 58, 2)])
def test_fp64_matches_oracle(nx, ny, nz, nsteps):
    _say(f"case: HEVI FP64 {nx}x{ny}x{nz}, {nsteps} steps")
    f = inputs.hevi_fields(nx, ny, nz, seed=nx + nz)
    tau = inputs.HEVI_TAU_DEFAULT
    hv = wx.Hevi(f, tau, dtype="f64")
    hv.run(nsteps)
    errs = _errors(hv.download(), _oracle(f, nsteps, tau))
    _say(f"errors {errs}")
    for n, e in errs.items():
        assert e <= 1e-12, (n, errs)


@pytest.mark.parametrize("kernel,nz", [(0, 58), (1, 58), (0, 16), (1, 21), (2, 58), (2, 16)])
def test_fp32_matches_oracle(kernel, nz):
    # kernel 0 keeps the column in registers for nz 16 / 58, kernel 1 (and any
    # other nz) parks it in the outputs, kernel 2 gives a column two lanes and
    # solves from both ends (97 = 3 x 32 + 1: one live column in the last tile)
    _say(f"case: HEVI FP32 97x45x{nz} kernel {kernel}, 3 steps")
    f = inputs.hevi_fields(97, 45, nz, seed=3).astype(np.float32)
    tau = inputs.HEVI_TAU_DEFAULT
    hv = wx.Hevi(f, tau, dtype="f32", kernel=kernel)
    hv.run(3)
    errs = _errors(hv.download(), _oracle(f, 3, tau))
    _say(f"fp32 errors {errs}")
    for n, e in errs.items():
        assert e <= 2e-5, (n, errs)


@pytest.mark.parametrize("nz", [16, 58])
def test_fp64_two_sided_kernel_matches_oracle(nz):
    # the elimination from the ground and from the lid joined at face nz/2 is
    # an exact solve of the same system: the FP64 bar of the one-sided kernels
    _say(f"case: HEVI FP64 70x37x{nz} two-sided kernel, 4 steps")
    f = inputs.hevi_fields(70, 37, nz, seed=nz + 1)
    hv = wx.Hevi(f, inputs.HEVI_TAU_DEFAULT, dtype="f64", kernel=2)
    hv.run(4)
    errs = _errors(hv.download(), _oracle(f, 4, inputs.HEVI_TAU_DEFAULT))
    _say(f"fp64 two-sided errors {errs}")
    for n, e in errs.items():
        assert e <= 1e-12, (n, errs)


@pytest.mark.parametrize("nz", [16, 58])
def test_fp64_parked_kernel_matches_oracle(nz):
    _say(f"case: HEVI FP64 70x37x{nz} parked kernel, 4 steps")
    f = inputs.hevi_fields(70, 37, nz, seed=nz)
    hv = wx.Hevi(f, inputs.HEVI_TAU_DEFAULT, dtype="f64", kernel=1)
    hv.run(4)
    errs = _errors(hv.download(), _oracle(f, 4, inputs.HEVI_TAU_DEFAULT))
    for n, e in errs.items():
        assert e <= 1e-12, (n, errs)


def test_zero_steps_and_rest_state_bitwise():
    _say("case: HEVI zero steps, rest state")
    f = inputs.hevi_fields(40, 12, 7, seed=9)
    hv = wx.Hevi(f, 2.0, dtype="f32")
    before = hv.download()
    hv.run(0)                      # fills the halo rings, changes no interior value
    after = hv.download()
    for n in NAMES:
        np.testing.assert_array_equal(after[n], before[n])
    z = inputs.FastFields(*(np.zeros_like(a) for a in (f.u, f.v, f.w, f.b, f.pi)), f.dz, f.dx)
    hv = wx.Hevi(z, 2.0, dtype="f64")
    hv.run(4)
    for n in NAMES:
        assert np.all(hv.download_raw(n) == 0.0), n


def test_translation_and_run_to_run_bitwise():
    _say("case: HEVI translation and reproducibility FP32")
    f = inputs.hevi_fields(72, 40, 9, seed=10)
    p, q = 13, 7
    sh = inputs.FastFields(*(np.roll(np.roll(a, q, axis=-2), p, axis=-1) for a in (f.u, f.v, f.w, f.b, f.pi)),
                           f.dz, f.dx)
    runs = []
    for src in (f, f, sh):
        hv = wx.Hevi(src, 2.0, dtype="f32")
        hv.run(3)
        runs.append(hv.download())
    for n in NAMES:
        np.testing.assert_array_equal(runs[0][n], runs[1][n])
        np.testing.assert_array_equal(np.roll(np.roll(runs[0][n], q, axis=-2), p, axis=-1), runs[2][n])


@pytest.mark.parametrize("nsteps", [1, 2])
def test_halo_ring_is_periodic(nsteps):
    _say(f"case: HEVI halo ring after {nsteps} steps")
    f = inputs.hevi_fields(20, 12, 5, seed=11)
    hv = wx.Hevi(f, 2.0, dtype="f64")
    hv.run(nsteps)
    for n in ("u", "v", "pi"):
        a = hv.download_raw(n)[:, :, :f.u.shape[2] + 4]
        inner = a[:, 2:-2, 2:-2]
        np.testing.assert_array_equal(a, np.pad(inner, ((0, 0), (2, 2), (2, 2)), mode="wrap"))


def test_full_grid_fp32_sampled_against_oracle():
    # the benchmark's fast-mode workload, 1581 x 1301 x 58 in FP32, one short
    # step, checked on windows: one short step reaches 2 cells horizontally
    # (the vertical solve is column-local), so the oracle on a periodic crop
    # enlarged by 4 cells reproduces the full-grid result inside it
    nx, ny, nz = 1581, 1301, 58
    _say(f"case: HEVI FP32 {nx}x{ny}x{nz}, 1 short step, windows")
    f = inputs.hevi_fields(nx, ny, nz, seed=2).astype(np.float32)
    hv = wx.Hevi(f, 2.0, dtype="f32")
    hv.run(1)
    got = hv.download()
    del hv
    m = 4
    worst = {}
    for (i0, j0, cx, cy) in [(0, 0, 24, 24), (1560, 1280, 21, 21), (700, 640, 24, 24)]:
        ii = np.arange(i0 - m, i0 + cx + m) % nx
        jj = np.arange(j0 - m, j0 + cy + m) % ny
        sub = inputs.FastFields(*(a[:, jj][:, :, ii] for a in (f.u, f.v, f.w, f.b, f.pi)), f.dz, f.dx)
        ref = _oracle(sub, 1, 2.0)
        for n in NAMES:
            g = got[n][:, jj[m:m + cy]][:, :, ii[m:m + cx]]
            r = getattr(ref, n)[:, m:m + cy, m:m + cx]
            worst[n] = max(worst.get(n, 0.0), nmax(g, r))
    _say(f"full grid fp32 errors {worst}")
    for n, e in worst.items():
        assert e <= 2e-5, (n, worst)


@pytest.mark.parametrize("kernel", [0, 1, 2])
def test_run_stays_inside_its_workspace(kernel):
    # an odd number of short steps (the result copied back from the second
    # field set) on a ragged grid: a guard band after wx_hevi_workspace_bytes
    # comes back untouched
    import torch
    _say(f"case: HEVI workspace bounds kernel {kernel}")
    f = inputs.hevi_fields(97, 45, 58, seed=9).astype(np.float32)
    hv = wx.Hevi(f, inputs.HEVI_TAU_DEFAULT, dtype="f32", kernel=kernel)
    nb = hv.ws.numel()
    guard = 1 << 16
    big = torch.full((nb + guard,), 0xA5, dtype=torch.uint8, device=hv.device)
    hv.ws = big[:nb]
    hv.run(3)
    torch.cuda.synchronize()
    tail = big[nb:].cpu().numpy()
    assert np.all(tail == 0xA5), f"{int(np.sum(tail != 0xA5))} guard bytes written"


def test_bad_arguments_are_rejected():
    _say("case: HEVI argument errors")
    f = inputs.hevi_fields(8, 8, 4, seed=12)
    hv = wx.Hevi(f, 2.0, dtype="f64")
    before = hashlib.sha256(hv.download_raw("pi").tobytes()).hexdigest()
    with pytest.raises(wx.WxError, match="nsteps"):
        hv.run(-1)
    hv.dz[1] = -1.0
    with pytest.raises(wx.WxError, match="dz"):
        hv.run(1)
    # rejected calls leave the device untouched
    assert hashlib.sha256(hv.download_raw("pi").tobytes()).hexdigest() == before
