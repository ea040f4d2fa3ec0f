"""wx_mass_noalloc (the mass sums with the block partials in the library's
static device array) against wx_mass (partials in the caller's workspace).

Both run the same kernels in the same order, so mass_out must agree bit for
bit; two calls in a row, the second on a smaller grid (and the other dtype),
show that nothing left in the shared array from the first call leaks into the
second.  The values themselves are also checked against exactly rounded sums
of the stored state.
"""
import math
import sys

import numpy as np
import pytest

from paper_1802_05839_amd import inputs, wx

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _exact(st, inp, dtype):
    nx, ny = inp.nx, inp.ny
    npd = np.float32 if dtype == "f32" else np.float64
    raw = {n: st.download_raw(n)[:, 2:2 + ny, 2:2 + nx].astype(npd).astype(np.float64)
           for n in ("rho", "theta", "q")}
    m = raw["rho"] * (inp.dx * inp.dx * inp.dz)[:, None, None]
    return np.array([math.fsum(m.ravel()), math.fsum((m * raw["theta"]).ravel()),
                     math.fsum((m * raw["q"]).ravel())])


def _compare(nx, ny, nz, dtype, seed):
    _say(f"case: wx_mass_noalloc vs wx_mass {nx}x{ny}x{nz} {dtype}")
    inp = inputs.generate(nx, ny, nz, seed=seed)
    st = wx.state_from_inputs(inp, dtype=dtype, theta_offset=0.0)
    st.t["mass_out"].fill_(-1.0)
    st.t["flags_out"].zero_()
    st.mass(compute=True)
    ref = st.mass_raw()
    ref_flags = st.flags()
    st.t["mass_out"].fill_(-1.0)
    st.t["flags_out"].zero_()
    st.mass_noalloc()
    got = st.mass_raw()
    got_flags = st.flags()
    want = _exact(st, inp, dtype)
    st.close()
    assert np.array_equal(got, ref), (got, ref)
    assert got_flags == ref_flags
    sums = np.array([got[0] + got[1], got[2] + got[3], got[4] + got[5]])
    rel = np.abs(sums - want) / np.abs(want)
    _say(f"bitwise equal to wx_mass; relative error against exact sums {rel}")
    assert np.all(rel <= 1e-13), rel


def test_noalloc_mass_matches_wx_mass_then_smaller_grid():
    _compare(400, 320, 58, "f32", 41)      # 7 x 320 = 2240 partial blocks
    _compare(67, 37, 5, "f64", 42)         # smaller, other dtype, ragged tile
