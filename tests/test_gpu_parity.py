"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 state, normalized max error max|gpu - oracle| / max|oracle|
<= 1e-12 after 10 steps; FP32 state <= 1e-5 per field after one step from
identical FP32-representable inputs, with theta measured as theta - 300.
Bitwise checks: constant fields, uniform states, translation, run-to-run.
"""
import hashlib
import math
import sys
from dataclasses import replace

import numpy as np
import pytest

from oracle import dycore, physics, step
from oracle.mass import mass_sums
from oracle.params import DEFAULT
from paper_1802_05839_amd import inputs, wx
from tests._util import nmax, uniform_inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_gpu(inp, nsteps, dtype="f64", phys=wx.WX_PHYS_PLAIN, params=None, theta_offset=None):
    st = wx.state_from_inputs(inp, dtype=dtype, phys_mode=phys, theta_offset=theta_offset)
    for k, v in (params or {}).items():
        st.set_param(k, v)
    st.step(nsteps)
    out = st.download()
    out["flags"] = st.flags()
    out["mass"] = st.mass()
    out["mass_raw"] = st.mass_raw()
    st.close()
    return out


def _oracle(inp, nsteps, physics_on=True, p=DEFAULT):
    return step.run(inp, nsteps, p=p, physics_on=physics_on)


def _compare(gpu, ref, tol, theta_ref=0.0):
    errs = {"rho": nmax(gpu["rho"], ref.rho),
            "theta": nmax(gpu["theta"] - theta_ref, ref.theta - theta_ref),
            "q": nmax(gpu["q"], ref.q)}
    for k, e in errs.items():
        assert e <= tol, (k, errs)
    return errs


def test_tiny_fp64_ten_steps_matches_oracle():
    _say("case: 64x64x16 FP64 10 steps")
    inp = inputs.generate_config("tiny")
    gpu = _run_gpu(inp, 10, "f64")
    ref = _oracle(inp, 10)
    errs = _compare(gpu, ref, FP64_TOL)
    _say(f"errors {errs}")
    assert gpu["flags"]["nonfinite"] == 0 and gpu["flags"]["rho_le0"] == 0
    # mass sums of the final state agree with the oracle's sums of its state
    np.testing.assert_allclose(gpu["mass"], step.masses(ref, inp), rtol=1e-12)


def test_tiny_fp64_dycore_only_matches_oracle():
    _say("case: 64x64x16 FP64 dycore only 10 steps")
    inp = inputs.generate_config("tiny")
    gpu = _run_gpu(inp, 10, "f64", phys=wx.WX_PHYS_OFF)
    ref = _oracle(inp, 10, physics_on=False)
    _compare(gpu, ref, FP64_TOL)


def test_tiny_fp32_one_step_matches_oracle():
    _say("case: 64x64x16 FP32 1 step")
    inp = inputs.generate_config("tiny")
    # identical FP32-representable inputs on both sides (theta stored as theta - 300)
    inp32 = inp.astype(np.float32)
    inp32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    inp32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    gpu = _run_gpu(inp32, 1, "f32", theta_offset=300.0)
    ref = _oracle(inp32, 1)
    errs = _compare(gpu, ref, FP32_TOL, theta_ref=300.0)
    _say(f"fp32 errors {errs}")


@pytest.mark.parametrize("nx,ny,nz", [(4, 4, 3), (67, 37, 5), (130, 9, 7), (65, 5, 4)])
def test_ragged_sizes_fp64(nx, ny, nz):
    _say(f"case: ragged {nx}x{ny}x{nz} FP64 3 steps")
    inp = inputs.generate(nx, ny, nz, seed=21)
    gpu = _run_gpu(inp, 3, "f64")
    ref = _oracle(inp, 3)
    _compare(gpu, ref, FP64_TOL)


def test_ragged_fp32():
    _say("case: ragged 97x45x11 FP32 1 step")
    inp = inputs.generate(97, 45, 11, seed=22)
    inp32 = inp.astype(np.float32)
    inp32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    inp32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    gpu = _run_gpu(inp32, 1, "f32", theta_offset=300.0)
    ref = _oracle(inp32, 1)
    _compare(gpu, ref, FP32_TOL, theta_ref=300.0)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_constant_field_bitwise(dtype):
    _say(f"case: constant field {dtype}")
    inp = inputs.generate(40, 24, 9, seed=23)
    c1, c2 = 287.25, 0.0075
    inp.theta[:] = c1
    inp.q[:] = c2
    inp.theta_s[:] = c1
    inp.q_s[:] = c2
    inp.f0[:] = 0.0
    st = wx.state_from_inputs(inp, dtype=dtype, theta_offset=0.0)
    st.step(3)
    th = st.download_raw("theta")[:, 2:-2, 2:2 + inp.nx]
    q = st.download_raw("q")[:, 2:-2, 2:2 + inp.nx]
    st.close()
    npd = np.float32 if dtype == "f32" else np.float64
    assert np.all(th == npd(c1)) and np.all(q == npd(c2))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_uniform_state_bitwise(dtype):
    _say(f"case: uniform state {dtype}")
    inp = uniform_inputs(nx=70, ny=11, nz=6, u0=7.5, v0=-3.25, rho0=1.0625, theta0=301.5, q0=0.004)
    st = wx.state_from_inputs(inp, dtype=dtype, theta_offset=0.0)
    st.step(2)
    npd = np.float32 if dtype == "f32" else np.float64
    for name, val in (("rho", 1.0625), ("theta", 301.5), ("q", 0.004)):
        a = st.download_raw(name)[:, 2:2 + inp.ny, 2:2 + inp.nx]
        assert np.all(a == npd(val)), name
    st.close()


def test_translation_bitwise():
    _say("case: translation invariance FP32")
    inp = inputs.generate(72, 40, 8, seed=24)
    p, qq = 13, 7
    sh = inp.copy()
    for name, a in sh.fields().items():
        setattr(sh, name, np.roll(np.roll(a, qq, axis=-2), p, axis=-1))
    o1 = _run_gpu(inp, 2, "f32")
    o2 = _run_gpu(sh, 2, "f32")
    for name in ("rho", "theta", "q"):
        np.testing.assert_array_equal(np.roll(np.roll(o1[name], qq, axis=-2), p, axis=-1), o2[name])


def test_run_to_run_bitwise():
    _say("case: reproducibility FP32 5 steps x2")
    inp = inputs.generate(150, 70, 12, seed=25)
    digests = []
    for _ in range(2):
        st = wx.state_from_inputs(inp, dtype="f32")
        st.step(5)
        h = hashlib.sha256()
        for name in ("rho", "theta", "q"):
            h.update(st.download_raw(name).tobytes())
        h.update(st.mass_raw().tobytes())
        digests.append(h.hexdigest())
        st.close()
    assert digests[0] == digests[1]


def test_halo_ring_is_periodic_after_step():
    _say("case: halo ring FP64")
    inp = inputs.generate(20, 12, 5, seed=26)
    st = wx.state_from_inputs(inp, dtype="f64")
    st.step(2)
    for name in ("rho", "theta", "q"):
        a = st.download_raw(name)[:, :, :inp.nx + 4]
        inner = a[:, 2:-2, 2:-2]
        full = np.pad(inner, ((0, 0), (2, 2), (2, 2)), mode="wrap")
        np.testing.assert_array_equal(a, full)
    st.close()


def test_tendencies_match_oracle():
    _say("case: wx_physics tendencies FP64 and FP32")
    inp = inputs.generate(50, 30, 16, seed=27)
    ref = physics.column_physics(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, inp.dt)
    st = wx.state_from_inputs(inp, dtype="f64")
    tt, tq = st.tendencies()
    st.close()
    assert nmax(tt, ref.t_theta) <= FP64_TOL and nmax(tq, ref.t_q) <= FP64_TOL
    inp32 = inp.astype(np.float32)
    inp32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    inp32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    ref32 = physics.column_physics(inp32.rho, inp32.theta, inp32.q, inp32.u, inp32.v, inp32.theta_s,
                                   inp32.q_s, inp32.f0, inp32.ch, inp32.dz, inp32.dt)
    st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
    tt, tq = st.tendencies()
    st.close()
    e = (nmax(tt, ref32.t_theta), nmax(tq, ref32.t_q))
    _say(f"fp32 tendency errors {e}")
    assert max(e) <= FP32_TOL


def _stiff_f32_inputs(nz, dt_scale, mix_len, seed=28):
    """FP32-representable problem whose columns are stiff: the dominance
    ratio r = (alpha_lo + alpha_hi)/m scales with dt and with mix_len^2."""
    inp = inputs.generate(70, 20, nz, seed=seed)
    inp.dt = inp.dt * dt_scale
    inp32 = inp.astype(np.float32)
    inp32.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    inp32.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    return inp32, replace(DEFAULT, mix_len=mix_len)


def _exact_mass_of_f32_state(raw, inp, theta_offset=300.0):
    """The three mass sums of a stored state, exactly rounded (math.fsum) over
    the FP64 cell terms rho V, rho V (theta' + offset), rho V q formed from the
    stored values, V = dx dy dz_k.  raw: padded arrays (halo 2)."""
    nx, ny = inp.nx, inp.ny
    rho = raw["rho"][:, 2:2 + ny, 2:2 + nx].astype(np.float64)
    th = raw["theta"][:, 2:2 + ny, 2:2 + nx].astype(np.float64) + theta_offset
    q = raw["q"][:, 2:2 + ny, 2:2 + nx].astype(np.float64)
    m = rho * (inp.dx * inp.dx * inp.dz)[:, None, None]
    return np.array([math.fsum(m.ravel()), math.fsum((m * th).ravel()), math.fsum((m * q).ravel())])


@pytest.mark.parametrize("nx,ny,nz,phys", [(400, 320, 58, wx.WX_PHYS_PLAIN), (130, 66, 16, wx.WX_PHYS_PLAIN),
                                           (97, 45, 11, wx.WX_PHYS_PLAIN), (97, 45, 58, wx.WX_PHYS_OFF)])
def test_fp32_mass_sums_are_exact_sums_of_the_state(nx, ny, nz, phys):
    # The FP32 state's compensated FP64 sums against the exactly rounded sums
    # of the same stored values.  nz 58 and 16 take the register-column
    # physics (per-column FP64 sums folded into Neumaier sums), other nz the
    # general physics kernel (Neumaier per cell), physics off the mass pass;
    # every term is positive, so the bound is a few ulp of the total.
    _say(f"case: FP32 mass sums {nx}x{ny}x{nz} phys {phys}")
    inp = _f32_inputs(inputs.generate(nx, ny, nz, seed=33))
    st = wx.state_from_inputs(inp, dtype="f32", phys_mode=phys, theta_offset=300.0)
    st.step(2)
    mass = st.mass()
    raw = {name: st.download_raw(name) for name in ("rho", "theta", "q")}
    st.close()
    want = _exact_mass_of_f32_state(raw, inp)
    rel = np.abs(mass - want) / np.abs(want)
    _say(f"relative error of the mass sums {rel}")
    assert np.all(rel <= 1e-13), rel


@pytest.mark.parametrize("kernel", [0, 4])
@pytest.mark.parametrize("nz", [12, 16, 58])
def test_fp64_elimination_is_what_stiff_columns_need(nz, kernel):
    # Columns with dominance ratios r ~ 1e3 .. 4e4 (dt x 40, mixing length
    # 500 m), radiation off so the tendencies are the implicit diffusion alone.
    # The FP32 forward elimination loses about r * eps32 relative to the
    # solution (its rounding of each diagonal m + alpha_lo + alpha_hi is a
    # perturbation r times larger relative to the layer mass m), ~1e-4 here;
    # the FP64 elimination of the same FP32 inputs is limited by the FP32
    # inputs and the FP32 rounding of the stored result (the matrix is a
    # diagonally dominant M-matrix, whose solution is insensitive to relative
    # perturbations of its off-diagonals and of m), ~1e-7.  T_dd = 0 forces
    # every column through FP64, T_dd = 1e30 none; the counter says which.
    # (kernel 0: one thread per column; kernel 4: two lanes per column, the
    # elimination run from both ends; nz 12 takes the generic kernel)
    _say(f"case: stiff columns nz={nz} kernel {kernel}, forced FP32 and forced FP64 elimination")
    inp32, p = _stiff_f32_inputs(nz, 40.0, 500.0)
    inp32.f0[:] = 0.0
    ref = physics.column_physics(inp32.rho, inp32.theta, inp32.q, inp32.u, inp32.v, inp32.theta_s,
                                 inp32.q_s, inp32.f0, inp32.ch, inp32.dz, inp32.dt, p)
    assert ref.ratio.max() > 1e4 and ref.ratio.min() > 64
    ncol = inp32.nx * inp32.ny
    errs = {}
    for tdd in (0.0, 1e30):
        st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
        st.set_param("mix_len", p.mix_len)
        st.set_param("t_dd", tdd)
        st.set_param("phys_kernel", kernel)
        st.t["flags_out"].zero_()
        tt, tq = st.tendencies()
        flags = st.flags()
        st.close()
        assert flags["fp64_columns"] == (ncol if tdd == 0.0 else 0)
        errs[tdd] = (nmax(tt, ref.t_theta), nmax(tq, ref.t_q))
    _say(f"r in [{ref.ratio.min():.3g}, {ref.ratio.max():.3g}]; FP64 elimination errors {errs[0.0]}, "
         f"FP32 elimination errors {errs[1e30]}")
    assert max(errs[0.0]) <= 1e-6
    assert max(errs[1e30]) > 1e-5


@pytest.mark.parametrize("nz", [16, 58])
def test_stiff_step_fp64_branch_matches_oracle(nz):
    # A whole FP32 step (dycore, then physics updating the state in place)
    # with every column through the FP64 elimination: the mixing length 2000 m
    # makes r ~ 1e4, so the default T_dd = 64 picks FP64 for every column.
    # The state, its periodic halo images and the compensated mass sums must
    # match the oracle; forcing FP32 elimination misses the 1e-5 bar.
    _say(f"case: stiff FP32 step nz={nz} through the FP64 elimination branch")
    inp32, p = _stiff_f32_inputs(nz, 1.0, 2000.0, seed=32)
    ref = step.run(inp32, 1, p=p)
    cf = physics.diffusion_coeffs(ref.rho, inp32.u, inp32.v, inp32.ch, inp32.dz, inp32.dt, p)
    ncol = inp32.nx * inp32.ny
    res = {}
    for tdd in (64.0, 1e30):
        st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
        st.set_param("mix_len", p.mix_len)
        st.set_param("t_dd", tdd)
        st.step(1)
        gpu = st.download()
        flags = st.flags()
        mass = st.mass()
        raw = {name: st.download_raw(name)[:, :, :inp32.nx + 4] for name in ("rho", "theta", "q")}
        st.close()
        res[tdd] = (gpu, flags, mass, raw)
    gpu, flags, mass, raw = res[64.0]
    assert physics.dominance_ratio(cf).min() > 64.0
    assert flags["fp64_columns"] == ncol and flags["nonfinite"] == 0
    errs = _compare(gpu, ref, FP32_TOL, theta_ref=300.0)
    for name, a in raw.items():
        inner = a[:, 2:-2, 2:-2]
        np.testing.assert_array_equal(a, np.pad(inner, ((0, 0), (2, 2), (2, 2)), mode="wrap"))
    want = _exact_mass_of_f32_state(raw, inp32)
    rel = np.abs(mass - want) / np.abs(want)
    assert np.all(rel <= 1e-13), rel
    e32 = {k: nmax(res[1e30][0][k] - (300.0 if k == "theta" else 0.0),
                   getattr(ref, k) - (300.0 if k == "theta" else 0.0)) for k in ("rho", "theta", "q")}
    _say(f"FP64 branch errors {errs}, mass rel {rel}; forced FP32 elimination errors {e32}")
    assert res[1e30][1]["fp64_columns"] == 0
    assert max(e32["theta"], e32["q"]) > FP32_TOL


def test_fp64_column_count_matches_dominance_ratio():
    _say("case: FP64 column count at default T_dd on stiff columns")
    inp = inputs.generate(64, 32, 16, seed=29)
    inp.dt = inp.dt * 25.0
    ref = physics.column_physics(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, inp.dt)
    lo = int(np.sum(ref.ratio > DEFAULT.t_dd * (1 + 1e-6)))
    hi = int(np.sum(ref.ratio > DEFAULT.t_dd * (1 - 1e-6)))
    assert 0 < lo < inp.nx * inp.ny
    st = wx.state_from_inputs(inp, dtype="f64")
    st.t["flags_out"].zero_()
    st.tendencies()
    n = st.flags()["fp64_columns"]
    st.close()
    assert lo <= n <= hi


def test_mass_conservation_fp64_and_fp32_drift():
    _say("case: mass conservation FP64 10 steps, FP32 drift")
    inp = inputs.generate_config("tiny")
    inp.ch[:] = 0.0
    inp.f0[:] = 0.0
    m0 = step.masses(dycore.State(inp.rho, inp.theta, inp.q), inp)
    gpu = _run_gpu(inp, 10, "f64")
    rel = np.abs(gpu["mass"] - m0) / m0
    assert np.all(rel <= 1e-12), rel
    gpu32 = _run_gpu(inp, 10, "f32")
    rel32 = np.abs(gpu32["mass"] - m0) / m0
    _say(f"FP32 relative mass drift after 10 steps: {rel32}")
    assert np.all(rel32 <= 1e-5)


def test_nonfinite_input_is_flagged():
    _say("case: NaN flag")
    inp = inputs.generate(32, 16, 6, seed=30)
    inp.q[2, 5, 7] = np.nan
    gpu = _run_gpu(inp, 1, "f32")
    assert gpu["flags"]["nonfinite"] > 0


def test_wx_mass_entry_point():
    _say("case: wx_mass")
    inp = inputs.generate(33, 17, 7, seed=31)
    st = wx.state_from_inputs(inp, dtype="f64")
    m = st.mass(compute=True)
    st.close()
    np.testing.assert_allclose(m, mass_sums(inp.rho, inp.theta, inp.q, inp.dx, inp.dx, inp.dz),
                               rtol=1e-15)


def _f32_inputs(inp):
    """FP32-representable copy of a problem (theta rounded as theta - 300)."""
    out = inp.astype(np.float32)
    out.theta = (inp.theta - 300.0).astype(np.float32).astype(np.float64) + 300.0
    out.theta_s = (inp.theta_s - 300.0).astype(np.float32).astype(np.float64) + 300.0
    return out


def _crop_check(inp, gpu, nsteps, windows, tol):
    """Oracle on periodic crops enlarged by the light cone, compared inside.

    One step reads at most 2 cells around a cell per RK stage (6 per step);
    the physics is column-local, so a crop enlarged by 6 n cells on each side
    reproduces the full-grid result in its inner window.
    """
    m = 6 * nsteps
    worst = {}
    for (i0, j0, cx, cy) in windows:
        sub = inputs.crop(inp, i0 - m, j0 - m, cx + 2 * m, cy + 2 * m)
        ref = step.run(sub, nsteps)
        ii = np.arange(i0, i0 + cx) % inp.nx
        jj = np.arange(j0, j0 + cy) % inp.ny
        for name in ("rho", "theta", "q"):
            g = gpu[name][:, jj][:, :, ii]
            r = getattr(ref, name)[:, m:m + cy, m:m + cx]
            off = 300.0 if name == "theta" else 0.0
            e = nmax(g - off, r - off)
            worst[name] = max(worst.get(name, 0.0), e)
    for k, e in worst.items():
        assert e <= tol, worst
    return worst


def test_share_grid_fp32_crops():
    # 400 x 320 x 58: one GPU's share of the 1581 x 1301 grid
    _say("case: 400x320x58 FP32 1 step, crops")
    inp = _f32_inputs(inputs.generate_config("share"))
    gpu = _run_gpu(inp, 1, "f32", theta_offset=300.0)
    w = [(0, 0, 40, 40), (380, 300, 40, 40), (197, 123, 48, 32)]
    worst = _crop_check(inp, gpu, 1, w, FP32_TOL)
    _say(f"share grid fp32 errors {worst}")


def test_share_grid_fp64_three_steps_crops():
    _say("case: 400x320x58 FP64 3 steps, crops")
    inp = inputs.generate_config("share")
    gpu = _run_gpu(inp, 3, "f64")
    worst = _crop_check(inp, gpu, 3, [(390, 5, 24, 24), (150, 160, 24, 24)], FP64_TOL)
    _say(f"share grid fp64 errors {worst}")


def test_full_grid_fp32_crops_and_mass():
    # the benchmark's workload: 1581 x 1301 x 58 in FP32, one step
    _say("case: 1581x1301x58 FP32 1 step, crops")
    inp = inputs.generate_config("full", dtype=np.float32)
    inp64 = inp.astype(np.float64)
    inp64.theta = (inp.theta.astype(np.float64) - 300.0).astype(np.float32).astype(np.float64) + 300.0
    inp64.theta_s = (inp.theta_s.astype(np.float64) - 300.0).astype(np.float32).astype(np.float64) + 300.0
    st = wx.state_from_inputs(inp64, dtype="f32", theta_offset=300.0)
    m0 = st.mass(compute=True)
    st.step(1)
    gpu = st.download()
    flags = st.flags()
    m1 = st.mass()
    raw = {name: st.download_raw(name) for name in ("rho", "theta", "q")}
    st.close()
    del inp
    assert flags["nonfinite"] == 0 and flags["rho_le0"] == 0
    # density is conserved exactly by the dycore and untouched by the physics
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-6
    # the production sums equal the exactly rounded sums of the stored state
    want = _exact_mass_of_f32_state(raw, inp64)
    del raw
    rel = np.abs(m1 - want) / np.abs(want)
    _say(f"full grid mass sums, relative error against exact sums {rel}")
    assert np.all(rel <= 1e-13), rel
    w = [(0, 0, 32, 32), (1565, 1285, 32, 32), (790, 650, 32, 32), (1500, 20, 32, 32)]
    worst = _crop_check(inp64, gpu, 1, w, FP32_TOL)
    _say(f"full grid fp32 errors {worst}")


@pytest.mark.parametrize("nz", [16, 58])
def test_step_stays_inside_its_workspace(nz):
    # wx_step (stage tiles of both shapes, both walk directions, the two-lane
    # physics with its block partials) and wx_physics tendencies on a ragged
    # grid: a guard band after the wx_workspace_bytes the state was given
    # comes back untouched
    _say(f"case: state workspace bounds nz={nz}")
    import torch
    inp = _f32_inputs(inputs.generate(97, 23, nz, seed=48))
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    nb = st.t["workspace"].numel()
    guard = 1 << 16
    big = torch.full((nb + guard,), 0xA5, dtype=torch.uint8, device=st.device)
    st.t["workspace"] = big[:nb]
    st._p.contents.workspace = big.data_ptr()
    st.step(3)
    st.tendencies()
    torch.cuda.synchronize()
    tail = big[nb:].cpu().numpy()
    st.close()
    assert np.all(tail == 0xA5), f"{int(np.sum(tail != 0xA5))} guard bytes written"


@pytest.mark.parametrize("tile", [1, 2, 3, 4])
def test_stage_tile_shapes_bitwise(tile):
    # the stage kernel's tile-shape ablation: each cell's arithmetic does not
    # depend on the tile, so every shape gives the production tile's bytes
    # (ragged tiles in i and j, FP32 and FP64)
    for dtype, (nx, ny, nz) in (("f32", (150, 37, 12)), ("f64", (67, 29, 7))):
        _say(f"case: stage tile {tile} vs tile 0, {nx}x{ny}x{nz} {dtype}")
        inp = inputs.generate(nx, ny, nz, seed=40 + tile)
        outs = []
        for t in (0, tile):
            st = wx.state_from_inputs(inp, dtype=dtype)
            st.set_param("stage_tile", t)
            st.step(2)
            outs.append({n: st.download_raw(n) for n in ("rho", "theta", "q")})
            outs[-1]["mass"] = st.mass_raw()
            st.close()
        for n in ("rho", "theta", "q", "mass"):
            np.testing.assert_array_equal(outs[0][n], outs[1][n])


@pytest.mark.parametrize("nz", [16, 58])
def test_physics_kernel_variants_bitwise(nz):
    # the physics kernel that reads the column again on the way down (two
    # waves per SIMD) and the one whose upward pass fetches whole rows with
    # 16-byte loads do the same arithmetic as the one that keeps the column
    # in registers: same state, mass sums, counters and tendencies (130 x 21:
    # the last tile has 2 live columns of 64, the last row of tiles 1 live row
    # of 4)
    _say(f"case: physics kernel variants nz={nz}")
    inp = _f32_inputs(inputs.generate(130, 21, nz, seed=44))
    res = []
    for v in (0, 1, 3):
        st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
        st.set_param("phys_kernel", v)
        tt, tq = st.tendencies()
        st.step(2)
        res.append(({n: st.download_raw(n) for n in ("rho", "theta", "q")}, st.mass_raw(), st.flags(), tt, tq))
        st.close()
    for other in res[1:]:
        for n in ("rho", "theta", "q"):
            np.testing.assert_array_equal(res[0][0][n], other[0][n])
        np.testing.assert_array_equal(res[0][1], other[1])
        assert res[0][2] == other[2]
        np.testing.assert_array_equal(res[0][3], other[3])
        np.testing.assert_array_equal(res[0][4], other[4])


def test_shared_face_stage_kernel_matches_oracle():
    # the variant that forms each face, mass flux and Laplacian once per tile
    # in LDS: the same formulas, but a value read back from LDS is rounded
    # where the per-cell kernel could fuse its last multiply into the next
    # add, so it agrees with the oracle at the usual bars rather than with
    # the per-cell kernel bit for bit; it is reproducible run to run
    _say("case: shared-face stage kernel, FP64 3 steps ragged, FP32 1 step")
    inp = inputs.generate(67, 37, 7, seed=45)
    st = wx.state_from_inputs(inp, dtype="f64")
    st.set_param("stage_tile", 5)
    st.step(3)
    gpu = st.download()
    st.close()
    _compare(gpu, _oracle(inp, 3), FP64_TOL)
    inp32 = _f32_inputs(inputs.generate(150, 37, 12, seed=46))
    outs = []
    for _ in range(2):
        st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
        st.set_param("stage_tile", 5)
        st.step(1)
        outs.append((st.download(), st.download_raw("theta")))
        st.close()
    errs = _compare(outs[0][0], _oracle(inp32, 1), FP32_TOL, theta_ref=300.0)
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    _say(f"shared-face fp32 errors {errs}")


@pytest.mark.parametrize("nz", [16, 58])
def test_split_physics_kernel_matches_oracle(nz):
    # two lanes per column, the elimination run from the ground and from the
    # lid and joined at mid-column: the same arithmetic in another order, so
    # the FP32 bar against the oracle (state after a step, tendencies), mass
    # sums equal to the exactly rounded sums of the stored state, the
    # counters and the halo ring; 97 x 23 leaves one live column in the last
    # tile of 32 and three live rows in the last row of tiles; on stiff
    # columns the whole-column FP64 path meets the tight bar with every
    # column counted
    _say(f"case: split physics kernel nz={nz}")
    inp = _f32_inputs(inputs.generate(97, 23, nz, seed=48))
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    st.set_param("phys_kernel", 4)
    tt, tq = st.tendencies()
    st.step(1)
    gpu = st.download()
    mass = st.mass()
    raw = {name: st.download_raw(name) for name in ("rho", "theta", "q")}
    flags = st.flags()
    st.close()
    ref = physics.column_physics(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, inp.dt)
    e_t = (nmax(tt, ref.t_theta), nmax(tq, ref.t_q))
    errs = _compare(gpu, _oracle(inp, 1), FP32_TOL, theta_ref=300.0)
    want = _exact_mass_of_f32_state(raw, inp)
    rel = np.abs(mass - want) / np.abs(want)
    _say(f"split kernel: tendency errors {e_t}, state errors {errs}, mass rel {rel}")
    assert max(e_t) <= FP32_TOL
    assert np.all(rel <= 1e-13), rel
    assert flags["nonfinite"] == 0 and flags["rho_le0"] == 0 and flags["fp64_columns"] == 0
    for name, a in raw.items():
        inner = a[:, 2:-2, 2:2 + inp.nx]
        np.testing.assert_array_equal(a[:, :, :inp.nx + 4], np.pad(inner, ((0, 0), (2, 2), (2, 2)), mode="wrap"))
    # stiff columns: FP64 for the whole column
    inp32, p = _stiff_f32_inputs(nz, 40.0, 500.0)
    inp32.f0[:] = 0.0
    ref = physics.column_physics(inp32.rho, inp32.theta, inp32.q, inp32.u, inp32.v, inp32.theta_s,
                                 inp32.q_s, inp32.f0, inp32.ch, inp32.dz, inp32.dt, p)
    st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
    st.set_param("mix_len", p.mix_len)
    st.set_param("phys_kernel", 4)
    st.t["flags_out"].zero_()
    tt, tq = st.tendencies()
    n64 = st.flags()["fp64_columns"]
    st.close()
    e64 = (nmax(tt, ref.t_theta), nmax(tq, ref.t_q))
    _say(f"stiff columns, split kernel: errors {e64}, FP64 columns {n64} of {inp32.nx * inp32.ny}")
    assert n64 == int(np.sum(ref.ratio > DEFAULT.t_dd))
    assert max(e64) <= 1e-6


@pytest.mark.parametrize("nz", [16, 58, 11])
def test_scan_physics_kernel_matches_oracle(nz):
    # one wave per column, the elimination, back substitution and optical
    # depth as lane scans: the same arithmetic in another order, so the FP32
    # bar against the oracle (state after a step, tendencies), mass sums equal
    # to the exactly rounded sums of the stored state, the counters; and on
    # stiff columns the FP64 scans meet the tight bar the FP64 elimination
    # meets, with every column counted
    _say(f"case: scan physics kernel nz={nz}")
    inp = _f32_inputs(inputs.generate(97, 23, nz, seed=47))
    st = wx.state_from_inputs(inp, dtype="f32", theta_offset=300.0)
    st.set_param("phys_kernel", 2)
    tt, tq = st.tendencies()
    st.step(1)
    gpu = st.download()
    mass = st.mass()
    raw = {name: st.download_raw(name) for name in ("rho", "theta", "q")}
    flags = st.flags()
    st.close()
    ref = physics.column_physics(inp.rho, inp.theta, inp.q, inp.u, inp.v, inp.theta_s, inp.q_s,
                                 inp.f0, inp.ch, inp.dz, inp.dt)
    e_t = (nmax(tt, ref.t_theta), nmax(tq, ref.t_q))
    errs = _compare(gpu, _oracle(inp, 1), FP32_TOL, theta_ref=300.0)
    want = _exact_mass_of_f32_state(raw, inp)
    rel = np.abs(mass - want) / np.abs(want)
    _say(f"scan kernel: tendency errors {e_t}, state errors {errs}, mass rel {rel}")
    assert max(e_t) <= FP32_TOL
    assert np.all(rel <= 1e-13), rel
    assert flags["nonfinite"] == 0 and flags["rho_le0"] == 0
    for name, a in raw.items():
        inner = a[:, 2:-2, 2:2 + inp.nx]
        np.testing.assert_array_equal(a[:, :, :inp.nx + 4], np.pad(inner, ((0, 0), (2, 2), (2, 2)), mode="wrap"))
    # stiff columns: FP64 scans
    inp32, p = _stiff_f32_inputs(nz, 40.0, 500.0)
    inp32.f0[:] = 0.0
    ref = physics.column_physics(inp32.rho, inp32.theta, inp32.q, inp32.u, inp32.v, inp32.theta_s,
                                 inp32.q_s, inp32.f0, inp32.ch, inp32.dz, inp32.dt, p)
    st = wx.state_from_inputs(inp32, dtype="f32", theta_offset=300.0)
    st.set_param("mix_len", p.mix_len)
    st.set_param("phys_kernel", 2)
    st.t["flags_out"].zero_()
    tt, tq = st.tendencies()
    n64 = st.flags()["fp64_columns"]
    st.close()
    e64 = (nmax(tt, ref.t_theta), nmax(tq, ref.t_q))
    _say(f"stiff columns, FP64 scans: errors {e64}, FP64 columns {n64} of {inp32.nx * inp32.ny}")
    assert n64 == int(np.sum(ref.ratio > DEFAULT.t_dd))
    assert max(e64) <= 1e-6
