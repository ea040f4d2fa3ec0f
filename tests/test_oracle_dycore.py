"""Pins of the oracle dycore against closed forms and invariants (CPU only).

Each test checks something fixed by mathematics, not by re-typing the
oracle's formulas: polynomial exactness of the third-order face values,
von Neumann amplification of a Fourier mode under RK3, the textbook 13-point
biharmonic stencil, a manufactured density-weighting case, exact
conservation, exact preservation of constants, and translation invariance.
"""
import numpy as np
import pytest

from oracle import dycore, step
from oracle.params import DEFAULT
from paper_1802_05839_amd import inputs
from tests._util import nmax, uniform_inputs


def _cell_avg_quadratic(n, c0, c1, c2):
    """Cell averages over [i-1/2, i+1/2] of c0 + c1 x + c2 x^2 (x in index units)."""
    x = np.arange(n, dtype=np.float64)
    return c0 + c1 * x + c2 * (x * x + 1.0 / 12.0)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_upwind3_exact_for_quadratic_cell_averages(sign):
    # A third-order reconstruction from cell averages returns the exact point
    # value of any quadratic at the face, for either upwind direction.
    n = 40
    c0, c1, c2 = 0.7, -1.3, 0.05
    phi = _cell_avg_quadratic(n, c0, c1, c2)[None, None, :]
    vel = np.full_like(phi, sign)
    f = dycore.upwind3_face(phi, vel, axis=2)[0, 0]
    xf = np.arange(n) + 0.5
    exact = c0 + c1 * xf + c2 * xf * xf
    sl = slice(2, n - 3)       # away from the periodic wrap
    np.testing.assert_allclose(f[sl], exact[sl], rtol=0, atol=1e-12)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_vertical_faces_exact_for_quadratic_and_linear(sign):
    nz = 12
    c0, c1, c2 = 1.5, 0.4, -0.02
    phi = _cell_avg_quadratic(nz, c0, c1, c2)[:, None, None]
    w = np.full((nz + 1, 1, 1), sign)
    f = dycore.vertical_faces(phi, w)[:, 0, 0]
    xf = np.arange(nz + 1) - 0.5           # face f lies at level f - 1/2
    exact = c0 + c1 * xf + c2 * xf * xf
    # upwind faces 2 .. nz-2 are exact for quadratics
    np.testing.assert_allclose(f[2:nz - 1], exact[2:nz - 1], rtol=0, atol=1e-12)
    # the centred faces next to the ground and lid are exact for linear profiles
    lin = (c0 + c1 * np.arange(nz))[:, None, None]
    fl = dycore.vertical_faces(lin, w)[:, 0, 0]
    np.testing.assert_allclose(fl[[1, nz - 1]], (c0 + c1 * xf)[[1, nz - 1]], rtol=0, atol=1e-13)


def _symbol_upwind(theta, positive):
    """Fourier symbol of (phi_{f,i+1/2} - phi_{f,i-1/2}) for third-order upwind faces.

    Cell-average reconstruction weights: (-1, 5, 2)/6 on (i-1, i, i+1) for
    positive velocity, (2, 5, -1)/6 on (i, i+1, i+2) for negative.
    """
    e = np.exp(1j * theta)
    face = (-1.0 / e + 5.0 + 2.0 * e) / 6.0 if positive else (2.0 + 5.0 * e - e * e) / 6.0
    return (1.0 - 1.0 / e) * face


@pytest.mark.parametrize("mx,my,u0,v0", [(1, 0, 12.0, 0.0), (3, 2, 8.0, -5.0), (5, 7, -9.0, 4.0),
                                          (16, 0, 10.0, 3.0), (16, 12, -6.0, -7.0),
                                          (0, 12, 2.0, 9.0)])
def test_fourier_mode_amplification_rk3(mx, my, u0, v0):
    # P4: uniform rho, uniform winds, w = 0, physics off.  A Fourier mode is an
    # eigenfunction of the linear stage operator L with eigenvalue
    # lambda = -(u0/dx) S_x - (v0/dy) S_y - K4 s^2, and WS-RK3 multiplies it by
    # G = 1 + z + z^2/2 + z^3/6, z = dt lambda, per step.  mx = nx/2 is the
    # 2 dx wave.
    nx, ny, nz = 32, 24, 3
    dx = 2000.0
    dt = 0.3 / (abs(u0) / dx + abs(v0) / dx)
    inp = uniform_inputs(nx=nx, ny=ny, nz=nz, dx=dx, dt=dt, u0=u0, v0=v0, rho0=1.1)
    tx, ty = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    ii = np.arange(nx)[None, None, :]
    jj = np.arange(ny)[None, :, None]
    amp = 0.37
    phase = tx * ii + ty * jj + 0.3
    inp.theta = np.broadcast_to(amp * np.cos(phase), (nz, ny, nx)).copy()
    k4 = DEFAULT.k4(dx, dt)
    s = (4.0 / dx ** 2) * (np.sin(tx / 2) ** 2 + np.sin(ty / 2) ** 2)
    lam = (-(u0 / dx) * _symbol_upwind(tx, u0 >= 0) - (v0 / dx) * _symbol_upwind(ty, v0 >= 0)
           - k4 * s * s)
    z = dt * lam
    g = 1.0 + z + z * z / 2.0 + z ** 3 / 6.0
    nsteps = 10
    out = step.run(inp, nsteps, physics_on=False)
    expect = np.real(amp * g ** nsteps * np.exp(1j * phase))
    err = np.max(np.abs(out.theta - np.broadcast_to(expect, out.theta.shape)))
    assert err <= 1e-12 * amp, err
    np.testing.assert_array_equal(out.rho, inp.rho)


def test_biharmonic_textbook_stencil():
    # With uniform density the biharmonic term is -K4 times the 13-point
    # del^4 stencil: 20 at the centre, -8 at the 4 neighbours, 2 at the 4
    # diagonals and 1 at distance 2 along the axes (all / dx^4).
    n = 11
    dx = 3.0
    phi = np.zeros((1, n, n))
    phi[0, 5, 5] = 1.0
    rho = np.full_like(phi, 1.7)
    k4 = 0.25
    b = dycore.biharmonic_tendency(phi, rho, k4, dx, dx)[0] / (-k4 * 1.7) * dx ** 4
    expect = np.zeros((n, n))
    expect[5, 5] = 20.0
    for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        expect[5 + dj, 5 + di] = -8.0
        expect[5 + 2 * dj, 5 + 2 * di] = 1.0
    for dj, di in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
        expect[5 + dj, 5 + di] = 2.0
    np.testing.assert_allclose(b, expect, rtol=0, atol=1e-11)


def test_biharmonic_density_weighting_cubic():
    # phi = x^3/6 has Laplacian exactly x; then G_{i+1/2} = K4 rho_{i+1/2} and
    # B_i = -K4 (rho_{i+1} - rho_{i-1}) / (2 dx) when the face density is the
    # arithmetic mean of the two cells.
    n = 40
    dx = 2.0
    x = np.arange(n) * dx
    phi = np.broadcast_to((x ** 3 / 6.0)[None, None, :], (1, 5, n)).copy()
    rho_x = 1.0 + 0.3 * np.sin(0.37 * np.arange(n)) + 0.01 * np.arange(n)
    rho = np.broadcast_to(rho_x[None, None, :], (1, 5, n)).copy()
    k4 = 1.3
    b = dycore.biharmonic_tendency(phi, rho, k4, dx, dx)[0, 2]
    expect = -k4 * (np.roll(rho_x, -1) - np.roll(rho_x, 1)) / (2 * dx)
    sl = slice(4, n - 4)
    np.testing.assert_allclose(b[sl], expect[sl], rtol=1e-9, atol=1e-9)


def test_vertical_advection_linear_profile_single_stage():
    # Upward wind w0 on interior faces, uniform dz and rho, theta linear in k:
    # every face value is exact, so with F = w0 rho inside and 0 at the ground
    # and lid:  rho_new = rho -/+ h w0 rho/dz at the bottom/top level (0 inside)
    # and A = -(b/2)(F_up + F_down)/dz, i.e. -w0 rho b/dz inside.
    nz, h, w0, rho0, dzv, a, bgrad = 9, 3.0, 0.4, 1.2, 100.0, 290.0, 0.7
    dz = np.full(nz, dzv)
    inp = uniform_inputs(nx=6, ny=5, nz=nz, dz=dz, rho0=rho0)
    inp.w[1:nz] = w0
    th = (a + bgrad * np.arange(nz))[:, None, None] * np.ones((nz, 5, 6))
    s = dycore.State(inp.rho.copy(), th, inp.q.copy())
    k4 = 0.0
    out = dycore.stage(s, s, inp.u, inp.v, inp.w, inp.dx, inp.dx, dz, h, k4)
    rho_exp = np.full(nz, rho0)
    rho_exp[0] -= h * w0 * rho0 / dzv
    rho_exp[-1] += h * w0 * rho0 / dzv
    f_up = np.full(nz, w0 * rho0)
    f_up[-1] = 0.0
    f_dn = np.full(nz, w0 * rho0)
    f_dn[0] = 0.0
    a_term = -(bgrad / 2.0) * (f_up + f_dn) / dzv
    th_exp = (a + bgrad * np.arange(nz)) + h * a_term / rho_exp
    np.testing.assert_allclose(out.rho[:, 2, 3], rho_exp, rtol=1e-14)
    np.testing.assert_allclose(out.theta[:, 2, 3], th_exp, rtol=1e-14)
    # q is uniform: unchanged bitwise
    np.testing.assert_array_equal(out.q, s.q)


def _random_small(seed=5, nx=24, ny=20, nz=10):
    return inputs.generate(nx, ny, nz, seed=seed)


def test_constant_field_preserved_bitwise():
    # P2: theta and q constant, any winds and density, surface values equal to
    # the constants and no radiation: the whole step leaves them bit-identical.
    inp = _random_small()
    inp.theta[:] = 287.25
    inp.q[:] = 0.0075
    inp.theta_s[:] = 287.25
    inp.q_s[:] = 0.0075
    inp.f0[:] = 0.0
    out = step.run(inp, 3)
    np.testing.assert_array_equal(out.theta, inp.theta)
    np.testing.assert_array_equal(out.q, inp.q)
    assert not np.array_equal(out.rho, inp.rho)      # density did move


def test_uniform_state_preserved_bitwise():
    # P3: every field uniform, w = 0: nothing changes.
    inp = uniform_inputs(nx=10, ny=9, nz=7, u0=7.5, v0=-3.25, rho0=1.05, theta0=301.5, q0=0.004)
    out = step.run(inp, 2)
    np.testing.assert_array_equal(out.rho, inp.rho)
    np.testing.assert_array_equal(out.theta, inp.theta)
    np.testing.assert_array_equal(out.q, inp.q)


def test_mass_conservation_ten_steps():
    # P1: periodic boundaries, no surface exchange and no radiation: total
    # mass, rho*theta and rho*q are conserved to rounding.
    inp = inputs.generate_config("tiny")
    inp.ch[:] = 0.0
    inp.f0[:] = 0.0
    s0 = dycore.State(inp.rho, inp.theta, inp.q)
    m0 = step.masses(s0, inp)
    out = step.run(inp, 10)
    m1 = step.masses(out, inp)
    rel = np.abs(m1 - m0) / np.abs(m0)
    assert np.all(rel <= 1e-12), rel


def test_mass_changes_only_by_surface_and_radiation():
    # With exchange and radiation on, rho is still conserved exactly (physics
    # does not touch rho) while rho*theta changes.
    inp = inputs.generate_config("tiny")
    s0 = dycore.State(inp.rho, inp.theta, inp.q)
    m0 = step.masses(s0, inp)
    out = step.run(inp, 2)
    m1 = step.masses(out, inp)
    assert abs(m1[0] - m0[0]) / m0[0] <= 1e-13
    assert abs(m1[1] - m0[1]) / m0[1] > 1e-9


def test_translation_invariance_bitwise():
    # P5: shifting every input by (p, q) cells shifts the result by (p, q).
    inp = _random_small(seed=7, nx=20, ny=16, nz=6)
    p, qq = 5, 3
    sh = inp.copy()
    for name, a in sh.fields().items():
        setattr(sh, name, np.roll(np.roll(a, qq, axis=-2), p, axis=-1))
    o1 = step.run(inp, 2)
    o2 = step.run(sh, 2)
    for a, b in zip(o1, o2):
        np.testing.assert_array_equal(np.roll(np.roll(a, qq, axis=-2), p, axis=-1), b)


def test_theta_offset_invariance():
    # The step only sees differences of theta (increment-form transport,
    # delta-form diffusion toward theta_s, additive heating): theta + c in,
    # theta + c out.  This is what lets the FP32 path store theta - 300.
    inp = _random_small(seed=9, nx=16, ny=16, nz=8)
    sh = inp.copy()
    sh.theta = sh.theta - 300.0
    sh.theta_s = sh.theta_s - 300.0
    o1 = step.run(inp, 2)
    o2 = step.run(sh, 2)
    assert nmax(o2.theta + 300.0, o1.theta) <= 1e-14
    assert np.max(np.abs((o2.theta + 300.0) - o1.theta)) <= 1e-10
    np.testing.assert_allclose(o2.q, o1.q, rtol=1e-12, atol=0)
