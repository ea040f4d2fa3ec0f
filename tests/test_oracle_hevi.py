"""Pins of the HEVI fast-mode oracle (CPU only).

Each pin follows from the continuous system or from the scheme's Fourier
symbol, independently of the oracle's array code:
* a vertical normal mode between rigid lids (uniform levels, no horizontal
  variation) is an eigenvector of the vertical operator with frequency
  omega^2 = N^2 + c^2 k_d^2, k_d = (2/dz) sin(kappa dz / 2); the trapezoidal
  step multiplies it by (1 + i omega tau/2)/(1 - i omega tau/2) per step;
* a horizontal acoustic mode (no vertical variation) follows the 2x2
  amplification matrix of the two forward-backward stages;
* the vertical part alone conserves the discrete energy exactly on any
  stretched column (the trapezoidal rule keeps the quadratic invariant of a
  skew-adjoint system) -- which fixes the face and cell weights dz_{k+1/2},
  dz_k of the vertical differences;
* a linear pressure profile in hydrostatic balance with the buoyancy is an
  exact steady state on stretched levels (fixes the distance between cell
  centres as the face spacing);
* a single three-dimensional mode (one horizontal wave times one vertical
  normal mode) follows the 4x4 stage map written out from the symbols of the
  differences (fixes the coupling of the horizontal divergence into the
  vertical implicit solve);
* the mean of pi is conserved; a shifted state gives the shifted result.
"""
import numpy as np
import pytest

from oracle import hevi

C, N = hevi.C_SOUND, hevi.N_BV


def _zeros(nx, ny, nz):
    z = np.zeros((nz, ny, nx))
    zf = np.zeros((nz + 1, ny, nx))
    return hevi.Fast(z.copy(), z.copy(), zf.copy(), zf.copy(), z.copy())


def test_rest_stays_at_rest():
    x = _zeros(5, 4, 6)
    out = hevi.run(x, 3, 2000.0, 2000.0, np.full(6, 100.0), 2.0)
    for f in out:
        assert np.all(f == 0.0)


@pytest.mark.parametrize("m,tau,nsteps", [(1, 2.0, 7), (3, 1.5, 5), (7, 3.0, 4)])
def test_vertical_normal_mode_closed_form(m, tau, nsteps):
    nz, dzv = 16, 250.0
    height = nz * dzv
    kappa = m * np.pi / height
    kd = (2.0 / dzv) * np.sin(kappa * dzv / 2.0)
    omega = np.sqrt(N * N + C * C * kd * kd)
    e = np.array([1.0, 1j * N * N / omega, 1j * C * C * kd / omega])     # (W, B, Pi)
    zc = (np.arange(nz) + 0.5) * dzv
    zf = np.arange(nz + 1) * dzv

    def state(amp):
        x = _zeros(3, 2, nz)
        w = np.real(amp[0] * np.sin(kappa * zf))
        b = np.real(amp[1] * np.sin(kappa * zf))
        p = np.real(amp[2] * np.cos(kappa * zc))
        return hevi.Fast(x.u, x.v, np.broadcast_to(w[:, None, None], x.w.shape).copy(),
                         np.broadcast_to(b[:, None, None], x.b.shape).copy(),
                         np.broadcast_to(p[:, None, None], x.pi.shape).copy())

    g = (1.0 + 0.5j * omega * tau) / (1.0 - 0.5j * omega * tau)
    got = hevi.run(state(e), nsteps, 2000.0, 2000.0, np.full(nz, dzv), tau)
    want = state(g ** nsteps * e)
    for name in ("w", "b", "pi"):
        a, r = getattr(got, name), getattr(want, name)
        assert np.max(np.abs(a - r)) <= 1e-12 * np.max(np.abs(r)), name
    assert np.all(got.u == 0.0) and np.all(got.v == 0.0)


@pytest.mark.parametrize("axis,mx,tau", [("x", 1, 2.0), ("x", 5, 2.5), ("y", 3, 1.0), ("x", 8, 1.5)])
def test_horizontal_acoustic_mode_closed_form(axis, mx, tau):
    # pi_i = Re(P e^{i theta i}) at centres, wind Re(U e^{i theta (i + 1/2)}) at
    # faces: the difference operators act as multiplication by i s with
    # s = 2 sin(theta/2)/dx.  Stage h: U' = U0 - h i s P_prev,
    # P' = P0 - h c^2 i s U'; stages h = tau/2 then tau from the base.
    nx = ny = 16
    nz, dx = 3, 2000.0
    n = nx if axis == "x" else ny
    theta = 2.0 * np.pi * mx / n
    s = 2.0 * np.sin(theta / 2.0) / dx

    def stage(u0, p0, p_prev, h):
        u1 = u0 - h * 1j * s * p_prev
        return u1, p0 - h * C * C * 1j * s * u1

    u0, p0 = 0.3 + 0.1j, 1.0 - 0.4j
    u, p = u0, p0
    nsteps = 6
    for _ in range(nsteps):
        u1, p1 = stage(u, p, p, tau / 2.0)
        u, p = stage(u, p, p1, tau)

    idx = np.arange(n)

    def fields(uu, pp):
        x = _zeros(nx, ny, nz)
        wave_c = np.real(pp * np.exp(1j * theta * idx))
        wave_f = np.real(uu * np.exp(1j * theta * (idx + 0.5)))
        if axis == "x":
            pi = np.broadcast_to(wave_c[None, None, :], x.pi.shape).copy()
            return hevi.Fast(np.broadcast_to(wave_f[None, None, :], x.u.shape).copy(), x.v, x.w, x.b, pi)
        pi = np.broadcast_to(wave_c[None, :, None], x.pi.shape).copy()
        return hevi.Fast(x.u, np.broadcast_to(wave_f[None, :, None], x.v.shape).copy(), x.w, x.b, pi)

    got = hevi.run(fields(u0, p0), nsteps, dx, dx, np.array([40.0, 90.0, 300.0]), tau)
    want = fields(u, p)
    wind = "u" if axis == "x" else "v"
    for name in (wind, "pi"):
        a, r = getattr(got, name), getattr(want, name)
        assert np.max(np.abs(a - r)) <= 1e-12 * np.max(np.abs(r)), name
    assert np.max(np.abs(got.w)) <= 1e-12 * np.max(np.abs(want.pi)) / C


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vertical_part_conserves_energy_on_stretched_columns(seed):
    rng = np.random.default_rng(seed)
    nz = 20
    dz = 50.0 * (20.0 ** (1.0 / (nz - 1))) ** np.arange(nz)
    x = _zeros(1, 1, nz)
    w = np.zeros(nz + 1)
    b = np.zeros(nz + 1)
    w[1:nz] = rng.normal(0, 0.5, nz - 1)
    b[1:nz] = rng.normal(0, 0.01, nz - 1)
    p = rng.normal(0, 50.0, nz)
    x = hevi.Fast(x.u, x.v, w.reshape(-1, 1, 1), b.reshape(-1, 1, 1), p.reshape(-1, 1, 1))
    e0 = hevi.energy(x, 2000.0, 2000.0, dz)
    out = hevi.run(x, 10, 2000.0, 2000.0, dz, 3.0)
    e1 = hevi.energy(out, 2000.0, 2000.0, dz)
    assert abs(e1 - e0) <= 1e-13 * e0
    # and the scheme does move the state (c tau / dz ~ 20 at the ground)
    assert np.max(np.abs(out.w - x.w)) > 1e-3


def test_mean_pressure_is_conserved():
    rng = np.random.default_rng(4)
    nx, ny, nz = 12, 9, 7
    dz = np.linspace(60.0, 400.0, nz)
    x = hevi.Fast(rng.normal(0, 3, (nz, ny, nx)), rng.normal(0, 3, (nz, ny, nx)),
                  np.concatenate([np.zeros((1, ny, nx)), rng.normal(0, 0.3, (nz - 1, ny, nx)),
                                  np.zeros((1, ny, nx))]),
                  np.concatenate([np.zeros((1, ny, nx)), rng.normal(0, 0.01, (nz - 1, ny, nx)),
                                  np.zeros((1, ny, nx))]),
                  rng.normal(0, 40, (nz, ny, nx)))
    vol = dz[:, None, None] * np.ones((nz, ny, nx))
    out = hevi.run(x, 5, 2000.0, 2000.0, dz, 2.0)
    assert abs(np.sum(out.pi * vol) - np.sum(x.pi * vol)) <= 1e-12 * np.sum(np.abs(x.pi) * vol)
    assert np.all(out.w[0] == 0.0) and np.all(out.w[nz] == 0.0)


def test_translation_invariance_bitwise():
    rng = np.random.default_rng(5)
    nx, ny, nz = 10, 8, 5
    dz = np.linspace(60.0, 300.0, nz)
    x = hevi.Fast(rng.normal(0, 3, (nz, ny, nx)), rng.normal(0, 3, (nz, ny, nx)),
                  np.concatenate([np.zeros((1, ny, nx)), rng.normal(0, 0.3, (nz - 1, ny, nx)),
                                  np.zeros((1, ny, nx))]),
                  np.zeros((nz + 1, ny, nx)), rng.normal(0, 40, (nz, ny, nx)))
    sh = hevi.Fast(*(np.roll(np.roll(f, 3, axis=2), 2, axis=1) for f in x))
    a = hevi.run(x, 2, 2000.0, 2000.0, dz, 2.0)
    b = hevi.run(sh, 2, 2000.0, 2000.0, dz, 2.0)
    for fa, fb in zip(a, b):
        np.testing.assert_array_equal(np.roll(np.roll(fa, 3, axis=2), 2, axis=1), fb)


def test_hydrostatic_balance_is_steady_on_stretched_levels():
    # pi = alpha z (z at cell centres) with b = alpha on every interior face
    # and no motion is an exact steady state: the vertical pressure gradient
    # at a face, (pi_{k+1} - pi_k) / (distance between the two centres),
    # equals alpha, and the centres of a stretched column lie
    # (dz_k + dz_{k+1})/2 apart.
    nz = 12
    dz = 50.0 * 1.4 ** np.arange(nz)
    zc = np.concatenate(([0.0], np.cumsum(dz)[:-1])) + dz / 2.0
    alpha = 0.0123
    x = _zeros(4, 3, nz)
    b = np.zeros(nz + 1)
    b[1:nz] = alpha
    pi = np.broadcast_to((alpha * zc)[:, None, None], x.pi.shape).copy()
    x = hevi.Fast(x.u, x.v, x.w, np.broadcast_to(b[:, None, None], x.b.shape).copy(), pi)
    out = hevi.run(x, 5, 2000.0, 2000.0, dz, 2.0)
    assert np.max(np.abs(out.w)) <= 1e-12
    assert np.max(np.abs(out.pi - x.pi)) <= 1e-12 * np.max(np.abs(x.pi))
    assert np.max(np.abs(out.b - x.b)) <= 1e-14


@pytest.mark.parametrize("mx,m,tau", [(1, 1, 2.0), (4, 3, 2.5), (7, 6, 1.0)])
def test_three_dimensional_mode_closed_form(mx, m, tau):
    # One x-mode (theta) times one vertical mode (kappa) on uniform levels:
    # u, pi ~ cos(kappa z) at cell levels, w, b ~ sin(kappa z) on faces.  With
    # s = 2 sin(theta/2)/dx and k_d = (2/dz) sin(kappa dz/2) the differences
    # act on the amplitudes as  dpi/dx -> i s P, du/dx -> i s U,
    # dpi/dz -> -k_d P, dw/dz -> k_d W, d(D)/dz -> -k_d D, d(dw/dz)/dz -> -k_d^2 W,
    # so a stage of length h from base (U0, W0, B0, P0) with previous P_prev is
    #   U = U0 - h i s P_prev,  D = i s U,
    #   Wm (1 + h^2 N^2/4 + h^2 c^2 k_d^2/4) = W0 + (h/2)(k_d P0 + B0) - (h^2 c^2/4) k_d D,
    #   W = 2 Wm - W0,  B = B0 - h N^2 Wm,  P = P0 - h c^2 (D + k_d Wm).
    nx, ny, nz, dx, dzv = 16, 2, 10, 2000.0, 300.0
    theta = 2.0 * np.pi * mx / nx
    kappa = m * np.pi / (nz * dzv)
    s = 2.0 * np.sin(theta / 2.0) / dx
    kd = (2.0 / dzv) * np.sin(kappa * dzv / 2.0)

    def stage(x0, p_prev, h):
        u0, w0, b0, p0 = x0
        u = u0 - h * 1j * s * p_prev
        d = 1j * s * u
        wm = (w0 + (h / 2.0) * (kd * p0 + b0) - (h * h * C * C / 4.0) * kd * d) / (
            1.0 + h * h * N * N / 4.0 + h * h * C * C * kd * kd / 4.0)
        return (u, 2.0 * wm - w0, b0 - h * N * N * wm, p0 - h * C * C * (d + kd * wm))

    amp = (0.4 + 0.2j, 0.05 - 0.01j, 0.002 + 0.001j, 30.0 - 12.0j)
    nsteps = 5
    cur = amp
    for _ in range(nsteps):
        s1 = stage(cur, cur[3], tau / 2.0)
        cur = stage(cur, s1[3], tau)

    i = np.arange(nx)
    zc = (np.arange(nz) + 0.5) * dzv
    zf = np.arange(nz + 1) * dzv

    def fields(a):
        u, w, b, p = a
        cx_f = np.exp(1j * theta * (i + 0.5))[None, None, :]
        cx_c = np.exp(1j * theta * i)[None, None, :]
        shape = (1, ny, 1)
        uu = np.real(u * np.cos(kappa * zc)[:, None, None] * cx_f) * np.ones(shape)
        pp = np.real(p * np.cos(kappa * zc)[:, None, None] * cx_c) * np.ones(shape)
        ww = np.real(w * np.sin(kappa * zf)[:, None, None] * cx_c) * np.ones(shape)
        bb = np.real(b * np.sin(kappa * zf)[:, None, None] * cx_c) * np.ones(shape)
        return hevi.Fast(uu, np.zeros_like(uu), ww, bb, pp)

    got = hevi.run(fields(amp), nsteps, dx, dx, np.full(nz, dzv), tau)
    want = fields(cur)
    for name in ("u", "w", "b", "pi"):
        a, r = getattr(got, name), getattr(want, name)
        assert np.max(np.abs(a - r)) <= 1e-11 * np.max(np.abs(r)), name
