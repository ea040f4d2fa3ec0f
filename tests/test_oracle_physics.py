"""Pins of the oracle column physics against closed forms and LAPACK (CPU only)."""
import numpy as np
import pytest

from oracle import physics
from oracle.mass import mass_sums
from oracle.params import DEFAULT, Params


def _random_spd_tridiag(rng, n, ncol, rmax):
    """Diagonally dominant tridiagonal columns shaped like the diffusion matrix."""
    m = rng.uniform(0.5, 2.0, size=(n, ncol))
    alpha = np.zeros((n + 1, ncol))
    scale = np.exp(rng.uniform(np.log(1e-3), np.log(rmax), size=(1, ncol)))
    alpha[1:n] = rng.uniform(0.1, 1.0, size=(n - 1, ncol)) * scale * m.mean(axis=0)
    beta = rng.uniform(0.0, 1.0, size=ncol)
    return m, alpha, beta


@pytest.mark.parametrize("n", [3, 4, 5, 8, 16, 58])
def test_thomas_matches_dense_lapack(n):
    # P6: Thomas against numpy.linalg.solve (LAPACK gesv, partial pivoting) on
    # 1000 random diagonally dominant tridiagonals, dominance ratio up to 1e4.
    rng = np.random.default_rng(100 + n)
    ncol = 1000
    m, alpha, beta = _random_spd_tridiag(rng, n, ncol, 1e4)
    sub = -alpha[:-1]
    sup = -alpha[1:]
    diag = m + alpha[:-1] + alpha[1:]
    diag[0] += beta
    rhs = rng.normal(size=(n, ncol))
    x = physics.thomas(sub, diag, sup, rhs)
    worst = 0.0
    for c in range(ncol):
        a = np.diag(diag[:, c]) + np.diag(sub[1:, c], -1) + np.diag(sup[:-1, c], 1)
        ref = np.linalg.solve(a, rhs[:, c])
        worst = max(worst, np.max(np.abs(x[:, c] - ref)) / np.max(np.abs(ref)))
    assert worst <= 1e-12, worst


def _column_inputs(nz, dzv, rho0, u_profile, ch0=0.0):
    shape = (nz, 1, 1)
    dz = np.full(nz, dzv)
    rho = np.full(shape, rho0)
    u = np.broadcast_to(u_profile[:, None, None], shape).copy()
    v = np.zeros(shape)
    ch = np.full((1, 1), ch0)
    return dz, rho, u, v, ch


@pytest.mark.parametrize("mode", [1, 2, 5, 11])
def test_vertical_cosine_mode_decay_with_linear_shear(mode):
    # P7: uniform dz, rho and shear a (so K = K_min + l^2 a), no surface
    # exchange.  The backward-Euler step multiplies the Neumann eigenvector
    # cos(pi m (k+1/2)/nz) by 1 / (1 + 4 (dt K/dz^2) sin^2(pi m/(2 nz))).
    nz, dzv, rho0, dt, a = 24, 80.0, 1.1, 6.0, 0.004
    z = (np.arange(nz) + 0.5) * dzv
    dz, rho, u, v, ch = _column_inputs(nz, dzv, rho0, a * z)
    cf = physics.diffusion_coeffs(rho, u, v, ch, dz, dt)
    kz = DEFAULT.k_min + DEFAULT.mix_len ** 2 * a
    phi = np.cos(np.pi * mode * (np.arange(nz) + 0.5) / nz)[:, None, None]
    delta = physics.implicit_diffusion(phi, np.zeros((1, 1)), cf)
    factor = 1.0 / (1.0 + 4.0 * dt * kz / dzv ** 2 * np.sin(np.pi * mode / (2 * nz)) ** 2)
    np.testing.assert_allclose((phi + delta)[:, 0, 0], factor * phi[:, 0, 0], rtol=0, atol=1e-13)
    # the dominance ratio of this column is 2 dt K / dz^2 (interior levels)
    r = physics.dominance_ratio(cf)
    np.testing.assert_allclose(r[0, 0], 2.0 * dt * kz / dzv ** 2, rtol=1e-14)


def test_diffusion_matches_dense_backward_euler():
    # The delta-form system is the backward-Euler step of
    # m d(phi)/dt = flux divergence with a Robin ground: (M + A) phi_new = M phi + beta phi_s e0,
    # where A is the weighted graph Laplacian of the column with edge weights
    # alpha.  Solve that full-state form densely and compare.
    rng = np.random.default_rng(3)
    nz = 7
    dz = rng.uniform(40.0, 400.0, nz)
    rho = rng.uniform(0.5, 1.3, (nz, 1, 1))
    u = rng.normal(0, 8, (nz, 1, 1))
    v = rng.normal(0, 8, (nz, 1, 1))
    ch = np.full((1, 1), 0.013)
    dt = 7.0
    cf = physics.diffusion_coeffs(rho, u, v, ch, dz, dt)
    phi = rng.normal(300, 2, (nz, 1, 1))
    phi_s = np.full((1, 1), 303.0)
    delta = physics.implicit_diffusion(phi, phi_s, cf)
    al = cf.alpha[:, 0, 0]
    lap = np.zeros((nz, nz))
    for e in range(1, nz):                   # edge between levels e-1 and e
        lap[e - 1, e - 1] += al[e]
        lap[e, e] += al[e]
        lap[e - 1, e] -= al[e]
        lap[e, e - 1] -= al[e]
    mm = np.diag(cf.m[:, 0, 0])
    lhs = mm + lap
    lhs[0, 0] += cf.beta[0, 0]
    rhs = mm @ phi[:, 0, 0]
    rhs[0] += cf.beta[0, 0] * phi_s[0, 0]
    ref = np.linalg.solve(lhs, rhs)
    np.testing.assert_allclose((phi + delta)[:, 0, 0], ref, rtol=1e-13)


def test_surface_flux_budget():
    # P9: sum_k m_k delta_k = beta (phi_s - phi_0 - delta_0).
    rng = np.random.default_rng(4)
    nz = 30
    dz = np.geomspace(50.0, 1000.0, nz)
    rho = rng.uniform(0.3, 1.3, (nz, 4, 5))
    u = rng.normal(0, 10, (nz, 4, 5))
    v = rng.normal(0, 10, (nz, 4, 5))
    ch = rng.uniform(0.005, 0.02, (4, 5))
    cf = physics.diffusion_coeffs(rho, u, v, ch, dz, 6.5)
    phi = rng.normal(0.0, 1.0, (nz, 4, 5))
    phi_s = rng.normal(0.0, 1.0, (4, 5))
    d = physics.implicit_diffusion(phi, phi_s, cf)
    lhs = np.sum(cf.m * d, axis=0)
    rhs = cf.beta * (phi_s - phi[0] - d[0])
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-13 * np.max(np.abs(cf.m)))


def test_radiation_zero_absorber_gives_zero_heating():
    nz = 12
    rho = np.full((nz, 2, 3), 1.0)
    q = np.zeros((nz, 2, 3))
    q[3, 1, 1] = -0.01                        # negative q does not absorb either
    h, t = physics.radiation(rho, q, np.full((2, 3), 700.0), np.full(nz, 100.0))
    assert np.all(h == 0.0)
    assert np.all(t == 1.0)


def test_radiation_uniform_optical_depth_closed_form():
    # P8: uniform dtau gives T_{k+1/2} = exp(-(nz-1-k) dtau) and the column
    # heating integrates to the absorbed flux: sum c_p m_k H_k = F0 (1 - T_{-1/2}).
    nz, rho0, q0, dzv, f0 = 20, 0.9, 0.005, 120.0, 640.0
    p = Params()
    rho = np.full((nz, 1, 1), rho0)
    q = np.full((nz, 1, 1), q0)
    h, t = physics.radiation(rho, q, np.full((1, 1), f0), np.full(nz, dzv), p)
    dtau = p.kappa_q * rho0 * q0 * dzv
    k = np.arange(nz)
    np.testing.assert_allclose(t[1:, 0, 0], np.exp(-(nz - 1 - k) * dtau), rtol=1e-14)
    np.testing.assert_allclose(t[0, 0, 0], np.exp(-nz * dtau), rtol=1e-14)
    absorbed = np.sum(p.cp * rho0 * dzv * h[:, 0, 0])
    np.testing.assert_allclose(absorbed, f0 * (1.0 - np.exp(-nz * dtau)), rtol=1e-13)
    assert np.all(h > 0.0)


def test_radiation_energy_closure_random_column():
    rng = np.random.default_rng(8)
    nz = 58
    dz = np.geomspace(50.0, 1000.0, nz)
    rho = rng.uniform(0.2, 1.3, (nz, 3, 2))
    q = rng.uniform(-0.001, 0.02, (nz, 3, 2))
    f0 = rng.uniform(400, 800, (3, 2))
    h, t = physics.radiation(rho, q, f0, dz)
    absorbed = np.sum(DEFAULT.cp * rho * dz[:, None, None] * h, axis=0)
    np.testing.assert_allclose(absorbed, f0 * (1.0 - t[0]), rtol=1e-12)


def test_physics_conserves_column_mass_without_sources():
    # With C_h = 0 and F0 = 0 the physics conserves sum m_k phi_k per column.
    rng = np.random.default_rng(11)
    nz = 16
    dz = np.geomspace(50.0, 1000.0, nz)
    rho = rng.uniform(0.3, 1.3, (nz, 3, 4))
    th = rng.normal(300, 3, (nz, 3, 4))
    q = rng.uniform(0.0, 0.02, (nz, 3, 4))
    u = rng.normal(0, 10, (nz, 3, 4))
    v = rng.normal(0, 10, (nz, 3, 4))
    z2 = np.zeros((3, 4))
    out = physics.column_physics(rho, th, q, u, v, z2 + 301, z2 + 0.01, z2, z2, dz, 7.0)
    m0 = mass_sums(rho, th, q, 1.0, 1.0, dz)
    m1 = mass_sums(rho, out.theta, out.q, 1.0, 1.0, dz)
    np.testing.assert_allclose(m1, m0, rtol=1e-14)


def test_tendencies_consistent_with_update():
    rng = np.random.default_rng(12)
    nz = 10
    dz = np.geomspace(50.0, 1000.0, nz)
    sh = (nz, 2, 2)
    rho, th, q = rng.uniform(0.5, 1.2, sh), rng.normal(300, 2, sh), rng.uniform(0, 0.02, sh)
    u, v = rng.normal(0, 10, sh), rng.normal(0, 10, sh)
    z2 = np.zeros((2, 2))
    dt = 5.0
    out = physics.column_physics(rho, th, q, u, v, z2 + 302, z2 + 0.015, z2 + 650, z2 + 0.01, dz, dt)
    np.testing.assert_allclose(th + dt * out.t_theta, out.theta, rtol=1e-14)
    np.testing.assert_allclose(q + dt * out.t_q, out.q, rtol=1e-12, atol=1e-17)


def test_mass_sums_closed_form():
    nx, ny, nz = 7, 5, 9
    dz = np.geomspace(50.0, 1000.0, nz)
    rho = np.full((nz, ny, nx), 1.25)
    th = np.full((nz, ny, nx), 300.0)
    q = np.full((nz, ny, nx), 0.01)
    m = mass_sums(rho, th, q, 2000.0, 2000.0, dz)
    mr = 1.25 * 2000.0 * 2000.0 * nx * ny * np.sum(dz)
    np.testing.assert_allclose(m, [mr, 300.0 * mr, 0.01 * mr], rtol=1e-15)


@pytest.mark.parametrize("i0,j0", [(0, 0), (3, 2), (4, 3)])
def test_centred_winds_single_face_perturbation(i0, j0):
    # C-grid staggering: u[..., i] sits on the east face of cell i, so it is
    # the east wind of cell i and the west wind of cell i+1 (periodic).  A
    # perturbation of one east face must move the centred wind of exactly
    # those two cells, by half the perturbation; the same for v in j.  A roll
    # in the wrong direction moves cells i and i-1 instead and fails here.
    nz, ny, nx = 3, 4, 5
    rng = np.random.default_rng(7 + i0 + 10 * j0)
    u = rng.normal(0.0, 5.0, (nz, ny, nx))
    v = rng.normal(0.0, 5.0, (nz, ny, nx))
    ub0, vb0 = physics.centred_winds(u, v)
    du = np.zeros_like(u)
    du[1, j0, i0] = 2.0
    ub1, vb1 = physics.centred_winds(u + du, v)
    want = np.zeros_like(u)
    want[1, j0, i0] = 1.0
    want[1, j0, (i0 + 1) % nx] = 1.0
    np.testing.assert_allclose(ub1 - ub0, want, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(vb1, vb0)
    dv = np.zeros_like(v)
    dv[2, j0, i0] = -4.0
    ub2, vb2 = physics.centred_winds(u, v + dv)
    want = np.zeros_like(v)
    want[2, j0, i0] = -2.0
    want[2, (j0 + 1) % ny, i0] = -2.0
    np.testing.assert_allclose(vb2 - vb0, want, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(ub2, ub0)


def test_diffusion_coeffs_on_a_stretched_three_level_column():
    # Hand-worked column with unequal thicknesses and densities, so the
    # interface spacing (dz_k + dz_{k+1})/2 and the face density
    # (rho_k + rho_{k+1})/2 differ from either neighbour's own value.
    #   dz = 10, 30, 70 m;  rho = 1.2, 0.9, 0.5 kg/m^3;  dt = 4 s; C_h = 0.01
    #   centred winds (u, v) = (0, 0), (3, 4), (5, 4) m/s (a 1 x 1 grid, so
    #   the face mean of a horizontally uniform wind is the wind itself)
    # Interface 1/2: dz = 20, |dU| = 5 -> shear 0.25, K = 0.1 + 2500 * 0.25 = 625.1,
    #   rho_f = 1.05 -> alpha = 4 * 1.05 * 625.1 / 20 = 131.271
    # Interface 3/2: dz = 50, |dU| = 2 -> shear 0.04, K = 0.1 + 100 = 100.1,
    #   rho_f = 0.7 -> alpha = 4 * 0.7 * 100.1 / 50 = 5.6056
    # Layer masses 12, 27, 35; beta = 4 * 1.2 * 0.01 = 0.048.
    dz = np.array([10.0, 30.0, 70.0])
    rho = np.array([1.2, 0.9, 0.5]).reshape(3, 1, 1)
    u = np.array([0.0, 3.0, 5.0]).reshape(3, 1, 1)
    v = np.array([0.0, 4.0, 4.0]).reshape(3, 1, 1)
    ch = np.full((1, 1), 0.01)
    cf = physics.diffusion_coeffs(rho, u, v, ch, dz, 4.0)
    np.testing.assert_allclose(cf.alpha[:, 0, 0], [0.0, 131.271, 5.6056, 0.0], rtol=1e-14, atol=0)
    np.testing.assert_allclose(cf.m[:, 0, 0], [12.0, 27.0, 35.0], rtol=1e-15)
    np.testing.assert_allclose(cf.beta[0, 0], 0.048, rtol=1e-15)
    # dominance ratios: (0 + 131.271)/12, (131.271 + 5.6056)/27, 5.6056/35
    np.testing.assert_allclose(physics.dominance_ratio(cf)[0, 0], 131.271 / 12.0, rtol=1e-14)
