"""Pins of the oracle's gather and RK4 pusher: closed forms and invariants.

- flat space, uniform B: the discrete solution is u0 * R(z)^N with R the RK4
  stability polynomial (exact for the scheme, not just to truncation order);
- flat space, E x B: guiding-centre drift c E x B / B^2;
- Schwarzschild circular orbit (textbook Omega and u^t): E and L conserved and
  the radius held;
- Kerr inclined bound orbit: E, L_z and Carter's constant conserved;
- convergence order in coordinate time for both gamma readings;
- trilinear gather: partition of unity and exactness on linear fields.
"""
import numpy as np
import pytest

import oracle as O


def _uniform_nodes(p, F):
    nn = (p.nz + 1) * (p.ny + 1) * (p.nx + 1)
    return np.broadcast_to(np.asarray(F, dtype=float).reshape(1, 16), (nn, 16)).copy()


def _rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


@pytest.mark.parametrize("qm", [-1.0, 0.05])
@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_gyration_matches_rk4_stability_polynomial(qm, gamma_mode):
    N = 32
    B = 0.05 if qm == -1.0 else 1.0
    p = O.make_params(N, m=0.0, a=0.0, dt=0.5, gamma_mode=gamma_mode, species=((qm, 1.0),))
    s = O.Sim(p, 1)
    F = np.zeros((4, 4))
    F[0, 1] = B   # F^1_2 = F^{12} = B^z in flat space
    F[1, 0] = -B
    s.set_nodes(_uniform_nodes(p, F))
    u3 = np.array([0.3, 0.1, 0.0])
    u4 = np.sqrt(1.0 + u3 @ u3)
    x = np.array([[16.2], [15.7], [16.1]])
    u = np.array([[u3[0]], [u3[1]], [u3[2]], [u4]])
    s.set_particles(x, u, np.zeros(1, np.uint8))
    nsteps = 1000
    s.push_only(nsteps)
    _, uN, _ = s.particles()
    lam = -1j * qm * B / u4
    w_ref = (u3[0] + 1j * u3[1]) * _rk4_poly(lam * p.dt) ** nsteps
    w = uN[0, 0] + 1j * uN[1, 0]
    assert abs(w - w_ref) < 1e-13 * nsteps * abs(w_ref)
    assert abs(uN[3, 0] - u4) < 1e-15 * 10


@pytest.mark.parametrize("qm", [1.0, -1.0])
def test_exb_drift(qm):
    N = 48
    B, E = 0.5, 0.05
    p = O.make_params(N, m=0.0, a=0.0, dt=0.05, species=((qm, 1.0),))
    s = O.Sim(p, 1)
    F = np.zeros((4, 4))
    F[0, 1], F[1, 0] = B, -B
    F[1, 3] = E  # F^2_4 = -F^{24} = E^y
    F[3, 1] = E  # F^4_2 = F^{42} = E^y
    s.set_nodes(_uniform_nodes(p, F))
    x0 = np.array([[10.0], [24.0], [24.0]])
    u0 = np.array([[0.0], [0.0], [0.0], [1.0]])
    s.set_particles(x0, u0, np.zeros(1, np.uint8))
    # Whole gyro-periods.  In the drift frame B' = B / gamma_d and the particle
    # (at rest in the lab) moves with gamma' = gamma_d, so its period there is
    # 2 pi gamma_d^2 / (|q/m| B); one period in the lab lasts gamma_d times that.
    gamma_d = 1 / np.sqrt(1 - (E / B) ** 2)
    T = 5 * 2 * np.pi * gamma_d ** 3 / (abs(qm) * B)
    nsteps = int(round(T / p.dt))
    s.push_only(nsteps)
    xN, _, _ = s.particles()
    t = nsteps * p.dt
    vx = (xN[0, 0] - x0[0, 0]) / t
    vy = (xN[1, 0] - x0[1, 0]) / t
    assert abs(vx - E / B) < 2e-3 * (E / B)
    assert abs(vy) < 2e-2 * (E / B)


def _covariant(p, X, u):
    g, _, _ = O.metric(p, X[0] - p.center[0], X[1] - p.center[1], X[2] - p.center[2])
    return g @ u


def test_schwarzschild_circular_orbit_conserves_E_L():
    m, N = 1.5, 64
    p = O.make_params(N, m=m, a=0.0, dt=0.5, species=((0.0, 1.0),))
    r0 = 15 * m
    ut = 1.0 / np.sqrt(1.0 - 3.0 * m / r0)
    Om = np.sqrt(m / r0 ** 3)
    cen = np.array(p.center[:])
    X0 = cen + np.array([r0, 0.0, 0.0])
    u0 = np.array([0.0, r0 * Om * ut, 0.0, ut])
    s = O.Sim(p, 1)
    s.set_particles(X0.reshape(3, 1), u0.reshape(4, 1), np.zeros(1, np.uint8))
    ul0 = _covariant(p, X0, u0)
    E0 = -ul0[3]
    L0 = (X0[0] - cen[0]) * ul0[1] - (X0[1] - cen[1]) * ul0[0]
    for _ in range(10):
        s.push_only(1000, use_nodes=False)
        x, u, _ = s.particles()
        X = x[:, 0]
        ul = _covariant(p, X, u[:, 0])
        E = -ul[3]
        L = (X[0] - cen[0]) * ul[1] - (X[1] - cen[1]) * ul[0]
        assert abs(E - E0) < 1e-10 * abs(E0)
        assert abs(L - L0) < 1e-10 * abs(L0)
        r = np.linalg.norm(X - cen)
        assert abs(r - r0) < 1e-6 * r0


def _carter(p, X, u):
    cen = np.array(p.center[:])
    x, y, z = X - cen
    g, _, r = O.metric(p, x, y, z)
    ul = g @ u
    a = p.a
    E = -ul[3]
    Lz = x * ul[1] - y * ul[0]
    cth = z / r
    sth = np.sqrt(1.0 - cth * cth)
    pth = (cth / sth) * (x * ul[0] + y * ul[1]) - r * sth * ul[2]
    Q = pth ** 2 + cth ** 2 * (a * a * (1.0 - E * E) + Lz * Lz / (sth * sth))
    return E, Lz, Q, r


@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_kerr_inclined_orbit_conserves_E_Lz_Q(gamma_mode):
    m, N = 1.5, 128
    p = O.make_params(N, m=m, a=0.95 * m, dt=0.5, gamma_mode=gamma_mode, species=((0.0, 1.0),))
    cen = np.array(p.center[:])
    # bound orbit, inclined ~18 degrees, r between about 12.6 m and 32 m
    X0 = cen + np.array([35.0, 0.0, 5.0])
    u0 = O.mass_shell(p, X0, np.array([0.0, 4.4, 1.4]) * 0.045)
    s = O.Sim(p, 1)
    s.set_particles(X0.reshape(3, 1), u0.reshape(4, 1), np.zeros(1, np.uint8))
    E0, L0, Q0, _ = _carter(p, X0, u0)
    for _ in range(10):
        s.push_only(1000, use_nodes=False)
        x, u, _ = s.particles()
        E, L, Q, r = _carter(p, x[:, 0], u[:, 0])
        assert 10 * m < r < 60 * m
        assert abs(E - E0) < 1e-10 * abs(E0)
        assert abs(L - L0) < 1e-10 * abs(L0)
        assert abs(Q - Q0) < 1e-10 * abs(Q0)


def _infall_position(gamma_mode, dt, T):
    m = 1.5
    p = O.make_params(64, m=m, a=0.6 * m, dt=dt, gamma_mode=gamma_mode, species=((0.0, 1.0),))
    cen = np.array(p.center[:])
    X0 = cen + np.array([14.0, 3.0, 2.0])
    u0 = O.mass_shell(p, X0, np.array([-0.2, 0.12, 0.0]))
    s = O.Sim(p, 1)
    s.set_particles(X0.reshape(3, 1), u0.reshape(4, 1), np.zeros(1, np.uint8))
    s.push_only(int(round(T / dt)), use_nodes=False)
    x, u, _ = s.particles()
    return np.concatenate([x[:, 0], u[:, 0]])


@pytest.mark.parametrize("gamma_mode,expected", [(1, 16.0), (0, 2.0)])
def test_convergence_order_in_coordinate_time(gamma_mode, expected):
    T = 20.0
    dts = [0.4, 0.2, 0.1, 0.05]
    ys = [_infall_position(gamma_mode, dt, T) for dt in dts]
    e1 = np.abs(ys[0] - ys[1]).max()
    e2 = np.abs(ys[1] - ys[2]).max()
    e3 = np.abs(ys[2] - ys[3]).max()
    ratio = e2 / e3
    assert abs(np.log2(ratio) - np.log2(expected)) < 0.35, (e1, e2, e3)


def test_gather_partition_of_unity_and_linear_exactness():
    N = 8
    p = O.make_params(N, m=0.0)
    s = O.Sim(p, 0)
    kk, jj, ii = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    rng = np.random.default_rng(9)
    c0 = rng.normal(size=16)
    cx, cy, cz = rng.normal(size=(3, 16))
    F = c0 + cx * ii[..., None] + cy * jj[..., None] + cz * kk[..., None]
    s.set_nodes(F)
    import ctypes
    nodes = np.ascontiguousarray(F.reshape(-1))
    for _ in range(200):
        X = rng.uniform(0.0, N - 1e-9, 3)
        out = np.zeros(16)
        O.lib().or_gather(ctypes.byref(p), O._dp(nodes), O._dp(np.ascontiguousarray(X)), O._dp(out))
        ref = c0 + cx * X[0] + cy * X[1] + cz * X[2]
        assert np.abs(out - ref).max() < 1e-12
