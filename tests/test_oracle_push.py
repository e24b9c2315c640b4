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


@pytest.mark.parametrize("qm,c,dt", [(-1.0, 1.0, 0.5), (0.05, 1.0, 0.5), (-1e-3, 0.05, 1.0)])
@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_gyration_matches_rk4_stability_polynomial(qm, c, dt, gamma_mode):
    # in coordinate time dw/dt = -i (q/m) B (c / u^4) w (u^4 = dx^4/dtau = c dt/dtau)
    N = 32
    B = {-1.0: 0.05, 0.05: 1.0, -1e-3: 30.0}[qm]
    p = O.make_params(N, m=0.0, a=0.0, c=c, dt=dt, gamma_mode=gamma_mode, species=((qm, 1.0),))
    s = O.Sim(p, 1)
    F = np.zeros((4, 4))
    F[0, 1] = B   # F^1_2 = F^{12} = B^z in flat space
    F[1, 0] = -B
    s.set_nodes(_uniform_nodes(p, F))
    u3 = np.array([0.3, 0.1, 0.0]) * c
    u4 = np.sqrt(c * c + u3 @ u3)
    x = np.array([[16.2], [15.7], [16.1]])
    u = np.array([[u3[0]], [u3[1]], [u3[2]], [u4]])
    s.set_particles(x, u, np.zeros(1, np.uint8))
    nsteps = 1000
    s.push_only(nsteps)
    _, uN, _ = s.particles()
    lam = -1j * qm * B * c / u4
    w_ref = (u3[0] + 1j * u3[1]) * _rk4_poly(lam * p.dt) ** nsteps
    w = uN[0, 0] + 1j * uN[1, 0]
    assert abs(w - w_ref) < 1e-13 * nsteps * abs(w_ref)
    assert abs(uN[3, 0] - u4) < 1e-14 * u4


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


# --- ablations of the push readings (rk_mode 1: the printed RK steps taken
# literally; gather_mode 1: the field tensor gathered once at x_n) ---------

def _lit_poly(z):
    # u_{n+1} = P(z) u_n for du/dtau = Omega u at constant gamma, z = Omega dt/gamma
    return 1 + 5 * z / 6 + 7 * z * z / 24 + z ** 3 / 16 + z ** 4 / 192


def _lit_xpoly(z):
    # x_{n+1} - x_n = (dt/gamma) Q(z) u_n for the same equation
    return (5 + 7 * z / 4 + 3 * z * z / 8 + z ** 3 / 32) / 6


def _gyro_setup(gamma_mode, qm, B, rk_mode=0, gather_mode=0, nodes=None):
    N = 32
    p = O.make_params(N, m=0.0, a=0.0, dt=0.5, gamma_mode=gamma_mode, species=((qm, 1.0),),
                      rk_mode=rk_mode, gather_mode=gather_mode)
    s = O.Sim(p, 1)
    if nodes is None:
        F = np.zeros((4, 4))
        F[0, 1], F[1, 0] = B, -B   # F^1_2 = F^{12} = B^z in flat space
        nodes = _uniform_nodes(p, F)
    s.set_nodes(nodes)
    return p, s


@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_literal_rk_gyration_matches_its_polynomial(gamma_mode):
    qm, B = -1.0, 0.05
    p, s = _gyro_setup(gamma_mode, qm, B, rk_mode=1)
    u3 = np.array([0.3, 0.1, 0.2])
    u4 = np.sqrt(1.0 + u3 @ u3)
    x0 = np.array([16.2, 15.7, 16.1])
    s.set_particles(x0[:, None].copy(), np.array([[u3[0]], [u3[1]], [u3[2]], [u4]]), np.zeros(1, np.uint8))
    nsteps = 200
    s.push_only(nsteps)
    xN, uN, _ = s.particles()
    # closed form: a magnetic field leaves u^4 (so gamma = u^4/c) unchanged
    h = p.dt / u4
    z = -1j * qm * B * h
    w, pos = u3[0] + 1j * u3[1], x0[0] + 1j * x0[1]
    for _ in range(nsteps):
        pos += h * _lit_xpoly(z) * w
        w *= _lit_poly(z)
    assert abs(uN[0, 0] + 1j * uN[1, 0] - w) < 1e-13 * nsteps * abs(w)
    assert abs(xN[0, 0] + 1j * xN[1, 0] - pos) < 1e-13 * nsteps * abs(pos)
    # along B the particle drifts 5/6 of v dt per step (weights summing to 5/6)
    assert abs(xN[2, 0] - (x0[2] + nsteps * (5.0 / 6.0) * u3[2] / u4 * p.dt)) < 1e-12
    assert abs(uN[3, 0] - u4) < 1e-14


def test_literal_rk_free_particle_moves_five_sixths():
    p = O.make_params(16, m=0.0, a=0.0, dt=0.5, rk_mode=1)
    s = O.Sim(p, 1)
    s.set_nodes(np.zeros(((p.nz + 1) * (p.ny + 1) * (p.nx + 1), 16)))
    u3 = np.array([0.4, -0.2, 0.1])
    u4 = np.sqrt(1.0 + u3 @ u3)
    x0 = np.array([8.0, 8.0, 8.0])
    s.set_particles(x0[:, None].copy(), np.r_[u3, u4][:, None].copy(), np.zeros(1, np.uint8))
    s.push_only(3)
    xN, uN, _ = s.particles()
    assert np.abs(xN[:, 0] - (x0 + 3 * (5.0 / 6.0) * u3 / u4 * p.dt)).max() < 1e-13
    assert np.abs(uN[:3, 0] - u3).max() == 0.0


def test_per_step_gather_is_rk4_of_the_field_frozen_at_x_n():
    # B^z linear in x, so the trilinear gather is exact: B(x) = B0 + G x
    qm, B0, G = -1.0, 0.04, 0.004
    N = 32
    nn = (N + 1) ** 3
    kk, jj, ii = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    Bn = (B0 + G * ii).reshape(-1)
    nodes = np.zeros((nn, 16))
    nodes[:, 1], nodes[:, 4] = Bn, -Bn
    u3 = np.array([0.3, 0.1, 0.0])
    u4 = np.sqrt(1.0 + u3 @ u3)
    x0 = np.array([15.2, 15.7, 16.1])
    out = {}
    for gm in (0, 1):
        p, s = _gyro_setup(1, qm, None, gather_mode=gm, nodes=nodes)
        s.set_particles(x0[:, None].copy(), np.r_[u3, u4][:, None].copy(), np.zeros(1, np.uint8))
        s.push_only(100)
        out[gm] = s.particles()
    # closed form, step by step: classic RK4 of dw/dtau = -i qm B(x_n) w
    h = p.dt / u4
    w, pos = u3[0] + 1j * u3[1], x0[0] + 1j * x0[1]
    for _ in range(100):
        z = -1j * qm * (B0 + G * pos.real) * h
        pos += h * (1 + z / 2 + z * z / 6 + z ** 3 / 24) * w
        w *= _rk4_poly(z)
    xN, uN, _ = out[1]
    assert abs(uN[0, 0] + 1j * uN[1, 0] - w) < 1e-12 * abs(w)
    assert abs(xN[0, 0] + 1j * xN[1, 0] - pos) < 1e-11 * abs(pos)
    # the per-stage gather sees B change within the step: a different orbit
    x0N, u0N, _ = out[0]
    assert abs(u0N[0, 0] + 1j * u0N[1, 0] - w) > 1e-9


# --- gather reading B (gather_weights 1): CIC sub-volumes weighted by the
# spatial volume density sqrt(det g_ij) by the midpoint rule ----------------

def _ks_f(m, a, x, y, z):
    # textbook Kerr-Schild f = 2 m r^3 / (r^4 + a^2 z^2), r from the quartic
    b = x * x + y * y + z * z - a * a
    r2 = 0.5 * (b + np.sqrt(b * b + 4 * a * a * z * z))
    r = np.sqrt(r2)
    return 2 * m * r * r2 / (r2 * r2 + a * a * z * z)


def test_spatial_density_is_sqrt_one_plus_f():
    # det(delta_ij + f k_i k_j) = 1 + f |k|^2 and |k|^2 = 1 for the null k
    p = O.make_params(16, m=1.5, a=1.2, r_exc=0.0)
    rng = np.random.default_rng(11)
    for _ in range(200):
        x, y, z = rng.uniform(-7, 7, 3)
        if x * x + y * y + z * z < 4.0:
            continue
        assert abs(O.spatial_density(p, x, y, z) - np.sqrt(1 + _ks_f(1.5, 1.2, x, y, z))) < 1e-14


def test_gather_reading_b_reduces_to_trilinear_at_m0():
    pa = O.make_params(16, m=0.0, gather_weights=1)
    pb = O.make_params(16, m=0.0, gather_weights=0)
    rng = np.random.default_rng(12)
    for _ in range(100):
        X = rng.uniform(0, 15.999, 3)
        c = np.floor(X)
        Wa, Wb = O.gather_weights(pa, c, X), O.gather_weights(pb, c, X)
        w = X - c
        tri = np.array([(1 - w[0] if (n & 1) == 0 else w[0]) * (1 - w[1] if (n & 2) == 0 else w[1])
                        * (1 - w[2] if (n & 4) == 0 else w[2]) for n in range(8)])
        assert np.abs(Wb - tri).max() == 0.0
        assert np.abs(Wa - tri).max() < 1e-15


def test_gather_reading_b_unity_constant_field_and_mirror_symmetry():
    N = 16
    p = O.make_params(N, m=1.5, a=1.2, gather_weights=1)
    rng = np.random.default_rng(13)
    nodes = np.broadcast_to(rng.normal(size=16), ((N + 1) ** 3, 16)).copy()
    import ctypes
    flat = np.ascontiguousarray(nodes.reshape(-1))
    for _ in range(100):
        X = rng.uniform(2, 13.999, 3)
        W = O.gather_weights(p, np.floor(X), X)
        assert abs(W.sum() - 1.0) < 1e-15
        out = np.zeros(16)
        O.lib().or_gather(ctypes.byref(p), O._dp(flat), O._dp(np.ascontiguousarray(X)), O._dp(out))
        assert np.abs(out - nodes[0]).max() < 1e-14 * np.abs(nodes[0]).max()
    # Schwarzschild: the density is symmetric under y -> 2 c_y - y, so the
    # mirrored particle's weights are the mirrored nodes' weights
    ps = O.make_params(N, m=1.5, a=0.0, gather_weights=1)
    for _ in range(50):
        X = rng.uniform(3, 12.999, 3)
        Xm = X.copy()
        Xm[1] = N - X[1]
        W, Wm = O.gather_weights(ps, np.floor(X), X), O.gather_weights(ps, np.floor(Xm), Xm)
        perm = [n ^ 2 for n in range(8)]  # dj -> 1 - dj
        assert np.abs(Wm - W[perm]).max() < 1e-14


def test_gather_reading_b_sub_volumes_match_quadrature():
    # near the hole (R 4..8 cells) the midpoint rule differs from a 5-point
    # Gauss-Legendre integral of sqrt(1 + f) over each sub-volume by its own
    # O(h^2) error (< 2e-3 of the weights); a density taken half a cell
    # away would be off by ~1e-2
    m, a, N = 1.5, 1.2, 16
    p = O.make_params(N, m=m, a=a, gather_weights=1, r_exc=0.0)
    cen = np.array([N / 2.0] * 3)
    gx, gw = np.polynomial.legendre.leggauss(5)
    rng = np.random.default_rng(14)
    worst = 0.0
    done = 0
    while done < 60:
        X = cen + rng.uniform(-8, 8, 3)
        R = np.linalg.norm(X - cen)
        if not (4.0 < R < 8.0):
            continue
        c = np.floor(X)
        W = O.gather_weights(p, c, X)
        V = np.zeros(8)
        for n in range(8):
            d = [(n >> ax) & 1 for ax in range(3)]
            lo = np.array([c[ax] if d[ax] else X[ax] for ax in range(3)])
            hi = np.array([X[ax] if d[ax] else c[ax] + 1 for ax in range(3)])
            pts = [0.5 * (lo[ax] + hi[ax]) + 0.5 * (hi[ax] - lo[ax]) * gx for ax in range(3)]
            wts = [0.5 * (hi[ax] - lo[ax]) * gw for ax in range(3)]
            PX, PY, PZ = np.meshgrid(*pts, indexing="ij")
            WW = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
            V[n] = (WW * np.sqrt(1 + _ks_f(m, a, PX - cen[0], PY - cen[1], PZ - cen[2]))).sum()
        ref = V / V.sum()
        worst = max(worst, np.abs(W - ref).max())
        done += 1
    assert worst < 2e-3, worst
