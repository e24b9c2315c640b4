"""Pins of the oracle's metric module against closed forms and textbook Kerr.

Nothing here retypes the paper's metric formula: each check is a property
the Kerr metric has whatever the formula's implementation (null one-form,
unit determinant, Boyer-Lindquist Killing components, horizon condition,
Schwarzschild in ingoing Eddington-Finkelstein Cartesian form, numerical
derivatives of the oracle's own metric).
"""
import numpy as np
import pytest

import oracle as O

ETA = np.diag([1.0, 1.0, 1.0, -1.0])


def _points(rng, n, lo=1.0, hi=12.0):
    out = []
    while len(out) < n:
        v = rng.uniform(-hi, hi, 3)
        if lo < np.linalg.norm(v) < hi:
            out.append(v)
    return out


def test_radius_quartic_residual_and_special_cases():
    rng = np.random.default_rng(1)
    for _ in range(3000):
        a = rng.uniform(0.0, 3.0)
        x, y, z = rng.uniform(-10.0, 10.0, 3)
        r = O.radius(a, x, y, z)
        R2 = x * x + y * y + z * z
        res = r ** 4 - (R2 - a * a) * r ** 2 - a * a * z * z
        assert abs(res) <= 8 * np.finfo(float).eps * max(R2, a * a) ** 2
        assert r >= 0.0
    # a = 0: r = R
    for x, y, z in rng.uniform(-5, 5, (50, 3)):
        assert abs(O.radius(0.0, x, y, z) - np.sqrt(x * x + y * y + z * z)) < 1e-14 * 10
    # z = 0: r^2 = max(R^2 - a^2, 0)
    for x, y in rng.uniform(-5, 5, (50, 2)):
        a = 2.0
        r = O.radius(a, x, y, 0.0)
        assert abs(r * r - max(x * x + y * y - a * a, 0.0)) < 1e-13
    # on the axis: r = |z|
    for z in rng.uniform(-5, 5, 50):
        assert abs(O.radius(1.7, 0.0, 0.0, z) - abs(z)) < 1e-14 * 10


@pytest.mark.parametrize("a_frac", [0.0, 0.5, 0.95, 0.99])
def test_metric_identities(a_frac):
    m = 1.5
    p = O.make_params(32, m=m, a=a_frac * m)
    rng = np.random.default_rng(2)
    for x, y, z in _points(rng, 200):
        g, gi, r = O.metric(p, x, y, z)
        if r < 0.3:
            continue
        # g - eta is rank one, f k k with k_4 = 1, and k is null for eta
        h = g - ETA
        f = h[3, 3]
        k = h[:, 3] / f
        assert abs(k[3] - 1.0) < 1e-14
        assert np.abs(h - f * np.outer(k, k)).max() < 1e-13 * max(1.0, f)
        assert abs(k @ np.linalg.inv(ETA) @ k) < 1e-13
        # unit determinant and inverse
        assert abs(np.linalg.det(g) + 1.0) < 1e-12 * max(1.0, f * f)
        assert np.abs(g @ gi - np.eye(4)).max() < 1e-13 * max(1.0, f)


def test_schwarzschild_is_textbook_kerr_schild():
    m = 1.5
    p = O.make_params(32, m=m, a=0.0)
    rng = np.random.default_rng(3)
    for x, y, z in _points(rng, 100):
        g, _, _ = O.metric(p, x, y, z)
        R = np.sqrt(x * x + y * y + z * z)
        n = np.array([x / R, y / R, z / R, 1.0])
        ref = ETA + (2 * m / R) * np.outer(n, n)
        assert np.abs(g - ref).max() < 1e-14 * 10


@pytest.mark.parametrize("a_frac", [0.3, 0.95])
def test_boyer_lindquist_killing_components(a_frac):
    """g(d_t,d_t), g(d_t,d_phi), g(d_phi,d_phi) are coordinate invariants of the
    two Killing fields; compare with textbook Boyer-Lindquist Kerr (G = c = 1).
    The paper's one-form carries a(x dy - y dx), which gives g_tphi > 0 for a > 0:
    spin along -z in the usual convention (the sign is pinned as literal)."""
    m = 1.5
    a = a_frac * m
    p = O.make_params(32, m=m, a=a)
    rng = np.random.default_rng(4)
    for x, y, z in _points(rng, 200, lo=2.0):
        g, _, r = O.metric(p, x, y, z)
        cos2 = (z / r) ** 2
        sin2 = 1.0 - cos2
        Sig = r * r + a * a * cos2
        psi = np.array([-y, x, 0.0, 0.0])
        xi = np.array([0.0, 0.0, 0.0, 1.0])
        gtt = xi @ g @ xi
        gtp = xi @ g @ psi
        gpp = psi @ g @ psi
        assert abs(gtt - (-(1.0 - 2 * m * r / Sig))) < 1e-12
        assert abs(gtp - 2 * m * a * r * sin2 / Sig) < 1e-12 * max(1.0, r)
        ref_pp = sin2 * (r * r + a * a + 2 * m * a * a * r * sin2 / Sig)
        assert abs(gpp - ref_pp) < 1e-12 * max(1.0, r * r)


@pytest.mark.parametrize("a_frac", [0.0, 0.6, 0.99])
def test_horizon_condition(a_frac):
    """g^{mn} d_m r d_n r = Delta/Sigma (a scalar, so equal to its BL value)."""
    m = 1.5
    a = a_frac * m
    p = O.make_params(32, m=m, a=a)
    rng = np.random.default_rng(5)
    h = 1e-5
    for x, y, z in _points(rng, 100, lo=1.5):
        _, gi, r = O.metric(p, x, y, z)
        dr = np.zeros(4)
        X = np.array([x, y, z])
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            dr[i] = (O.radius(a, *(X + e)) - O.radius(a, *(X - e))) / (2 * h)
        lhs = dr @ gi @ dr
        Sig = r * r + a * a * (z / r) ** 2
        Delta = r * r - 2 * m * r + a * a
        assert abs(lhs - Delta / Sig) < 1e-8 * max(1.0, abs(Delta / Sig))


@pytest.mark.parametrize("a_frac", [0.0, 0.95])
def test_metric_derivative_matches_numerical_derivative(a_frac):
    m = 1.5
    p = O.make_params(32, m=m, a=a_frac * m)
    rng = np.random.default_rng(6)

    def D(X, i, h):
        e = np.zeros(3)
        e[i] = h
        return (O.metric(p, *(X + e))[0] - O.metric(p, *(X - e))[0]) / (2 * h)

    for pt in _points(rng, 40, lo=3.0):
        dg = O.metric_deriv(p, *pt)
        for i in range(3):
            h = 4e-3
            rich = (4 * D(pt, i, h / 2) - D(pt, i, h)) / 3.0
            assert np.abs(dg[i] - rich).max() < 1e-8, (pt, i)


@pytest.mark.parametrize("a_frac", [0.0, 0.5, 0.99])
def test_christoffel_symmetry_and_contraction(a_frac):
    """Gamma^a_{bc} = Gamma^a_{cb}; Gamma^b_{bc} = d_c ln sqrt(-g) = 0 since det g = -1."""
    m = 1.5
    p = O.make_params(32, m=m, a=a_frac * m)
    rng = np.random.default_rng(7)
    for pt in _points(rng, 100, lo=1.5):
        G = O.christoffel(p, *pt)
        scale = max(1.0, np.abs(G).max())
        assert np.abs(G - G.transpose(0, 2, 1)).max() < 1e-15 * 10 * scale
        assert np.abs(np.einsum("bbc->c", G)).max() < 1e-14 * scale


def test_mass_shell_root():
    m = 3.0
    p = O.make_params(64, m=m, a=0.95 * m)
    rng = np.random.default_rng(8)
    cen = np.array(p.center[:])
    for pt in _points(rng, 200, lo=4.5, hi=25.0):
        ucov = rng.normal(0.0, 0.3, 3)
        X = cen + pt
        u = O.mass_shell(p, X, ucov)
        g, gi, _ = O.metric(p, *pt)
        assert abs(u @ g @ u + 1.0) < 1e-13 * max(1.0, u[3] ** 2)
        assert u[3] > 0.0
        ul = g @ u
        assert np.abs(ul[:3] - ucov).max() < 1e-13 * max(1.0, u[3])
