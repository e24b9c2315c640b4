"""Pins of the oracle parts that the other CPU tests reach only through
limits and sums: the curved face-area weights of the deposition (Sec. 4),
the constitutive step and its node averaging in Kerr space-time (Sec. 3),
the relaxation layer inside the horizon, and the field-energy diagnostic.

- area weights: each sub-rectangle weight of a segment equals a 5-point
  Gauss-Legendre integral of the metric area density sqrt(g_II g_JJ - g_IJ^2)
  over the sub-rectangle opposite its node, in the segment's mid-plane,
  normalised by the face, within the midpoint rule's own O(h^2) error;
- constitutive step: at points around a spinning hole, the oracle's 6x6 solve
  returns exactly what raising and lowering with the metric give,
  F^{mn} = g^{ma} g^{nb} F_{ab}, for random F;
- Wald's vacuum solution in Kerr: the field of a Killing vector is a
  stationary vacuum solution, so one cycle of the discrete field solver
  changes it only by its truncation error; when m, a and the grid are doubled
  (the same physical region with twice the resolution) the one-step change
  falls by 8 in cell units, which is second order (an O(1) error in the
  curvature part of the map would fall by 2, a first-order one by 4); over
  hundreds of cycles the far field stays bounded (the inner boundary's
  disturbances, not the map, set that level);
- relaxation: one cycle with the relaxation layer equals the same cycle
  without it followed by F <- F - sigma(r) (F - F0) at the updated points
  with r_exc <= r < r_damp, sigma = damp_max ((r_damp - r)/(r_damp - r_exc))^2;
- field energy: at m = 0 the diagnostic of a cavity-mode field equals the
  closed-form sum (1/8 pi)(sum D^2 + sum B^2) over the in-domain points.
"""
import numpy as np
import pytest

import oracle as O


# --- test inputs: the Kerr-Schild metric of the method in closed form,
# vectorised (checked against the oracle's own, pinned, metric below) ---------

def ks_metric(m, a, x, y, z):
    """g_{mu nu} and g^{mu nu} (..., 4, 4) at hole-relative points, index 3 =
    x^4, for g = eta + f k k with the paper's k (frame dragging clockwise
    about +z for a > 0)."""
    b = x * x + y * y + z * z - a * a
    r2 = 0.5 * (b + np.sqrt(b * b + 4 * a * a * z * z))
    r = np.sqrt(r2)
    f = 2 * m * r * r2 / (r2 * r2 + a * a * z * z)
    k = np.stack([(r * x - a * y) / (r2 + a * a), (r * y + a * x) / (r2 + a * a), z / r, np.ones_like(r)], -1)
    eta = np.diag([1.0, 1.0, 1.0, -1.0])
    ku = k * np.array([1.0, 1.0, 1.0, -1.0])  # k^mu = eta^{mu nu} k_nu
    g = eta + f[..., None, None] * k[..., :, None] * k[..., None, :]
    gi = eta - f[..., None, None] * ku[..., :, None] * ku[..., None, :]
    return g, gi


def test_closed_form_metric_is_the_oracle_metric():
    m, a = 1.5, 1.35
    p = O.make_params(16, m=m, a=a, r_exc=0.0)
    rng = np.random.default_rng(40)
    for _ in range(50):
        x, y, z = rng.uniform(-6, 6, 3)
        g, gi, _ = O.metric(p, x, y, z)
        g2, gi2 = ks_metric(m, a, np.array(x), np.array(y), np.array(z))
        assert np.abs(g - g2).max() < 1e-13 and np.abs(gi - gi2).max() < 1e-12


# --- curved face-area weights (Sec. 4) ----------------------------------------

def _area_density(p, I, J, P, cen):
    g, _, _ = O.metric(p, *(np.asarray(P) - cen))
    return np.sqrt(g[I, I] * g[J, J] - g[I, J] * g[J, I])


def _face_weights_quadrature(p, K, cell, mid, cen, gx, gw, variant="opposite"):
    """Sub-rectangle weights of a K-segment with mid-point `mid` in `cell`:
    node (bi, bj) takes the sub-rectangle opposite it, its density
    integrated with 5x5 Gauss-Legendre points.  The other variants are
    plausible mistakes, to show the bar catches them: "flat" (no density),
    "corner" (the density at the node itself), "own" (the density of the
    node's own sub-rectangle over the opposite area)."""
    I, J = (K + 1) % 3, (K + 2) % 3

    def rect(bi, bj):
        i0, i1 = (cell[I], mid[I]) if bi else (mid[I], cell[I] + 1.0)
        j0, j1 = (cell[J], mid[J]) if bj else (mid[J], cell[J] + 1.0)
        return i0, i1, j0, j1

    V = np.zeros((2, 2))
    for bj in range(2):
        for bi in range(2):
            i0, i1, j0, j1 = rect(bi, bj)
            area = (i1 - i0) * (j1 - j0)
            P = np.array(mid, dtype=float)
            if variant == "flat":
                V[bi, bj] = area
            elif variant == "corner":
                P[I], P[J] = cell[I] + bi, cell[J] + bj
                V[bi, bj] = area * _area_density(p, I, J, P, cen)
            elif variant == "own":
                o0, o1, q0, q1 = rect(1 - bi, 1 - bj)
                P[I], P[J] = 0.5 * (o0 + o1), 0.5 * (q0 + q1)
                V[bi, bj] = area * _area_density(p, I, J, P, cen)
            else:
                tot = 0.0
                for u, wu in zip(gx, gw):
                    for v, wv in zip(gx, gw):
                        P[I] = 0.5 * (i0 + i1) + 0.5 * (i1 - i0) * u
                        P[J] = 0.5 * (j0 + j1) + 0.5 * (j1 - j0) * v
                        tot += 0.25 * wu * wv * area * _area_density(p, I, J, P, cen)
                V[bi, bj] = tot
    return V / V.sum()


def test_curved_area_weights_match_quadrature():
    # a chord along K inside one cell is split at its midpoint into two
    # segments whose mid-planes lie at 1/4 and 3/4 of the chord; the current
    # on the cell's four K-edges is sum over segments of (Q dK / 2 dt) w.
    # Near the hole (R 3..5 cells) the oracle's midpoint rule differs from the
    # quadrature by its own O(h^2) error (measured 6e-4 < 2e-3 of the
    # weights), while flat weights, the density at the node or the density of
    # the node's own sub-rectangle miss by more than 1e-2.
    m, a, N = 1.5, 1.2, 16
    p = O.make_params(N, m=m, a=a, dt=0.5, r_exc=0.0)
    cen = np.array([N / 2.0] * 3)
    gx, gw = np.polynomial.legendre.leggauss(5)
    rng = np.random.default_rng(41)
    worst = 0.0
    planted = {"flat": 0.0, "corner": 0.0, "own": 0.0}
    done = 0
    while done < 30:
        X = cen + rng.uniform(-8, 8, 3)
        R = np.linalg.norm(X - cen)
        if not (3.0 < R < 5.0):
            continue
        cell = np.floor(X)
        for K in range(3):
            d = rng.uniform(0.1, 0.6) * (cell[K] + 1.0 - X[K])  # stays in the cell
            X2 = X.copy()
            X2[K] += d
            s = O.Sim(p, 0)
            Q = 1.0
            s.deposit_moves(X[:, None], X2[:, None], np.array([Q]))
            JK = s.get("J")[K]
            I, J = (K + 1) % 3, (K + 2) % 3
            got = np.zeros((2, 2))
            for bj in range(2):
                for bi in range(2):
                    idx = cell.astype(int).copy()
                    idx[I] += bi
                    idx[J] += bj
                    got[bi, bj] = JK[idx[2] + 1, idx[1] + 1, idx[0] + 1]
            refs = {v: np.zeros((2, 2)) for v in ("opposite", "flat", "corner", "own")}
            for frac in (0.25, 0.75):
                mid = X.copy()
                mid[K] += frac * d
                for v in refs:
                    refs[v] += _face_weights_quadrature(p, K, cell, mid, cen, gx, gw, v)
            scale = Q * d / (2 * p.dt)
            worst = max(worst, np.abs(got / scale - refs["opposite"]).max())
            for v in planted:
                planted[v] = max(planted[v], np.abs(refs[v] - refs["opposite"]).max())
        done += 1
    print("area weights vs quadrature: %.2e; planted mistakes: %s" % (worst, planted))
    assert worst < 2e-3, worst
    assert min(planted.values()) > 5e-3, planted


# --- the constitutive step (Sec. 3) -------------------------------------------

@pytest.mark.parametrize("a_frac", [0.0, 0.5, 0.95])
def test_constitutive_step_is_raising_with_the_metric(a_frac):
    # from the evolved half of the field tensor, (F_23, F_31, F_12) and
    # (F^14, F^24, F^34), the oracle solves for (F_14, F_24, F_34) and
    # (F^23, F^31, F^12); numpy raises a random F_ab with the metric
    m = 1.5
    a = a_frac * m
    N = 16
    p = O.make_params(N, m=m, a=a, r_exc=0.0)
    rplus = m + np.sqrt(m * m - a * a)
    rng = np.random.default_rng(42)
    pairs_s, pairs_t = ((1, 2), (2, 0), (0, 1)), ((0, 3), (1, 3), (2, 3))
    worst = 0.0
    done = 0
    while done < 200:
        x = rng.uniform(-8, 8, 3)
        if O.radius(a, *x) < 1.05 * rplus:
            continue
        _, gi, _ = O.metric(p, *x)
        A = rng.normal(0, 1, (4, 4))
        Fl = A - A.T
        Fu = gi @ Fl @ gi.T
        Fs_lo = [Fl[i, j] for i, j in pairs_s]
        Ft_up = [Fu[i, j] for i, j in pairs_t]
        tl, su = O.constitutive_point(p, x + N / 2.0, Fs_lo, Ft_up)
        want_tl = np.array([Fl[i, j] for i, j in pairs_t])
        want_su = np.array([Fu[i, j] for i, j in pairs_s])
        scale = max(np.abs(Fl).max(), np.abs(Fu).max())
        worst = max(worst, np.abs(tl - want_tl).max() / scale, np.abs(su - want_su).max() / scale)
        done += 1
    assert worst < 1e-12, worst


# --- Wald's vacuum solution in Kerr --------------------------------------------

def _wald_A(m, a, B0, X, cen):
    """A_mu = (B0/2)(psi_mu - 2 a xi_mu) at node coordinates X (..., 3):
    psi = x d_y - y d_x (rotation about the hole's axis) and xi = d_4 are
    Killing vectors of the metric, so dA is a source-free Maxwell field.  With
    the frame dragging of this metric (the sign of a opposite to the usual
    Boyer-Lindquist one) this combination leaves the hole uncharged."""
    x, y, z = (X[..., q] - cen[q] for q in range(3))
    g, _ = ks_metric(m, a, x, y, z)
    psi = np.stack([-y, x, np.zeros_like(x), np.zeros_like(x)], -1)
    return 0.5 * B0 * (np.einsum("...mn,...n->...m", g, psi) - 2.0 * a * g[..., :, 3])


def _wald_fields(N, m, a, B0):
    """Ghosted D = F^{j4} and B_cov = (F_23, F_31, F_12) of Wald's solution:
    B_cov is the discrete curl of A_j taken at the E points (exactly
    divergence-free), D the raised analytic F at the E points."""
    cen = np.full(3, N / 2.0)
    idx = np.arange(-1, N + 3, dtype=float)  # one beyond the ghost layer for the curl
    K3, J3, I3 = np.meshgrid(idx, idx, idx, indexing="ij")
    base = np.stack([I3, J3, K3], -1)
    Aedge = []
    for c in range(3):
        P = base.copy()
        P[..., c] += 0.5
        Aedge.append(_wald_A(m, a, B0, P, cen)[..., c])
    Ax, Ay, Az = Aedge
    sl = slice(0, N + 3)
    B = np.zeros((3, N + 3, N + 3, N + 3))
    # F_23 at (i, j+1/2, k+1/2); F_31 at (i+1/2, j, k+1/2); F_12 at (i+1/2, j+1/2, k)
    B[0] = (Az[sl, 1:, sl] - Az[sl, :-1, sl])[:, :N + 3, :] - (Ay[1:, sl, sl] - Ay[:-1, sl, sl])[:N + 3]
    B[1] = (Ax[1:, sl, sl] - Ax[:-1, sl, sl])[:N + 3] - (Az[sl, sl, 1:] - Az[sl, sl, :-1])[:, :, :N + 3]
    B[2] = (Ay[sl, sl, 1:] - Ay[sl, sl, :-1])[:, :, :N + 3] - (Ax[sl, 1:, sl] - Ax[sl, :-1, sl])[:, :N + 3, :]
    D = np.zeros_like(B)
    h = 1e-5
    for c in range(3):
        P = base[:N + 3, :N + 3, :N + 3].copy()
        P[..., c] += 0.5
        x, y, z = (P[..., q] - cen[q] for q in range(3))
        _, gi = ks_metric(m, a, x, y, z)
        dA = np.zeros(P.shape[:3] + (4, 4))  # dA[..., mu, nu] = d_mu A_nu; d_4 = 0
        for mu in range(3):
            e = np.zeros(3)
            e[mu] = h
            dA[..., mu, :] = (_wald_A(m, a, B0, P + e, cen) - _wald_A(m, a, B0, P - e, cen)) / (2 * h)
        F = dA - np.swapaxes(dA, -1, -2)
        Fu = np.einsum("...ma,...ab,...nb->...mn", gi, F, gi)
        D[c] = np.nan_to_num(Fu[..., c, 3])
    return D, np.nan_to_num(B)


def _wald_sim(N, m, a, B0):
    p = O.make_params(N, m=m, a=a, dt=0.45)
    s = O.Sim(p, 0)
    s.init_fields([0.0, 0.0, 0.0])
    D, B = _wald_fields(N, m, a, B0)
    # points inside r_exc are frozen and never raised or lowered: zero there
    for F, half in ((D, lambda c, ax: ax == c), (B, lambda c, ax: ax != c)):
        for c, r in enumerate(_radius_of_points(N, a, half)):
            F[c][r < p.r_exc] = 0.0
    s.set_fields(D, B)
    s.make_reference()
    return p, s, D, B


def ks_radius(a, x, y, z):
    """r of the quartic, with the cancellation-free form for R^2 < a^2."""
    b = x * x + y * y + z * z - a * a
    sq = np.sqrt(b * b + 4 * a * a * z * z)
    with np.errstate(divide="ignore", invalid="ignore"):
        r2 = np.where(b >= 0, 0.5 * (b + sq), 2 * a * a * z * z / np.where(sq - b > 0, sq - b, 1.0))
    return np.sqrt(r2)


def _radius_of_points(N, a, kind_half):
    idx = np.arange(-1, N + 2, dtype=float)
    K3, J3, I3 = np.meshgrid(idx, idx, idx, indexing="ij")
    out = []
    for c in range(3):
        off = [0.5 if kind_half(c, ax) else 0.0 for ax in range(3)]
        out.append(ks_radius(a, I3 + off[0] - N / 2.0, J3 + off[1] - N / 2.0, K3 + off[2] - N / 2.0))
    return out


def _one_step_change(N, m, a, B0, lo, hi):
    """Largest one-cycle change of B and D (relative to B0) at points with
    lo <= r/m < hi."""
    p, s, D, B = _wald_sim(N, m, a, B0)
    s.step(1)
    dB = np.abs(s.get("B") - B)
    dD = np.abs(s.get("D") - D)
    rB = _radius_of_points(N, a, lambda c, ax: ax != c)
    rD = _radius_of_points(N, a, lambda c, ax: ax == c)
    out = []
    for d, r in ((dB, rB), (dD, rD)):
        w = max(float(d[c][(r[c] >= lo * m) & (r[c] < hi * m)].max()) for c in range(3))
        out.append(w / B0)
    return out


def test_wald_kerr_one_step_change_is_second_order():
    # the far region r/m in [6.7, 8.7] lies more than 8 cells from the
    # excision at the coarse resolution (the fixed-point passes of one cycle
    # reach about that far) and inside the frozen faces
    a_frac, B0 = 0.9, 0.1
    coarse = _one_step_change(32, 1.5, a_frac * 1.5, B0, 6.7, 8.7)
    fine = _one_step_change(64, 3.0, a_frac * 3.0, B0, 6.7, 8.7)
    ratios = [c / f for c, f in zip(coarse, fine)]
    print("Wald Kerr one-step change (B, D) / B0: coarse %s fine %s ratios %s" % (coarse, fine, ratios))
    assert coarse[0] > 1e-9  # the truncation error is measured, not round-off
    for r in ratios:
        assert 6.0 < r < 11.0, ratios


def test_wald_kerr_far_field_stays_bounded():
    # Over hundreds of cycles Wald's field around an a = 0.9 m hole is not
    # held at its truncation level everywhere: the region inside the horizon,
    # where the fields are excised and relaxed (readings), departs from the
    # solution by O(B0) within a few cycles, and the centred stencils, which
    # do not follow the inward tilt of the light cones there, let part of it
    # travel out at about c (one-cycle changes just outside the horizon fall
    # at second order with resolution; the interior's do not).  Far from the
    # hole (r > 3 r_+) the deviation stays bounded, without growth:
    # measured 0.04-0.13 B0 over 300 cycles.
    N, m, a, B0 = 24, 1.5, 1.35, 0.1
    p, s, D, B = _wald_sim(N, m, a, B0)
    rplus = m + np.sqrt(m * m - a * a)
    rB = _radius_of_points(N, a, lambda c, ax: ax != c)
    devs = []
    for _ in range(3):
        s.step(100)
        dB = np.abs(s.get("B") - B)
        devs.append(max(float(dB[c][rB[c] > 3.0 * rplus].max()) for c in range(3)) / B0)
    print("Wald Kerr deviation of B beyond 3 r_+ after 100, 200, 300 cycles / B0:", devs)
    assert max(devs) < 0.2, devs
    assert devs[2] < 1.5 * devs[0] + 0.05, devs


# --- relaxation inside the horizon --------------------------------------------

def test_inner_relaxation_is_the_stated_pull_toward_the_reference():
    N, m, a = 16, 1.5, 1.2
    rplus = m + np.sqrt(m * m - a * a)
    r_exc, r_damp, damp = 0.5 * rplus, rplus, 0.1
    runs = {}
    rng = np.random.default_rng(43)
    pert = None
    for dm in (damp, 0.0):
        p = O.make_params(N, m=m, a=a, dt=0.5, r_exc=r_exc, r_damp=r_damp, damp_max=dm)
        s = O.Sim(p, 0)
        s.init_fields([0.0, 0.0, 0.05])
        D0, B0 = s.get("D"), s.get("B")
        if pert is None:
            pert = (rng.normal(0, 1e-3, D0.shape), rng.normal(0, 1e-3, B0.shape))
        s.set_fields(D0 + pert[0], B0 + pert[1])
        s.step(1)
        runs[dm] = (s.get("D"), s.get("B"), D0, B0)
    Dd, Bd, D0, B0 = runs[damp]
    Dn, Bn, _, _ = runs[0.0]
    rD = _radius_of_points(N, a, lambda c, ax: ax == c)
    rB = _radius_of_points(N, a, lambda c, ax: ax != c)
    inside = 0
    worst = 0.0
    for got, free, ref, rr in ((Dd, Dn, D0, rD), (Bd, Bn, B0, rB)):
        for c in range(3):
            t = np.clip((r_damp - rr[c]) / (r_damp - r_exc), 0.0, None)
            sg = np.where((rr[c] >= r_exc) & (rr[c] < r_damp), damp * t * t, 0.0)
            want = free[c] - sg * (free[c] - ref[c])
            worst = max(worst, float(np.abs(got[c] - want).max()))
            inside += int((sg > 0).sum())
    assert inside > 50
    assert worst < 1e-15, worst


# --- field-energy diagnostic ---------------------------------------------------

def test_field_energy_of_cavity_modes_is_the_closed_form():
    # m = 0: E_cov = -D and H = B_cov at updated points, so the energy is
    # (1/8 pi)(sum D^2 + sum B^2).  Frozen points (the outermost node layers)
    # hold the derived values of the reference state, so they count only
    # when the reference is the field itself.  D^y = A sin(pi n x / N) at
    # (i, j+1/2, k): over i = 0..N the sum of sin^2 is N/2, N values of j;
    # B^z = A cos(pi n x / N) at (i+1/2, j+1/2, k): over i = 0..N-1 the sum
    # of cos^2 at the half points is N/2, N values of j.  k runs over the
    # N - 1 updated layers with a zero reference, over all N + 1 with the
    # mode as reference.
    N, amp, nx = 12, 0.3, 3
    i = np.arange(-1, N + 2, dtype=float)
    for as_reference, nk in ((False, N - 1), (True, N + 1)):
        p = O.make_params(N, m=0.0, dt=0.5)
        s = O.Sim(p, 0)
        s.init_fields([0.0, 0.0, 0.0])
        D0, B0 = s.get("D"), s.get("B")
        Dm = D0.copy()
        Dm[1][:, :, :] = amp * np.sin(np.pi * nx * i / N)[None, None, :]
        Bm = B0.copy()
        Bm[2][:, :, :] = amp * np.cos(np.pi * nx * (i + 0.5) / N)[None, None, :]
        want = amp ** 2 * (N / 2.0) * N * nk / (8 * np.pi)
        got = []
        for D, B in ((Dm, B0), (D0, Bm), (Dm, Bm)):
            s.set_fields(D, B)
            if as_reference:
                s.make_reference()
            got.append(s.diag()["energy_field"])
        print("cavity energies (reference = mode: %s): %s, closed form %.15g each" % (as_reference, got, want))
        assert abs(got[0] - want) < 1e-13 * want
        assert abs(got[1] - want) < 1e-13 * want
        assert abs(got[2] - 2 * want) < 1e-13 * want
