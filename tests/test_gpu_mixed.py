"""FP32-mixed form (packed cell + FP32 offset, FP32 push/gather/fields, FP64
radius and near-horizon metric) against the FP64 form and the FP64 oracle.

Accuracy contract: trajectories within 1e-4 relative of FP64 (positions
relative to max(|x|, 1 cell), four-velocities relative to max(|u|, c)) and
grid currents within 1e-5 of the FP64 current's scale.  Every comparison
prints its error against the FP64 reference it is checked on.
"""
import numpy as np
import pytest

import oracle as O
from common import alive, gpu_run, oracle_sim, params, rel_err, say

pytestmark = pytest.mark.gpu


def _run(P, capacity, precision, sort_every=0, fp_bits=50):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    cfg = R.make_config(P["n"], m=P["m"], a=P["a"], dt=P["dt"], B0=P["B0"], species=P["species"],
                        r_rm=P["r_rm"], gamma_mode=P["gamma_mode"], deposit_mode=P["deposit_mode"],
                        field_iters=P["field_iters"], damp_max=P["damp_max"], sort_every=sort_every,
                        capacity=capacity, fp_bits=fp_bits,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    return R.Run(cfg)


def _parts(seed, n, N, u_th=0.1):
    g = np.random.default_rng(seed)
    x = g.uniform(1.0, N - 1.0, (3, n))
    return [(0, x, g.normal(0.0, u_th, (3, n))), (1, x.copy(), g.normal(0.0, u_th / np.sqrt(20.0), (3, n)))]


P32 = params(32, m=1.5, a=1.425, dt=0.45, B0=(0.0, 0.0, 0.1), species=((-0.005, 0.005), (0.005, 0.1)))


def _pair(parts, P=P32, sort_every=0):
    cap = sum(p[1].shape[1] for p in parts)
    r64 = _run(P, cap, "fp64", sort_every)
    r32 = _run(P, cap, "fp32", sort_every)
    for sp, x, uc in parts:
        k64 = r64.load(sp, x, uc)
        k32 = r32.load(sp, x, uc)
        assert k64 == k32
    return r64, r32


def _traj_err(r64, r32):
    x6, u6, s6 = r64.particles()
    x3, u3, s3 = r32.particles()
    both = (s6 != O.DEAD) & (s3 != O.DEAD)
    ex = np.abs(x3[:, both] - x6[:, both]) / np.maximum(np.abs(x6[:, both]), 1.0)
    eu = np.abs(u3[:, both] - u6[:, both]) / np.maximum(np.abs(u6[:, both]), 1.0)
    return ex.max(axis=0), eu.max(axis=0), int(both.sum()), int(((s6 != O.DEAD) != (s3 != O.DEAD)).sum())


def test_mixed_load_matches_fp64_load():
    parts = _parts(1, 4000, 32)
    r64, r32 = _pair(parts)
    ex, eu, nboth, ndiff = _traj_err(r64, r32)
    say("load: x err %.2e u err %.2e" % (ex.max(), eu.max()))
    assert ndiff == 0
    assert ex.max() < 1e-7 and eu.max() < 1e-6


def test_mixed_cycle_tracks_fp64():
    parts = _parts(2, 20000, 32)
    r64, r32 = _pair(parts)
    r64.step(1)
    r32.step(1)
    J6, J3 = r64.fields("J"), r32.fields("J")
    ej = np.abs(J3 - J6).max() / np.abs(J6).max()
    ex, eu, nboth, ndiff = _traj_err(r64, r32)
    say("step 1: J err %.2e  x err %.2e u err %.2e  (%d compared, %d removal mismatches)" %
        (ej, ex.max(), eu.max(), nboth, ndiff))
    assert ej < 1e-5
    assert ex.max() < 1e-4 and eu.max() < 1e-4
    r64.step(49)
    r32.step(49)
    ex, eu, nboth, ndiff = _traj_err(r64, r32)
    frac = float(((ex < 1e-4) & (eu < 1e-4)).mean())
    say("step 50: x err max %.2e median %.2e, u err max %.2e, fraction within 1e-4: %.5f, removal mismatches %d"
        % (ex.max(), np.median(ex), eu.max(), frac, ndiff))
    assert frac > 0.99
    assert ndiff <= max(2, nboth // 1000)


def test_mixed_one_step_against_oracle():
    """One FP32-mixed step against the FP64 oracle, both loading the same
    inputs (the mixed form rounds them to FP32 offsets and velocities).
    Particle state and B within 1e-5; J within 1e-5 in L2 (the max norm is
    printed: a particle within an FP32 rounding of a cell face can take the
    other zigzag decision)."""
    P = P32
    parts = _parts(3, 5000, 32)
    cap = 10000
    r = _run(P, cap, "fp32")
    p, s = oracle_sim(P, cap)
    for sp, x, uc in parts:
        assert r.load(sp, x, uc) == s.load(sp, x, uc)
    r.step(1)
    s.step(1)
    xo, uo, so = alive(*s.particles())
    xg, ug, sg = alive(*r.particles())
    assert np.array_equal(so, sg)
    ex = rel_err(xg, xo, 1.0)
    eu = rel_err(ug, uo, 1.0)
    Jo, Jg = s.get("J"), r.fields("J")
    ej = np.abs(Jg - Jo).max() / np.abs(Jo).max()
    ej2 = np.linalg.norm(Jg - Jo) / np.linalg.norm(Jo)
    eB = np.abs(r.fields("B") - s.get("B")).max() / np.abs(s.get("B")).max()
    say("fp32-mixed vs FP64 oracle, one step: x %.2e u %.2e J max %.2e L2 %.2e B %.2e" % (ex, eu, ej, ej2, eB))
    assert ex < 1e-5 and eu < 1e-5 and ej2 < 1e-5 and eB < 1e-5


def test_mixed_sort_keys_bit_exact():
    P = P32
    parts = _parts(4, 6000, 32)
    r = _run(P, 12000, "fp32")
    for sp, x, uc in parts:
        r.load(sp, x, uc)
    r.step(3)
    x, u, sp = r.particles()
    keys, perm = r.sort()
    p = O.make_params(32, m=P["m"], a=P["a"])
    ko = O.sort_keys(p, r.cfg.tile, x, sp)
    po = O.stable_order(ko)
    assert np.array_equal(keys, ko[po])
    assert np.array_equal(perm, po)


def _torus_runs(nps, B0, start_same):
    """FP64 and FP32-mixed runs of the 128^3 torus workload (Kerr a = 0.5m,
    m = 4) with nps particles per species, in the same slot order.  With
    start_same the FP64 run starts from the mixed run's loaded state (the
    inputs rounded to FP32 offsets and velocities), so differences come from
    the FP32 arithmetic of the steps alone."""
    from paper_0904_0232_amd import inputs
    w = inputs.workload_params("torus128")
    P = params(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, B0), species=w["species"], r_rm=w["r_rm"])
    parts = inputs.workload_particles("torus128", seed=0, n_override=nps)
    cap = 2 * nps
    # 44 fraction bits: the densest torus cells sum ~10^4 contributions
    r64, r32 = _run(P, cap, "fp64", fp_bits=44), _run(P, cap, "fp32", fp_bits=44)
    for sp, x, uc in parts:
        r32.load(sp, x, uc)
        if not start_same:
            r64.load(sp, x, uc)
    r32.sort()
    if start_same:
        r64.restore_particles(*r32.particles())
    else:
        r64.sort()
    return w, r64, r32


def test_mixed_torus_geodesic_1000_steps():
    """Test particles of the torus workload on geodesics (no field) for 1000
    RK4 steps, FP32-mixed against FP64 from the same start.  Particles whose
    FP64 path leaves the grid or comes within 3m of the hole (plunging orbits
    from inside the marginally stable radius, which amplify any difference)
    are not counted as regular."""
    w, r64, r32 = _torus_runs(20000, 0.0, True)
    cen = np.full(3, w["n"] / 2.0)
    regular = None
    for block in range(10):
        r64.push_only(100)
        r32.push_only(100)
        x6, u6, s6 = r64.particles()
        R = np.sqrt(((x6 - cen[:, None]) ** 2).sum(0))
        ok = np.all((x6 >= 0) & (x6 < w["n"]), axis=0) & (R > 3.0 * w["m"]) & np.isfinite(u6).all(0)
        regular = ok if regular is None else (regular & ok)
    x3, u3, s3 = r32.particles()
    ex = (np.abs(x3 - x6) / np.maximum(np.abs(x6), 1.0)).max(axis=0)[regular]
    eu = (np.abs(u3 - u6) / np.maximum(np.abs(u6), 1.0)).max(axis=0)[regular]
    e = np.maximum(ex, eu)
    frac = float((e < 1e-4).mean())
    say("torus geodesics, 1000 steps: %d of %d regular, error median %.2e p90 %.2e p99 %.2e, "
        "fraction within 1e-4: %.4f" % (regular.sum(), regular.size, np.median(e), np.quantile(e, 0.9),
                                         np.quantile(e, 0.99), frac))
    assert regular.sum() > 0.5 * regular.size
    assert np.median(e) < 1e-5
    assert frac > 0.95


def _ks_radius(a, x, y, z):
    b = x * x + y * y + z * z - a * a
    return np.sqrt(0.5 * (b + np.sqrt(b * b + 4.0 * a * a * z * z)))


def _coarse_current(x, u, sp, w, mask, block=8):
    """Current of the particles in `mask` coarse-grained over blocks of
    block^3 cells: per species s, J_s^i(b) = sum over those particles in
    block b of q_s c u^i / u^4 (c = 1), and the net current; shape
    (nspecies + 1, 3, nblocks)."""
    n = w["n"]
    nb = n // block
    with np.errstate(invalid="ignore", over="ignore"):
        fin = np.isfinite(x).all(0) & np.isfinite(u).all(0)
        xs = np.where(fin, x, -1.0)
        inside = np.all((xs >= 0) & (xs < n), axis=0)
    kept = mask & (sp != O.DEAD) & fin & inside
    idx = np.clip(np.floor(xs[:, kept] / block).astype(np.int64), 0, nb - 1)
    flat = (idx[2] * nb + idx[1]) * nb + idx[0]
    v = u[:3, kept] / u[3, kept]
    out = np.zeros((len(w["species"]) + 1, 3, nb ** 3))
    for s, (q, _) in enumerate(w["species"]):
        sel = sp[kept] == s
        for i in range(3):
            out[s, i] = np.bincount(flat[sel], weights=q * v[i, sel], minlength=nb ** 3)
    out[-1] = out[:-1].sum(axis=0)
    return out


def test_mixed_torus_frozen_field_1000_steps():
    """Test particles of the torus workload in the frozen initial field
    (B_z = 0.1) for 1000 RK4 steps, 100,000 per species.  Three runs keep
    particle identity: A FP64 from the exact inputs, B FP64 from the inputs
    rounded to the mixed representation, C FP32-mixed.  The field dominates
    gravity here (the electrons' gyration radius is about 4.5 cells and
    their E x B drift tens of cells over the run), so most particles reach
    the hole or the faces, where nothing removes them in push-only steps;
    "regular" orbits are those whose FP64 path stays in the grid and
    outside 3m throughout (under 1% of them).  C - B (the FP32 arithmetic
    of the steps), over the regular orbits: at least 80% within 1e-4 and
    median below 3e-5 (about 45 radians of gyration phase at FP32's
    relative rounding); the current of the regular orbits of each species
    that has at least 200 of them, coarse-grained over 8^3-cell blocks,
    within 1e-4 in L2 at step 1000.
    C - A and the control B - A (how far FP64 carries one FP32 rounding of
    the start) are printed, and so is the coarse-grained current of every
    particle a cycle would keep (alive, in the grid, outside r_rm), which
    the plunging orbits dominate."""
    w, rb, r32 = _torus_runs(100000, 0.1, True)
    _, ra, r32b = _torus_runs(100000, 0.1, False)
    r32b.close()
    runs = {"A": ra, "B": rb, "C": r32}
    cen = np.full(3, w["n"] / 2.0)
    regular = None
    for block in range(10):
        for r in runs.values():
            r.push_only(100)
        xa, ua, sa = ra.particles()
        with np.errstate(invalid="ignore"):
            R = np.sqrt(((xa - cen[:, None]) ** 2).sum(0))
            ok = np.all((xa >= 0) & (xa < w["n"]), axis=0) & (R > 3.0 * w["m"]) & np.isfinite(ua).all(0)
        ok &= sa != O.DEAD
        regular = ok if regular is None else (regular & ok)
    st = {k: r.particles() for k, r in runs.items()}

    def err(P, Q):
        (x1, u1, s1), (x2, u2, s2) = P, Q
        both = regular & (s1 != O.DEAD) & (s2 != O.DEAD)
        with np.errstate(invalid="ignore", over="ignore"):
            ex = (np.abs(x2 - x1) / np.maximum(np.abs(x1), 1.0)).max(axis=0)[both]
            eu = (np.abs(u2 - u1) / np.maximum(np.abs(u1), 1.0)).max(axis=0)[both]
        e = np.maximum(ex, eu)
        return np.where(np.isfinite(e), e, np.inf)  # a non-finite particle counts as far off

    def kept_mask(x, u, sp):
        with np.errstate(invalid="ignore", over="ignore"):
            xs = np.where(np.isfinite(x).all(0), x, -1.0)
            return _ks_radius(w["a"], *(xs - w["n"] / 2.0)) > w["r_rm"]

    Jreg = {k: _coarse_current(*v, w, regular) for k, v in st.items()}
    Jall = {k: _coarse_current(*v, w, kept_mask(*v)) for k, v in st.items()}

    def jerr(J, a, b):
        return [float(np.linalg.norm(J[b][s] - J[a][s]) / np.linalg.norm(J[a][s])) for s in range(3)]

    e = {}
    for name, (a, b) in (("fp32 arithmetic C-B", ("B", "C")), ("FP32-mixed C-A", ("A", "C")),
                         ("FP64 control B-A", ("A", "B"))):
        e[name] = err(st[a], st[b])
        say("torus frozen field, 1000 steps, %s: %d regular of %d, median %.2e p99 %.2e, within 1e-4 %.4f; "
            "coarse J L2 (electrons, ions, net) of the regular orbits %s, of every kept particle %s" % (
                name, e[name].size, regular.size, np.median(e[name]), np.quantile(e[name], 0.99),
                float((e[name] < 1e-4).mean()), ["%.2e" % v for v in jerr(Jreg, a, b)],
                ["%.2e" % v for v in jerr(Jall, a, b)]))
    arith = e["fp32 arithmetic C-B"]
    sp = st["A"][2]
    nreg = [int((regular & (sp == s)).sum()) for s in range(2)]
    say("regular orbits per species (electrons, ions): %s" % nreg)
    assert regular.sum() >= 500
    assert np.median(arith) < 3e-5
    assert float((arith < 1e-4).mean()) > 0.80
    je = jerr(Jreg, "B", "C")
    # the current of a species is compared where it has enough regular
    # orbits to be a current (the electrons' gyration and drift leave few)
    checked = [s for s in range(2) if nreg[s] >= 200]
    assert checked
    for s in checked:
        assert je[s] < 1e-4, (s, je)
    for r in runs.values():
        r.close()


def test_mixed_torus_current_one_step():
    """One self-consistent cycle of the torus workload (1M particles per
    species, field B_z = 0.1): the FP32-mixed current against FP64 from the
    same start, within 1e-5 of max|J|.  From the exact inputs instead, a few
    particles within an FP32 rounding of a cell face take the other crossing
    decision, and the zigzag relay point jumps there; electrons and ions
    nearly cancel in this co-rotating plasma, so that shows in the max norm
    (printed, bounded only in L2)."""
    for same in (True, False):
        w, r64, r32 = _torus_runs(1 << 20, 0.1, same)
        r64.step(1)
        r32.step(1)
        J6, J3 = r64.fields("J"), r32.fields("J")
        emax = np.abs(J3 - J6).max() / np.abs(J6).max()
        el2 = np.linalg.norm(J3 - J6) / np.linalg.norm(J6)
        say("torus one cycle, %s start: J max-rel %.2e, L2-rel %.2e" % ("same" if same else "exact-input", emax, el2))
        if same:
            assert emax < 1e-5
        else:
            assert el2 < 1e-5
        r64.close()
        r32.close()


def test_mixed_gyration_closed_form():
    B = 0.05
    P = params(32, m=0.0, a=0.0, dt=0.5, B0=(0.0, 0.0, B), species=((-1.0, 1.0),))
    r = _run(P, 4, "fp32")
    u3 = np.array([0.3, 0.1, 0.0])
    u4 = np.sqrt(1 + u3 @ u3)
    r.restore_particles(np.array([[16.2], [15.7], [16.1]]), np.array([[u3[0]], [u3[1]], [0.0], [u4]]),
                        np.zeros(1, np.uint8))
    nsteps = 1000
    r.push_only(nsteps)
    _, u, _ = r.particles()
    z = 1j * B / u4 * 0.5
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    w_ref = (u3[0] + 1j * u3[1]) * R ** nsteps
    err = abs(u[0, 0] + 1j * u[1, 0] - w_ref) / abs(w_ref)
    say("fp32 gyration relative error after 1000 steps: %.2e" % err)
    assert err < 1e-4


def test_mixed_diagnostics_match_fp64():
    parts = _parts(6, 10000, 32)
    r64, r32 = _pair(parts)
    d6, d3 = r64.diag(), r32.diag()
    assert d6["n_alive"] == d3["n_alive"]
    for k in ("charge_total", "energy_particles", "lz_particles"):
        assert abs(d6[k] - d3[k]) <= 1e-6 * max(abs(d6[k]), 1e-30), (k, d6[k], d3[k])
    r64.step(10)
    r32.step(10)
    d6, d3 = r64.diag(), r32.diag()
    say("after 10 steps: energy fp64 %.10e fp32 %.10e" % (d6["energy_particles"], d3["energy_particles"]))
    assert abs(d6["energy_particles"] - d3["energy_particles"]) <= 1e-5 * abs(d6["energy_particles"])
