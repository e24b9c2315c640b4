"""GPU (HIP path through the C ABI) against the FP64 oracle.

Tolerances (FP64 path): particle state within 1e-12 relative per step
(positions relative to max(|x|, 1 cell), four-velocities to max(|u|, c));
fields within 1e-12 of the field's own scale, plus the fixed-point rounding
of the current (each contribution is rounded to 2^-fp_bits of the largest
species charge over dt).  Sort keys and order are compared bit for bit from
identical positions.
"""
import numpy as np
import pytest

import oracle as O
from common import alive, gpu_run, oracle_sim, params, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-12
FPB = 50  # fixed-point fraction bits used by the parity runs


def _load_both(P, s, r, parts):
    kept_o = kept_g = 0
    for sp, x, uc in parts:
        kept_o += s.load(sp, x, uc)
        kept_g += r.load(sp, x, uc)
    return kept_o, kept_g


def _small_parts(seed, n, N, u_th=0.1, margin=1.0):
    g = np.random.default_rng(seed)
    x = g.uniform(margin, N - margin, (3, n))
    ue = g.normal(0.0, u_th, (3, n))
    ui = g.normal(0.0, u_th / np.sqrt(20.0), (3, n))
    return [(0, x, ue), (1, x.copy(), ui)]


def _cmp_particles(s, r, tol=TOL, tag=""):
    xo, uo, spo = s.particles()
    xg, ug, spg = r.particles()
    xo, uo, spo = alive(xo, uo, spo)
    xg, ug, spg = alive(xg, ug, spg)
    assert np.array_equal(spo, spg), tag
    ex = rel_err(xg, xo, 1.0)
    eu = rel_err(ug, uo, 1.0)
    say(tag, "particles", xo.shape[1], "err x %.2e u %.2e" % (ex, eu))
    assert ex < tol and eu < tol, (tag, ex, eu)


def _cmp_field(a, b, name, tol=TOL, abs_floor=0.0):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    say(name, "err %.2e scale %.2e" % (err, scale))
    assert err <= tol * scale + abs_floor, (name, err, scale)


def _j_floor(P, ncontrib=64):
    qmax = max(abs(q) for q, _ in P["species"])
    return ncontrib * 0.5 * qmax / P["dt"] * 2.0 ** -FPB


def test_library_initial_fields_match_oracle():
    P = params(12, m=1.5, a=0.75, dt=0.5, B0=(0.01, -0.02, 0.05))
    say("case initial fields", P)
    p, s = oracle_sim(P, 0)
    r = gpu_run(P, 16, fp_bits=FPB)
    _cmp_field(r.fields("D"), s.get("D"), "D0", abs_floor=1e-300)
    _cmp_field(r.fields("B"), s.get("B"), "B0")
    r.diag()  # derives E_cov and H of the current state on the device
    s.compute_derived()
    _cmp_field(r.fields("E"), s.get("E"), "E_cov")
    _cmp_field(r.fields("H"), s.get("H"), "H")


@pytest.mark.parametrize("m,a", [(0.0, 0.0), (1.5, 0.0), (1.5, 1.4)])
def test_node_tensor_from_random_fields(m, a):
    P = params(10, m=m, a=a, dt=0.5)
    say("case node tensor", m, a)
    p, s = oracle_sim(P, 0)
    r = gpu_run(P, 16, fp_bits=FPB)
    g = np.random.default_rng(3)
    D = g.normal(0, 1e-2, (3,) + s.gshape)
    B = g.normal(0, 1e-2, (3,) + s.gshape) + np.array([0, 0, 0.05])[:, None, None, None]
    s.set_fields(D, B)
    r.restore_fields(D, B)
    s.compute_nodes()
    r.push_only(0)
    _cmp_field(r.nodes(), s.nodes(), "node F^a_b")


CASES = [
    dict(m=0.0, a=0.0, gamma_mode=0, deposit_mode=0),
    dict(m=1.5, a=0.0, gamma_mode=0, deposit_mode=0),
    dict(m=1.5, a=1.2, gamma_mode=0, deposit_mode=0),
    dict(m=1.5, a=1.2, gamma_mode=1, deposit_mode=1),
    # the units of the paper's application: c = 0.05, dt = 1
    dict(m=1.5, a=1.2, gamma_mode=0, deposit_mode=0, c=0.05, dt=1.0),
    # the outer absorbing layer
    dict(m=1.5, a=1.2, gamma_mode=0, deposit_mode=0, outer_layer=4.0, outer_damp=0.3),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "m%.1f_a%.1f_g%d_d%d_c%g_L%g" % (
    c["m"], c["a"], c["gamma_mode"], c["deposit_mode"], c.get("c", 1.0), c.get("outer_layer", 0.0)))
def test_cycle_parity_small(case):
    N = 16
    case = dict(case)
    dt = case.pop("dt", 0.5)
    P = params(N, dt=dt, B0=(0.0, 0.0, 0.08), species=((-0.02, 0.02), (0.02, 0.4)), **case)
    say("case cycle", case)
    parts = _small_parts(7, 1500, N)
    p, s = oracle_sim(P, 4000)
    r = gpu_run(P, 4000, fp_bits=FPB)
    ko, kg = _load_both(P, s, r, parts)
    assert ko == kg
    _cmp_particles(s, r, tag="load")
    for it in range(3):
        s.step(1)
        r.step(1)
        _cmp_particles(s, r, tag="step %d" % it)
        _cmp_field(r.fields("J"), s.get("J"), "J", abs_floor=_j_floor(P))
        _cmp_field(r.fields("B"), s.get("B"), "B")
        # the current enters D through (4 pi / c) dt
        _cmp_field(r.fields("D"), s.get("D"), "D", abs_floor=4 * np.pi * P["dt"] / P["c"] * _j_floor(P))
    do, dg = s.diag(), r.diag()
    for k in ("n_alive", "n_removed_horizon", "n_removed_outer", "gamma_clamps", "flags"):
        assert do[k] == dg[k], (k, do[k], dg[k])


def test_outer_layer_gauss_law_elsewhere():
    """Flat deposit with the outer absorbing layer: on the GPU, as in the
    oracle, Gauss's law holds to round-off at every node the diagnostic
    checks (outside the relaxation layers), and the relaxed fields agree."""
    N = 16
    P = params(N, m=1.5, a=0.75, dt=0.5, B0=(0.0, 0.0, 0.05), species=((-0.01, 0.01), (0.01, 0.2)),
               deposit_mode=1, outer_layer=4.0, outer_damp=0.3)
    parts = _small_parts(13, 3000, N)
    p, s = oracle_sim(P, 6000)
    r = gpu_run(P, 6000, fp_bits=FPB)
    _load_both(P, s, r, parts)
    s.step(4)
    r.step(4)
    do, dg = s.diag(), r.diag()
    say("outer layer: Gauss residual oracle %.2e GPU %.2e" % (do["gauss_residual_max"], dg["gauss_residual_max"]))
    assert do["gauss_residual_max"] < 1e-12 and dg["gauss_residual_max"] < 1e-9
    _cmp_field(r.fields("B"), s.get("B"), "B")
    _cmp_field(r.fields("D"), s.get("D"), "D", abs_floor=4 * np.pi * P["dt"] * _j_floor(P))


def test_schwarzschild32_parity_every_step():
    """The 32^3 Schwarzschild workload (65,536 particles, 10 steps): the
    oracle and the GPU load the same inputs and advance independently; the
    state is compared after every step."""
    from paper_0904_0232_amd import inputs
    w = inputs.workload_params("schwarzschild32")
    P = params(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
               r_rm=w["r_rm"])
    parts = inputs.workload_particles("schwarzschild32", seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    assert ntot == 65536
    p, s = oracle_sim(P, ntot)
    r = gpu_run(P, ntot, fp_bits=FPB)
    ko, kg = _load_both(P, s, r, parts)
    say("schwarzschild32 kept", ko, kg)
    assert ko == kg
    for it in range(w["steps"]):
        s.step(1)
        r.step(1)
        _cmp_particles(s, r, tag="s32 step %d" % it)
        _cmp_field(r.fields("B"), s.get("B"), "B")
        _cmp_field(r.fields("D"), s.get("D"), "D", abs_floor=4 * np.pi * P["dt"] * _j_floor(P, 256) * (it + 1))
    do, dg = s.diag(), r.diag()
    say("diag oracle", do)
    say("diag gpu", dg)
    assert do["n_alive"] == dg["n_alive"]
    for k in ("charge_total", "energy_particles", "lz_particles", "energy_field"):
        assert abs(do[k] - dg[k]) <= 1e-11 * max(abs(do[k]), 1e-30), k
    assert abs(do["gauss_residual_max"] - dg["gauss_residual_max"]) < 1e-9
    assert abs(do["mass_shell_residual_max"] - dg["mass_shell_residual_max"]) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_kerr64_one_cycle_parity_from_evolved_states(precision):
    """The 64^3 Kerr a = 0.95m workload at its full 4,194,304 particles,
    from states the GPU itself evolved: after 20 and after 40 cycles (cell
    sorts every 5 cycles, removals at the hole and the faces, the fields
    developed), the oracle takes the GPU's D, B and every particle slot, and
    both advance one cycle.  Particles, J, B and D are compared element by
    element: FP64 at the parity bar; FP32-mixed particles and B within 1e-5
    (max norm).  The FP32-mixed current: a particle that ends within an FP32
    rounding of a cell face can land in the other cell than in FP64, and the
    zigzag relay point jumps there (mid-chord inside one cell, the face when
    the chord crosses it), so that particle's share of J differs at the
    scale of its own flux.  J and D are therefore compared in L2 within
    1e-5 plus 1e-4 per particle whose end cell differs (counted)."""
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R
    w = inputs.workload_params("kerr64")
    P = params(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
               r_rm=w["r_rm"])
    parts = inputs.workload_particles("kerr64", seed=0)
    ntot = sum(x.shape[1] for _, x, _ in parts)
    cfg = R.make_config(P["n"], m=P["m"], a=P["a"], dt=P["dt"], B0=P["B0"], species=P["species"], r_rm=P["r_rm"],
                        sort_every=5, capacity=ntot, fp_bits=FPB,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    r = R.Run(cfg)
    for sp, x, uc in parts:
        r.load(sp, x, uc)
    done = 0
    for target in (20, 40):
        say("case kerr64 %s: GPU cycles to %d" % (precision, target))
        r.step(target - done)
        done = target
        x, u, sp = r.particles()
        p, s = oracle_sim(P, x.shape[1])
        s.set_fields(r.fields("D"), r.fields("B"))
        s.set_particles(x, u, sp)
        live0 = int((sp != O.DEAD).sum())
        s.step(1)
        r.step(1)
        done += 1
        tag = "kerr64 %s from cycle %d (%d live)" % (precision, target, live0)
        Jg, Jo = r.fields("J"), s.get("J")
        Dg, Do = r.fields("D"), s.get("D")
        if precision == "fp64":
            _cmp_particles(s, r, tag=tag)
            _cmp_field(Jg, Jo, "J", abs_floor=_j_floor(P, 256))
            _cmp_field(r.fields("B"), s.get("B"), "B")
            _cmp_field(Dg, Do, "D", abs_floor=4 * np.pi * P["dt"] * _j_floor(P, 256))
        else:
            _cmp_particles(s, r, tol=1e-5, tag=tag)
            _cmp_field(r.fields("B"), s.get("B"), "B", tol=1e-5)
            xg, _, sg = r.particles()
            xo, _, so = s.particles()
            both = (sg != O.DEAD) & (so != O.DEAD)
            flips = int(np.any(np.floor(xg[:, both]) != np.floor(xo[:, both]), axis=0).sum())
            for name, a, b in (("J", Jg, Jo), ("D", Dg, Do)):
                l2 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
                mx = float(np.abs(a - b).max() / np.abs(b).max())
                say(name, "L2 err %.2e, max err %.2e of max; particles ending in another cell: %d" % (l2, mx, flips))
                assert l2 < 1e-5 + 1e-4 * flips, (name, l2, flips)
        del s
    r.close()


def _sample_inputs(parts, sp_gpu, per_species, rng):
    """Pick per_species inputs of each species that the GPU kept; returns the
    picked (species, x, ucov) sub-arrays and the GPU slots they occupy (the
    GPU loads species after species, one slot per input, in input order)."""
    picked, slots, off = [], [], 0
    for spc, x, uc in parts:
        n = x.shape[1]
        live = np.nonzero(sp_gpu[off:off + n] != O.DEAD)[0]
        pk = np.sort(rng.choice(live, min(per_species, live.size), replace=False))
        picked.append((spc, x[:, pk], uc[:, pk]))
        slots.append(off + pk)
        off += n
    return picked, np.concatenate(slots)


def test_kerr64_full_size_sampled_push():
    """The 64^3 Kerr a=0.95m workload at its full 4,194,304 particles: one
    GPU step; the oracle recomputes the node tensor and pushes a sample."""
    from paper_0904_0232_amd import inputs
    w = inputs.workload_params("kerr64")
    P = params(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"])
    parts = inputs.workload_particles("kerr64", seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    assert ntot == 4194304
    r = gpu_run(P, ntot, fp_bits=44, sort_every=0)
    kept = sum(r.load(sp, x, uc) for sp, x, uc in parts)
    say("kerr64 kept", kept)
    x0, u0, sp0 = r.particles()
    r.step(1)
    x1, u1, sp1 = r.particles()
    # oracle: same initial fields, first half-cycle, node tensor; it loads a
    # sample of the same inputs itself and pushes it once
    p, s = oracle_sim(P, 4096)
    s.prepare_push()
    _cmp_field(r.nodes(), s.nodes(), "kerr64 node tensor")
    picked, slots = _sample_inputs(parts, sp0, 2000, np.random.default_rng(11))
    assert sum(s.load(spc, x, uc) for spc, x, uc in picked) == slots.size
    s.push_only(1)
    xs, us, _ = s.particles()
    ex = rel_err(x1[:, slots], xs, 1.0)
    eu = rel_err(u1[:, slots], us, 1.0)
    say("kerr64 sampled push err x %.2e u %.2e" % (ex, eu))
    assert ex < TOL and eu < TOL
    # total current per direction equals sum q dx / dt (any transverse weights)
    J = r.fields("J")
    qs = np.array([q for q, _ in P["species"]])
    ok = sp0 != O.DEAD
    for K in range(3):
        ref = (qs[sp0[ok]] * (x1[K, ok] - x0[K, ok])).sum() / P["dt"]
        floor = ok.sum() * 24 * 0.5 * np.abs(qs).max() / P["dt"] * 2.0 ** -44
        assert abs(J[K].sum() - ref) <= 1e-12 * np.abs(J[K]).sum() + floor, K


@pytest.mark.parametrize("N,tile,n", [(16, 8, 3000), (16, 4, 3000), (20, 8, 70000), (36, 4, 150000),
                                        (64, 4, 200000), (64, 8, 200000)])
def test_sort_bit_exact(N, tile, n):
    # one to 98 sort tiles of 4096 slots, a ragged last tile, grids that are
    # not a multiple of the cell tile, particles removed near the hole; keys
    # of 14 to 19 bits (two and three radix passes)
    P = params(N, m=1.5, a=0.9, dt=0.5, species=((-0.02, 0.02), (0.02, 0.4)))
    parts = _small_parts(9, n, N)
    r = gpu_run(P, 2 * n, fp_bits=FPB, tile=tile)
    for sp, x, uc in parts:
        r.load(sp, x, uc)
    r.step(3)
    x, u, sp = r.particles()
    say("case sort N=%d tile=%d: %d slots, %d removed" % (N, tile, sp.size, int((sp == O.DEAD).sum())))
    keys, perm = r.sort()
    p = O.make_params(N, m=1.5, a=0.9)
    ko = O.sort_keys(p, tile, x, sp)
    po = O.stable_order(ko)
    assert np.array_equal(keys, ko[po])
    assert np.array_equal(perm, po)
    x2, u2, sp2 = r.particles()
    nl = int((sp != O.DEAD).sum())
    assert x2.shape[1] == nl
    assert np.array_equal(x2, x[:, po[:nl]]) and np.array_equal(u2, u[:, po[:nl]])
    assert np.array_equal(sp2, sp[po[:nl]])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replay_equals_launches(precision):
    """A run whose cycles replay captured graphs (the default) equals, bit for
    bit after every cycle, a run that launches the kernels one by one; the
    cell sort falls between replays (every 5 cycles), and each replay is
    followed by host work (dumps, diagnostics)."""
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    N = 16
    P = params(N, m=1.5, a=1.2, dt=0.5, species=((-0.02, 0.02), (0.02, 0.4)))
    parts = _small_parts(5, 3000, N)
    runs = []
    for graphs in (False, True):
        r = gpu_run(P, 8000, sort_every=5, fp_bits=FPB)
        if precision == "fp32":
            r.close()
            cfg = R.make_config(N, m=P["m"], a=P["a"], dt=P["dt"], B0=P["B0"], species=P["species"], sort_every=5,
                                capacity=8000, fp_bits=FPB, precision=capi.FP32_MIXED)
            r = R.Run(cfg)
        capi.grpic_set_graphs(r.h, graphs)
        for sp, x, uc in parts:
            r.load(sp, x, uc)
        runs.append(r)
    for it in range(12):
        for r in runs:
            r.step(1)
        (xa, ua, sa), (xb, ub, sb) = runs[0].particles(), runs[1].particles()
        assert np.array_equal(sa, sb), it
        live = sa != O.DEAD
        assert np.array_equal(xa[:, live], xb[:, live]) and np.array_equal(ua[:, live], ub[:, live]), it
        for f in ("D", "B", "J"):
            assert np.array_equal(runs[0].fields(f), runs[1].fields(f)), (it, f)
        assert runs[0].diag() == runs[1].diag(), it
    for r in runs:
        r.close()


def test_deterministic_repeat():
    N = 16
    P = params(N, m=1.5, a=1.2, dt=0.5, species=((-0.02, 0.02), (0.02, 0.4)))
    parts = _small_parts(5, 3000, N)
    outs = []
    for rep in range(2):
        r = gpu_run(P, 8000, sort_every=2, fp_bits=FPB)
        for sp, x, uc in parts:
            r.load(sp, x, uc)
        r.step(5)
        outs.append((r.particles(), r.fields("D"), r.fields("B"), r.fields("J")))
        r.close()
    (pa, Da, Ba, Ja), (pb, Db, Bb, Jb) = outs
    for a, b in zip(pa, pb):
        assert np.array_equal(a, b)
    assert np.array_equal(Da, Db) and np.array_equal(Ba, Bb) and np.array_equal(Ja, Jb)


@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_gpu_gyration_closed_form(gamma_mode):
    B = 0.05
    P = params(32, m=0.0, a=0.0, dt=0.5, B0=(0.0, 0.0, B), species=((-1.0, 1.0),), gamma_mode=gamma_mode)
    r = gpu_run(P, 4)
    u3 = np.array([0.3, 0.1, 0.0])
    u4 = np.sqrt(1 + u3 @ u3)
    r.restore_particles(np.array([[16.2], [15.7], [16.1]]), np.array([[u3[0]], [u3[1]], [0.0], [u4]]),
                        np.zeros(1, np.uint8))
    nsteps = 1000
    r.push_only(nsteps)
    _, u, _ = r.particles()
    z = -1j * (-1.0) * B / u4 * 0.5
    R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    w_ref = (u3[0] + 1j * u3[1]) * R ** nsteps
    assert abs(u[0, 0] + 1j * u[1, 0] - w_ref) < 1e-13 * nsteps * abs(w_ref)


def test_gpu_schwarzschild_circular_orbit():
    m = 1.5
    P = params(64, m=m, a=0.0, dt=0.5, B0=(0.0, 0.0, 0.0), species=((0.0, 1.0),))
    r = gpu_run(P, 4)
    r0 = 15 * m
    ut = 1.0 / np.sqrt(1.0 - 3.0 * m / r0)
    Om = np.sqrt(m / r0 ** 3)
    X0 = np.array([32.0 + r0, 32.0, 32.0])
    u0 = np.array([0.0, r0 * Om * ut, 0.0, ut])
    r.restore_particles(X0.reshape(3, 1), u0.reshape(4, 1), np.zeros(1, np.uint8))
    p = O.make_params(64, m=m)
    g0, _, _ = O.metric(p, r0, 0.0, 0.0)
    ul0 = g0 @ u0
    E0, L0 = -ul0[3], r0 * ul0[1]
    r.push_only(10000)
    x, u, _ = r.particles()
    d = x[:, 0] - 32.0
    g, _, _ = O.metric(p, *d)
    ul = g @ u[:, 0]
    assert abs(-ul[3] - E0) < 1e-10 * E0
    assert abs((d[0] * ul[1] - d[1] * ul[0]) - L0) < 1e-10 * L0


def test_edge_cases():
    from paper_0904_0232_amd import capi
    N = 8
    P = params(N, m=0.5, a=0.2, dt=0.5, species=((-0.02, 0.02),))
    r = gpu_run(P, 16)
    r.step(2)  # no particles
    d = r.diag()
    assert d["n_alive"][0] == 0
    # non-finite, outside and inside-r_rm inputs are dropped
    x = np.array([[1.5, np.nan, -0.5, 4.0, 2.2], [1.5, 1.0, 1.0, 4.0, 3.3], [1.5, 1.0, 1.0, 4.0, 6.1]])
    uc = np.zeros((3, 5))
    kept = r.load(0, x, uc)
    assert kept == 2
    with pytest.raises(capi.GrpicError):
        r.load(0, np.full((3, 20), 2.0), np.zeros((3, 20)))  # capacity
    r.step(3)
    bad = capi.grpic_config_default(8)
    bad.dt = 0.9  # violates the Courant condition
    bad.capacity = 4
    with pytest.raises(capi.GrpicError):
        capi.grpic_create(bad)
