"""Parity at the full sizes of the torus (128^3, 33,554,432 particles) and
throughput (256^3, 268,435,456 particles) workloads, in the launch
configuration the benchmark times, in both precisions.

The oracle cannot redo a whole 256^3 cycle in seconds, so the full-size runs
are pinned two ways:

- sampled particles, one test-particle step (the node tensor of the initial
  fields, as grpic_push_only uses): the oracle runs on a 20^3 window of the
  big grid, placed by giving it the hole centre in window coordinates, and
  loads the sampled inputs itself; the initial fields and their node tensor
  are local, so the window's interior reproduces the big grid's exactly.
  Windows sit near the hole, in the bulk of the plasma and further out;
- one full cycle from the same state: the total current per direction
  equals sum q dx / dt over the particles' own moves (true for any
  transverse weights, at any size).

Tolerances: FP64 1e-12 relative per step (as the other parity tests);
FP32-mixed 1e-5 relative against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O
from common import rel_err, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

W = 20          # window edge in cells
MARGIN = 3      # sampled particles start and end this far inside the window
PER_WINDOW = 1500

_inputs = {}


def _workload(name):
    from paper_0904_0232_amd import inputs
    if name not in _inputs:
        _inputs.clear()
        say("generating the %s inputs" % name)
        _inputs[name] = inputs.workload_particles(name, seed=0)
    return inputs.workload_params(name), _inputs[name]


def _run(w, ntot, precision):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=0, capacity=ntot,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    return R.Run(cfg)


def _windows(w):
    """Window origins: centred at R = r_+ + 5, in the bulk and further out
    (torus: R = 24 and 34 in the equatorial plane, where its particles are;
    uniform plasmas: n/4 and 0.4 n), along x, y and a third direction."""
    n, c0 = w["n"], w["n"] / 2.0
    if w["plasma"] == "torus":
        far = ((24.0, (0.0, 1.0, 0.0)), (34.0, (-1.0, -1.0, 0.0)))
    else:
        far = ((n / 4.0, (0.0, 1.0, 0.0)), (0.4 * n, (1.0, 1.0, 1.0)))
    out = []
    for R, d in ((w["r_plus"] + 5.0, (1.0, 0.0, 0.0)),) + far:
        d = np.array(d) / np.linalg.norm(d)
        cen = c0 + R * d
        out.append(np.floor(cen - W / 2.0).astype(int))
    return out


@pytest.mark.parametrize("name,precision", [("torus128", "fp64"), ("torus128", "fp32"),
                                            ("shell256", "fp64"), ("shell256", "fp32")])
def test_full_size(name, precision):
    w, parts = _workload(name)
    ntot = sum(p[1].shape[1] for p in parts)
    say("case %s %s: %d particles, %d^3 grid" % (name, precision, ntot, w["n"]))
    r = _run(w, ntot, precision)
    kept = sum(r.load(sp, x, uc) for sp, x, uc in parts)
    x0, u0, sp0 = r.particles()
    say("  loaded %d live of %d" % (kept, ntot))
    live = sp0 != O.DEAD

    # sampled test-particle step against oracle windows
    r.push_only(1)
    x1, u1, _ = r.particles()
    tol = 1e-12 if precision == "fp64" else 1e-5
    g = np.random.default_rng(7)
    offs = np.cumsum([0] + [p[1].shape[1] for p in parts])
    for o in _windows(w):
        inside = live.copy()
        for ax in range(3):
            lo, hi = o[ax] + MARGIN, o[ax] + W - MARGIN
            inside &= (x0[ax] >= lo) & (x0[ax] < hi) & (x1[ax] >= lo) & (x1[ax] < hi)
        idx = np.nonzero(inside)[0]
        assert idx.size > 0, ("empty window", o)
        pick = np.sort(g.choice(idx, min(PER_WINDOW, idx.size), replace=False))
        cen = tuple(w["n"] / 2.0 - o)
        p = O.make_params(W, m=w["m"], a=w["a"], dt=w["dt"], center=cen, r_rm=w["r_rm"],
                          species=w["species"])
        s = O.Sim(p, pick.size)
        s.init_fields([0.0, 0.0, w["B0"]])
        s.compute_nodes()
        # the oracle loads the picked inputs itself (window coordinates)
        kept = 0
        for (spc, x, uc), a, b in zip(parts, offs[:-1], offs[1:]):
            k = pick[(pick >= a) & (pick < b)] - a
            kept += s.load(spc, x[:, k] - o[:, None], uc[:, k])
        assert kept == pick.size
        s.push_only(1)
        xs, us, _ = s.particles()
        ex = rel_err(x1[:, pick] - o[:, None], xs, 1.0)
        eu = rel_err(u1[:, pick], us, 1.0)
        Rw = np.linalg.norm(o + W / 2.0 - w["n"] / 2.0)
        say("  window at R=%.1f: %d particles, push err x %.2e u %.2e" % (Rw, pick.size, ex, eu))
        assert ex < tol and eu < tol
    del x1, u1

    # one full cycle from the loaded state: total current per direction
    r.restore_particles(x0, u0, sp0)
    del u0
    r.step(1)
    x1, _, _ = r.particles()
    J = r.fields("J")
    qs = np.array([q for q, _ in w["species"]])
    qlive = qs[sp0[live]]
    jtol = 1e-12 if precision == "fp64" else 1e-6
    for K in range(3):
        ref = float((qlive * (x1[K, live] - x0[K, live])).sum()) / w["dt"]
        floor = live.sum() * 24 * 0.5 * np.abs(qs).max() / w["dt"] * 2.0 ** -44
        got = float(J[K].sum())
        say("  full cycle: sum J_%d %.6e, sum q dx/dt %.6e" % (K, got, ref))
        assert abs(got - ref) <= jtol * float(np.abs(J[K]).sum()) + floor, K
    r.close()


WE = 40      # evolved-state window edge in cells
INNER = 12   # compared this far inside it (deeper than one cycle's field dependencies reach)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shell256_windows_from_an_evolved_state(precision):
    """The 256^3 shell workload in the benchmark's launch configuration
    (a cell sort after loading, then every 8 cycles, on 4^3 tiles), from a
    state the GPU evolved for 10 cycles: three 40^3 windows of the GPU's D, B and particles (near
    the hole, in the bulk, further out) are handed to the oracle, and both
    advance one cycle.  A window's outer layers are frozen at the reference
    state in the oracle, so only what lies at least 12 cells inside is
    compared: the particles that start and end there (FP64 1e-12, FP32-mixed
    1e-5), and in FP64 also J, B and D at those points."""
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    w, parts = _workload("shell256")
    ntot = sum(p[1].shape[1] for p in parts)
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=8, capacity=ntot,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    r = R.Run(cfg)
    for sp, x, uc in parts:
        r.load(sp, x, uc)
    r.sort(outputs=False)
    say("case shell256 %s: 10 cycles" % precision)
    r.step(10)
    x0, u0, sp0 = r.particles()
    D0, B0 = r.fields("D"), r.fields("B")
    r.step(1)
    x1, u1, sp1 = r.particles()
    J1, Bg, Dg = r.fields("J"), r.fields("B"), r.fields("D")
    r.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    n, c0 = w["n"], w["n"] / 2.0
    qmax = max(abs(q) for q, _ in w["species"])
    jfloor = 256 * 0.5 * qmax / w["dt"] * 2.0 ** -44
    for R_, d in ((w["r_plus"] + 14.0, (1.0, 0.0, 0.0)), (n / 4.0, (0.0, 1.0, 0.0)), (0.4 * n, (1.0, 1.0, 1.0))):
        d = np.array(d) / np.linalg.norm(d)
        o = np.floor(c0 + R_ * d - WE / 2.0).astype(int)
        assert (o >= 0).all() and (o + WE <= n).all()
        live = sp0 != O.DEAD
        inw = live & np.all((x0 >= o[:, None]) & (x0 < (o + WE)[:, None]), axis=0)
        idx = np.nonzero(inw)[0]
        p = O.make_params(WE, m=w["m"], a=w["a"], dt=w["dt"], center=tuple(c0 - o), r_rm=w["r_rm"],
                          species=w["species"])
        s = O.Sim(p, idx.size)
        s.init_fields([0.0, 0.0, w["B0"]])
        cut = (slice(None), slice(o[2], o[2] + WE + 3), slice(o[1], o[1] + WE + 3), slice(o[0], o[0] + WE + 3))
        s.set_fields(D0[cut], B0[cut])
        s.set_particles(x0[:, idx] - o[:, None], u0[:, idx], sp0[idx])
        s.step(1)
        xs, us, ss = s.particles()
        lo, hi = INNER, WE - INNER
        xw0 = x0[:, idx] - o[:, None]
        xw1 = x1[:, idx] - o[:, None]
        keep = (ss != O.DEAD) & (sp1[idx] != O.DEAD)
        keep &= np.all((xw0 >= lo) & (xw0 < hi) & (xw1 >= lo) & (xw1 < hi), axis=0)
        assert np.array_equal(ss[keep], sp1[idx][keep])
        ex = rel_err(xw1[:, keep], xs[:, keep], 1.0)
        eu = rel_err(u1[:, idx][:, keep], us[:, keep], 1.0)
        say("  window at R=%.0f: %d particles in it, %d compared: x %.2e u %.2e" % (R_, idx.size, keep.sum(), ex, eu))
        assert keep.sum() > 10000 and ex < tol and eu < tol
        inner = (slice(None), slice(lo + 1, hi + 1), slice(lo + 1, hi + 1), slice(lo + 1, hi + 1))
        win = (slice(None), slice(o[2] + lo + 1, o[2] + hi + 1), slice(o[1] + lo + 1, o[1] + hi + 1),
               slice(o[0] + lo + 1, o[0] + hi + 1))
        eB = np.abs(Bg[win] - s.get("B")[inner]).max() / np.abs(Bg[win]).max()
        say("    B err %.2e" % eB)
        assert eB < tol
        if precision == "fp64":
            Jo, Do = s.get("J")[inner], s.get("D")[inner]
            eJ = np.abs(J1[win] - Jo).max()
            eD = np.abs(Dg[win] - Do).max()
            say("    J err %.2e of %.2e, D err %.2e of %.2e" % (eJ, np.abs(Jo).max(), eD, np.abs(Do).max()))
            assert eJ <= 1e-12 * np.abs(Jo).max() + jfloor
            assert eD <= 1e-12 * np.abs(Do).max() + 4 * np.pi * w["dt"] * jfloor
        del s
