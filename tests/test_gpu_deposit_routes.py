"""The two routes of the current deposition (Sec. 4: FLUX^K times the
face-area weights, int64 fixed point), element by element against the FP64
oracle, in both precisions.

A deposit block takes 1024 consecutive particle slots.  When the edges they
touch fit a small box (particles in cell order), the block sums its current
in an LDS box and flushes it once with global atomics; otherwise it adds to
the global sums directly.  The device counts the blocks of each route
(grpic_diag.deposit_blocks_lds / _global), so each case proves which route
it ran:

- cell order: the uniform plasma of a 32^3 Kerr grid at 8 particles per cell
  and species in generation order (cell by cell, x fastest): every block
  covers four rows of cells, so every block takes the LDS route;
- random order: the same particles shuffled, so every block spans the grid
  and takes the global route;
- mixed: the first half of each species in cell order, the rest shuffled.

Both routes add the same integers, so J, D and B must be bit-identical in
the three orders (and the particles, up to the permutation).  The cell-order
run is compared with the oracle node by node: FP64 within 1e-12 of the
field's scale plus the fixed-point rounding, FP32-mixed within 1e-5 (L2 for
J; the max norm is printed).

The fixed-point range check: with fp_bits = 50 and tens of thousands of
particles moving together through one cell, an edge's int64 sum leaves the
int64 range; the device raises flags bit 1, grpic_diagnostics and then
grpic_step return GRPIC_EOVERFLOW.  A thousand such particles stay in range.
"""
import numpy as np
import pytest

from common import alive, oracle_sim, params, rel_err, say

pytestmark = pytest.mark.gpu

N = 32
PPC = 8
STEPS = 2
FPB = 44


def _params():
    from paper_0904_0232_amd import inputs
    return params(N, m=1.5, a=1.2, dt=0.45, B0=(0.0, 0.0, 0.1), species=inputs.species_table(0.45, PPC))


_cache = {}


def _inputs():
    from paper_0904_0232_amd import inputs
    if "parts" not in _cache:
        _cache["parts"] = inputs.uniform_plasma(3, N, N, N, PPC, 0.1)
    return _cache["parts"]


def _orders():
    """Per species, the slot order of each case (indices into the inputs)."""
    n = _inputs()[0][1].shape[1]
    g = np.random.default_rng(21)
    half = n // 2
    out = {"cell": [np.arange(n), np.arange(n)],
           "random": [g.permutation(n), g.permutation(n)],
           "mixed": [np.concatenate([np.arange(half), half + g.permutation(n - half)]) for _ in range(2)]}
    return out


def _oracle():
    """The oracle on the inputs in cell order: J after each step, final
    particles, B and D."""
    if "oracle" not in _cache:
        P = _params()
        parts = _inputs()
        p, s = oracle_sim(P, sum(x.shape[1] for _, x, _ in parts))
        for sp, x, uc in parts:
            s.load(sp, x, uc)
        Js = []
        for _ in range(STEPS):
            s.step(1)
            Js.append(s.get("J"))
        _cache["oracle"] = dict(J=Js, B=s.get("B"), D=s.get("D"), particles=s.particles())
    return _cache["oracle"]


def _gpu(precision, order):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    P = _params()
    parts = _inputs()
    ntot = sum(x.shape[1] for _, x, _ in parts)
    cfg = R.make_config(N, m=P["m"], a=P["a"], dt=P["dt"], B0=P["B0"], species=P["species"], sort_every=0,
                        capacity=ntot, fp_bits=FPB,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    r = R.Run(cfg)
    for (sp, x, uc), perm in zip(parts, order):
        r.load(sp, x[:, perm], uc[:, perm])
    Js = []
    for _ in range(STEPS):
        r.step(1)
        Js.append(r.fields("J"))
    d = r.diag()
    out = dict(J=Js, B=r.fields("B"), D=r.fields("D"), particles=r.particles(), diag=d)
    r.close()
    return out


def _j_floor(P, ncontrib=256):
    qmax = max(abs(q) for q, _ in P["species"])
    return ncontrib * 0.5 * qmax / P["dt"] * 2.0 ** -FPB


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_deposit_routes_against_oracle(precision):
    P = _params()
    orders = _orders()
    runs = {}
    for name, order in orders.items():
        say("case deposit routes %s, %s order" % (precision, name))
        runs[name] = _gpu(precision, order)
        d = runs[name]["diag"]
        say("  blocks: %d on the LDS route, %d on the global route" %
            (d["deposit_blocks_lds"], d["deposit_blocks_global"]))
    # which route ran
    assert runs["cell"]["diag"]["deposit_blocks_global"] == 0 and runs["cell"]["diag"]["deposit_blocks_lds"] > 0
    assert runs["random"]["diag"]["deposit_blocks_lds"] == 0 and runs["random"]["diag"]["deposit_blocks_global"] > 0
    assert runs["mixed"]["diag"]["deposit_blocks_lds"] > 0 and runs["mixed"]["diag"]["deposit_blocks_global"] > 0
    # the push's node box: staged in LDS for cell-ordered blocks (one row of
    # 32 cells: 132 nodes, which the first cycle's drift can take past the
    # 272-node budget), global gathers for blocks spread over the grid
    for name in ("cell", "random"):
        say("  push blocks (%s): %d with an LDS node box, %d without" %
            (name, runs[name]["diag"]["push_blocks_lds"], runs[name]["diag"]["push_blocks_global"]))
    assert runs["cell"]["diag"]["push_blocks_lds"] > 0
    assert runs["random"]["diag"]["push_blocks_lds"] == 0 and runs["random"]["diag"]["push_blocks_global"] > 0
    # order independence: the same integers on either route
    ref = runs["cell"]
    n = _inputs()[0][1].shape[1]
    for name in ("random", "mixed"):
        got = runs[name]
        for k in range(STEPS):
            assert np.array_equal(got["J"][k], ref["J"][k]), (name, k)
        assert np.array_equal(got["B"], ref["B"]) and np.array_equal(got["D"], ref["D"]), name
        # particles: slot i of this order holds input orders[name][sp][i]
        slot = np.concatenate([o + s * n for s, o in enumerate(orders[name])])
        inv = np.empty_like(slot)
        inv[slot] = np.arange(slot.size)
        (xr, ur, sr), (xg, ug, sg) = ref["particles"], got["particles"]
        assert np.array_equal(sg[inv], sr), name
        live = sr != 0xFF
        assert np.array_equal(xg[:, inv][:, live], xr[:, live]) and np.array_equal(ug[:, inv][:, live], ur[:, live])
    # the cell-order run against the oracle, node by node
    o = _oracle()
    for k in range(STEPS):
        Jo, Jg = o["J"][k], ref["J"][k]
        err = np.abs(Jg - Jo).max()
        scale = np.abs(Jo).max()
        l2 = np.linalg.norm(Jg - Jo) / np.linalg.norm(Jo)
        say("  step %d: J max err %.2e of scale %.2e, L2 %.2e" % (k + 1, err, scale, l2))
        if precision == "fp64":
            assert err <= 1e-12 * scale + _j_floor(P), k
        else:
            assert l2 < 1e-5, k
    eB = np.abs(ref["B"] - o["B"]).max() / np.abs(o["B"]).max()
    eD = np.abs(ref["D"] - o["D"]).max()
    Dscale = np.abs(o["D"]).max()
    xo, uo, so = alive(*o["particles"])
    xg, ug, sg = alive(*ref["particles"])
    assert np.array_equal(so, sg)
    ex, eu = rel_err(xg, xo, 1.0), rel_err(ug, uo, 1.0)
    say("  B err %.2e, D err %.2e of %.2e, particles x %.2e u %.2e (%d live)" % (eB, eD, Dscale, ex, eu, so.size))
    if precision == "fp64":
        assert eB < 1e-12 and ex < 1e-12 and eu < 1e-12
        assert eD <= 1e-12 * Dscale + 4 * np.pi * P["dt"] * _j_floor(P) * STEPS
    else:
        eD2 = np.linalg.norm(ref["D"] - o["D"]) / np.linalg.norm(o["D"])
        say("  D L2 err %.2e" % eD2)
        assert eB < 1e-5 and ex < 1e-5 and eu < 1e-5 and eD2 < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fixed_point_overflow_is_reported(precision):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    say("case fixed-point range", precision)
    results = {}
    for count in (1000, 40000):
        cfg = R.make_config(8, m=0.0, a=0.0, dt=0.5, B0=(0.0, 0.0, 0.0), species=((-1.0, 1.0),), sort_every=0,
                            capacity=count, fp_bits=50,
                            precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
        r = R.Run(cfg)
        # every particle at the same point of one cell, moving along x at
        # 0.89 c: each adds about 2^48.5 to the same x-edge per step
        x = np.tile(np.array([[3.1], [3.1], [3.1]]), (1, count))
        uc = np.tile(np.array([[2.0], [0.0], [0.0]]), (1, count))
        assert r.load(0, x, uc) == count
        r.step(1)
        d = r.diag(allow_overflow=True)
        say("  %d particles: flags %d" % (count, d["flags"]))
        results[count] = d["flags"]
        if count > 1000:
            with pytest.raises(capi.GrpicError) as e:
                r.diag()
            assert e.value.code == capi.EOVERFLOW
            with pytest.raises(capi.GrpicError) as e:
                r.step(1)
            assert e.value.code == capi.EOVERFLOW
        r.close()
    assert results[1000] & 2 == 0
    assert results[40000] & 2 == 2
