"""One full cycle of the jet workload (the paper's application: 64 x 64 x
128, c = 0.05, dt = 1, B^z = 30, electrons and positrons, disk + corona) on
the GPU (FP64, through the C ABI) against the oracle, for a sample of the
inputs both sides load.  Tolerances as the other FP64 parity tests."""
import numpy as np
import pytest

import oracle as O
from common import alive, rel_err, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

PER_SPECIES = 50000


def test_jet_one_cycle_parity():
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R
    w = inputs.jet_params()
    parts = inputs.jet_particles(0)
    g = np.random.default_rng(3)
    pick = np.sort(g.choice(parts[0][1].shape[1], PER_SPECIES, replace=False))
    sub = [(sp, x[:, pick], u[:, pick]) for sp, x, u in parts]
    n = 2 * PER_SPECIES
    p = O.make_params(w["nx"], w["ny"], w["nz"], c=w["c"], dt=w["dt"], m=w["m"], a=w["a"], center=w["center"],
                      r_rm=w["r_rm"], species=w["species"])
    s = O.Sim(p, n)
    s.init_fields([0.0, 0.0, w["B0"]])
    cfg = R.make_config(w["nx"], ny=w["ny"], nz=w["nz"], m=w["m"], a=w["a"], c=w["c"], dt=w["dt"],
                        B0=(0.0, 0.0, w["B0"]), species=w["species"], r_rm=w["r_rm"], capacity=n, fp_bits=50,
                        center=w["center"], precision=capi.FP64)
    r = R.Run(cfg)
    ko = sum(s.load(sp, x, u) for sp, x, u in sub)
    kg = sum(r.load(sp, x, u) for sp, x, u in sub)
    assert ko == kg
    say("jet sample: %d loaded" % kg)
    s.step(1)
    r.step(1)
    xo, uo, spo = alive(*s.particles())
    xg, ug, spg = alive(*r.particles())
    assert np.array_equal(spo, spg)
    ex, eu = rel_err(xg, xo, 1.0), rel_err(ug, uo, w["c"])
    say("jet cycle: particles err x %.2e u %.2e" % (ex, eu))
    assert ex < 1e-12 and eu < 1e-12
    qmax = abs(w["species"][0][0])
    jfloor = 64 * 0.5 * qmax / w["dt"] * 2.0 ** -50
    for name, floor in (("J", jfloor), ("B", 0.0), ("D", 4 * np.pi * w["dt"] / w["c"] * jfloor)):
        a_, b_ = r.fields(name), s.get(name)
        err, scale = np.abs(a_ - b_).max(), np.abs(b_).max()
        say("jet cycle: %s err %.2e scale %.2e" % (name, err, scale))
        assert err <= 1e-12 * scale + floor, name
    r.close()
