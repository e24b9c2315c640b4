"""Checkpoint and resume through the C ABI (grpic_save_state /
grpic_load_state): a run created with the same configuration that loads a
saved state continues bit-identically to the run that saved it (particles,
fields, current, diagnostics, counters, sort schedule), in both precisions;
malformed or mismatched states are rejected with GRPIC_EINVAL and leave the
run unchanged."""
import numpy as np
import pytest

from common import say

pytestmark = pytest.mark.gpu


def _cfg(precision, n=16, capacity=6000, sort_every=3):
    from paper_0904_0232_amd import run as R
    return R.make_config(n, m=1.5, a=1.2, dt=0.5, B0=(0.0, 0.0, 0.08), species=((-0.02, 0.02), (0.02, 0.4)),
                         sort_every=sort_every, capacity=capacity, precision=precision, fp_bits=50)


def _parts(N, n=2000, seed=5):
    g = np.random.default_rng(seed)
    x = g.uniform(1.0, N - 1.0, (3, n))
    # a few particles 1e-10 below a cell face: the FP32-mixed form rounds
    # their offset to the next cell's face, which a checkpoint must keep
    x[:, :4] = np.array([[5.0, 9.0, 11.0, 3.0], [7.0, 6.5, 12.0, 4.0], [9.0, 10.0, 3.5, 13.0]]) - 1e-10
    return [(0, x, g.normal(0.0, 0.1, (3, n))), (1, x.copy(), g.normal(0.0, 0.02, (3, n)))]


def _snapshot(r):
    from paper_0904_0232_amd import capi
    x, u, sp = r.particles()
    live = sp != 0xFF
    return {"sp": sp, "x": x[:, live], "u": u[:, live], "D": r.fields("D"), "B": r.fields("B"),
            "J": r.fields("J"), "diag": r.diag(), "steps": capi.grpic_particle_steps(r.h)}


def _same(a, b):
    assert np.array_equal(a["sp"], b["sp"])
    for k in ("x", "u", "D", "B", "J"):
        assert np.array_equal(a[k], b[k]), k
    assert a["steps"] == b["steps"]
    for k, v in a["diag"].items():
        assert v == b["diag"][k], (k, v, b["diag"][k])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_resume_is_bit_identical(precision):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    prec = capi.FP32_MIXED if precision == "fp32" else capi.FP64
    say("case checkpoint", precision)
    a = R.Run(_cfg(prec))
    for sp, x, uc in _parts(16):
        a.load(sp, x, uc)
    a.step(4)  # one sort behind it, the next one due in two cycles
    state = a.save_state()
    a.step(5)
    ref = _snapshot(a)
    a.close()
    b = R.Run(_cfg(prec, capacity=9000))  # capacity may differ
    b.load_state(state)
    b.step(5)
    got = _snapshot(b)
    b.close()
    say("  resumed: %d live, state %d bytes" % (got["x"].shape[1], state.size))
    _same(ref, got)


def test_rejects_malformed_or_mismatched_states():
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    a = R.Run(_cfg(capi.FP64))
    for sp, x, uc in _parts(16):
        a.load(sp, x, uc)
    a.step(2)
    state = a.save_state()
    before = _snapshot(a)

    def rejected(run, st):
        with pytest.raises(capi.GrpicError) as e:
            run.load_state(st)
        assert e.value.code == capi.EINVAL

    rejected(a, state[:-8])                       # short
    bad = state.copy()
    bad[0] ^= 0xFF                                # not a state
    rejected(a, bad)
    _same(before, _snapshot(a))                   # unchanged
    other = R.Run(_cfg(capi.FP64, n=20))          # different grid
    rejected(other, state)
    other.close()
    small = R.Run(_cfg(capi.FP64, capacity=100))  # too many slots
    rejected(small, state)
    small.close()
    mixed = R.Run(_cfg(capi.FP32_MIXED))          # different precision
    rejected(mixed, state)
    mixed.close()
    a.close()
