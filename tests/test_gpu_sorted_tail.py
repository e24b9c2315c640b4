"""The particle kernels skip the slots past the live count that the last
cell sort left (the sort moves removed particles to the end).  Particles
loaded or restored after a sort occupy slots past that count, and every one
of them must still be pushed: the pushed-particle counter must grow by the
live count each cycle, in both precisions."""
import numpy as np
import pytest

from common import say

pytestmark = pytest.mark.gpu


def _cfg(precision):
    from paper_0904_0232_amd import run as R
    return R.make_config(16, m=1.5, a=1.2, dt=0.5, B0=(0.0, 0.0, 0.08), species=((-0.02, 0.02), (0.02, 0.4)),
                         sort_every=2, capacity=8000, precision=precision, fp_bits=50)


def _live(r):
    return int(sum(r.diag()["n_alive"]))


def _pushed_once(r):
    """One cycle; the pushed-particle counter must grow by the live count."""
    from paper_0904_0232_amd import capi
    live = _live(r)
    before = capi.grpic_particle_steps(r.h)
    r.step(1)
    return capi.grpic_particle_steps(r.h) - before, live


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_particles_placed_after_a_sort_are_pushed(precision):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    g = np.random.default_rng(11)
    r = R.Run(_cfg(capi.FP32_MIXED if precision == "fp32" else capi.FP64))
    # uniform in the grid: the ones inside the removal radius are kept as
    # removed slots at load, so the first sort leaves a removed tail
    x = g.uniform(1.0, 15.0, (3, 3000))
    r.load(0, x, g.normal(0.0, 0.1, (3, 3000)))
    r.load(1, x.copy(), g.normal(0.0, 0.02, (3, 3000)))
    r.step(2)  # the second cycle ends with a sort
    n_slots, _ = capi.grpic_particle_count(r.h)
    live = _live(r)
    say("case %s: %d slots, %d live after the sort" % (precision, n_slots, live))
    assert live < n_slots - 50  # a removed tail exists
    # a load appends past the sort's live count
    xb = g.uniform(5.0, 11.0, (3, 500))
    xb[0] = np.where(xb[0] < 8.0, xb[0] - 3.5, xb[0] + 3.5)  # outside the removal radius
    r.load(0, xb, g.normal(0.0, 0.1, (3, 500)))
    x0, u0, sp0 = r.particles()
    d, live = _pushed_once(r)
    assert d == live, (d, live)
    x1, u1, sp1 = r.particles()
    tail = np.arange(n_slots, n_slots + 500)
    moved = (sp1[tail] == 0xFF) | np.any(x1[:, tail] != x0[:, tail], axis=0)
    assert moved.all()
    # the cycle that ends with the next sort, the one after it (slots past
    # the sort's live count skipped), and a restore that puts the live
    # particles at the end of the slots
    for _ in range(2):
        d, live = _pushed_once(r)
        assert d == live, (d, live)
    x, u, sp = r.particles()
    order = np.argsort(sp != 0xFF, kind="stable")  # removed first, live last
    r.restore_particles(x[:, order], u[:, order], sp[order])
    d, live = _pushed_once(r)
    assert d == live and live > 0, (d, live)
    r.close()
