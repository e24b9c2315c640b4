"""grpic_load_particles_noalloc through the C ABI against
grpic_load_particles: two loads in a row on the same run, the second with
fewer particles, give bit-identical particle state (and the same kept
counts), in both precisions; one cycle afterwards stays identical; the
no-allocation variant makes no device allocation (counted through the run's
allocator callbacks) and refuses more particles than its staging holds."""
import numpy as np
import pytest

from common import say

pytestmark = pytest.mark.gpu


def _cfg(precision, capacity):
    from paper_0904_0232_amd import run as R
    return R.make_config(16, m=1.5, a=1.2, dt=0.5, B0=(0.0, 0.0, 0.08), species=((-0.02, 0.02), (0.02, 0.4)),
                         sort_every=0, capacity=capacity, precision=precision, fp_bits=50)


def _parts(n, seed):
    g = np.random.default_rng(seed)
    x = g.uniform(0.5, 15.5, (3, n))
    x[:, 0] = (5.0 - 1e-10, 7.0, 9.0)  # an offset that rounds to the next cell's face in FP32
    return x, g.normal(0.0, 0.1, (3, n))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_load_matches_load(precision):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    prec = capi.FP32_MIXED if precision == "fp32" else capi.FP64
    first, second = _parts(30000, 1), _parts(7000, 2)
    cap = 40000
    a = R.Run(_cfg(prec, cap))
    b = R.Run(_cfg(prec, cap))
    say("case no-alloc load", precision)
    for k, (x, uc) in enumerate((first, second)):
        ka = capi.grpic_load_particles(a.h, k, x, uc)
        calls = b.memory.alloc_calls
        kb = capi.grpic_load_particles_noalloc(b.h, k, x, uc)
        assert b.memory.alloc_calls == calls  # no device allocation in the call
        xa, ua, sa = a.particles()
        xb, ub, sb = b.particles()
        say("  call %d: %d inputs, kept %d / %d, %d slots" % (k + 1, x.shape[1], ka, kb, sb.size))
        assert ka == kb and np.array_equal(sa, sb)
        live = sa != 0xFF
        assert np.array_equal(xa[:, live], xb[:, live]) and np.array_equal(ua[:, live], ub[:, live])
    a.step(1)
    b.step(1)
    xa, ua, sa = a.particles()
    xb, ub, sb = b.particles()
    live = sa != 0xFF
    assert np.array_equal(sa, sb)
    assert np.array_equal(xa[:, live], xb[:, live]) and np.array_equal(ua[:, live], ub[:, live])
    assert np.array_equal(a.fields("J"), b.fields("J"))
    # more than the staging holds: refused on the host, nothing loaded
    big = 1 << 20
    c = R.Run(_cfg(prec, big + 8))
    with pytest.raises(capi.GrpicError) as e:
        capi.grpic_load_particles_noalloc(c.h, 0, np.full((3, big + 1), 4.0), np.zeros((3, big + 1)))
    assert e.value.code == capi.EINVAL
    assert capi.grpic_particle_count(c.h)[0] == 0
    for r in (a, b, c):
        r.close()
