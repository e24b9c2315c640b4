"""Push reading ablations on the GPU (FP64), through the C ABI, against the
FP64 oracle run in the same reading:

- rk_mode PRINTED: the four RK steps of Sec. 3.3 exactly as printed (final
  weights summing to 5/6), also against its closed form on uniform-B
  gyration (the polynomial I + 5M/6 + 7M^2/24 + M^3/16 + M^4/192);
- gather_mode STEP: the field tensor gathered once at x_n for all stages;
- gather_weights SPATIAL: reading B, sub-volumes weighted by sqrt(1 + f);
- their combinations.

Tolerances as the other FP64 parity tests: 1e-12 relative per step for the
particle state, 1e-12 of scale plus the fixed-point rounding for the fields.
The FP32-mixed form rejects these modes.
"""
import numpy as np
import pytest

import oracle as O
from common import alive, gpu_run, oracle_sim, params, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-12
FPB = 50


def _parts(seed, n, N, u_th=0.1, margin=1.0):
    g = np.random.default_rng(seed)
    x = g.uniform(margin, N - margin, (3, n))
    ue = g.normal(0.0, u_th, (3, n))
    ui = g.normal(0.0, u_th / np.sqrt(20.0), (3, n))
    return [(0, x, ue), (1, x.copy(), ui)]


def _cmp_particles(s, r, tag):
    xo, uo, spo = alive(*s.particles())
    xg, ug, spg = alive(*r.particles())
    assert np.array_equal(spo, spg), tag
    ex, eu = rel_err(xg, xo, 1.0), rel_err(ug, uo, 1.0)
    say(tag, "particles", xo.shape[1], "err x %.2e u %.2e" % (ex, eu))
    assert ex < TOL and eu < TOL, (tag, ex, eu)


def _cmp_field(a, b, name, abs_floor=0.0):
    scale = max(np.abs(b).max(), 1e-300)
    err = np.abs(a - b).max()
    say(name, "err %.2e scale %.2e" % (err, scale))
    assert err <= TOL * scale + abs_floor, (name, err, scale)


@pytest.mark.parametrize("rk_mode,gather_mode,weights", [(1, 0, 0), (0, 1, 0), (1, 1, 0), (0, 0, 1), (0, 1, 1),
                                                         (1, 0, 1), (1, 1, 1)])
@pytest.mark.parametrize("gamma_mode", [0, 1])
def test_ablation_cycle_parity(rk_mode, gather_mode, weights, gamma_mode):
    N = 16
    P = params(N, m=1.5, a=1.2, dt=0.5, B0=(0.0, 0.0, 0.08), species=((-0.02, 0.02), (0.02, 0.4)),
               gamma_mode=gamma_mode, rk_mode=rk_mode, gather_mode=gather_mode, gather_weights=weights)
    say("case ablation rk %d gather %d weights %d gamma %d" % (rk_mode, gather_mode, weights, gamma_mode))
    p, s = oracle_sim(P, 4000)
    r = gpu_run(P, 4000, fp_bits=FPB)
    ko = kg = 0
    for sp, x, uc in _parts(7, 1500, N):
        ko += s.load(sp, x, uc)
        kg += r.load(sp, x, uc)
    assert ko == kg
    qmax = max(abs(q) for q, _ in P["species"])
    jfloor = 64 * 0.5 * qmax / P["dt"] * 2.0 ** -FPB
    for it in range(3):
        s.step(1)
        r.step(1)
        _cmp_particles(s, r, "step %d" % it)
        _cmp_field(r.fields("J"), s.get("J"), "J", abs_floor=jfloor)
        _cmp_field(r.fields("B"), s.get("B"), "B")
        _cmp_field(r.fields("D"), s.get("D"), "D", abs_floor=4 * np.pi * P["dt"] * jfloor)
    do, dg = s.diag(), r.diag()
    for k in ("n_alive", "n_removed_horizon", "n_removed_outer", "gamma_clamps", "flags"):
        assert do[k] == dg[k], (k, do[k], dg[k])
    r.close()


def test_printed_rk_gyration_closed_form():
    # m = 0, uniform B: u^4 is constant, so gamma = u^4/c in both readings of
    # gamma and the printed steps reduce to a polynomial in z = -i (q/m) B dt/gamma
    N = 32
    qm, B = -1.0, 0.05
    P = params(N, m=0.0, a=0.0, dt=0.5, B0=(0.0, 0.0, B), species=((qm, 1.0),), rk_mode=1)
    r = gpu_run(P, 8)
    u3 = np.array([0.3, 0.1, 0.1])
    x0 = np.array([16.2, 15.7, 12.1])
    # covariant spatial components equal the contravariant ones in flat space
    assert r.load(0, x0[:, None].copy(), u3[:, None].copy()) == 1
    nsteps = 200
    r.push_only(nsteps)
    xN, uN, _ = r.particles()
    u4 = np.sqrt(1.0 + u3 @ u3)
    h = P["dt"] / u4
    z = -1j * qm * B * h
    w, pos = u3[0] + 1j * u3[1], x0[0] + 1j * x0[1]
    for _ in range(nsteps):
        pos += h * (5 + 7 * z / 4 + 3 * z * z / 8 + z ** 3 / 32) / 6 * w
        w *= 1 + 5 * z / 6 + 7 * z * z / 24 + z ** 3 / 16 + z ** 4 / 192
    say("printed RK gyration: u err %.2e x err %.2e" % (abs(uN[0, 0] + 1j * uN[1, 0] - w),
                                                          abs(xN[0, 0] + 1j * xN[1, 0] - pos)))
    assert abs(uN[0, 0] + 1j * uN[1, 0] - w) < 1e-13 * nsteps * abs(w)
    assert abs(xN[0, 0] + 1j * xN[1, 0] - pos) < 1e-13 * nsteps * abs(pos)
    assert abs(xN[2, 0] - (x0[2] + nsteps * (5.0 / 6.0) * u3[2] / u4 * P["dt"])) < 1e-11
    r.close()


@pytest.mark.parametrize("rk_mode,gather_mode,weights", [(1, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_fp32_mixed_rejects_ablations(rk_mode, gather_mode, weights):
    from paper_0904_0232_amd import capi
    from paper_0904_0232_amd import run as R
    cfg = R.make_config(16, m=1.5, a=1.2, dt=0.5, capacity=64, precision=capi.FP32_MIXED,
                        rk_mode=rk_mode, gather_mode=gather_mode, gather_weights=weights)
    with pytest.raises(capi.GrpicError) as e:
        R.Run(cfg)
    assert e.value.code == capi.EINVAL
