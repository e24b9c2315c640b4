"""Serving form: continuous batching of independent runs (batch C ABI and the
Python request loop).

- a run's result is the same alone and in the mix (bit for bit: every run is
  deterministic and owns its memory);
- the captured cycle graphs replayed by the batch equal eager stepping
  through grpic_step, including a cell sort between replays;
- admission respects the slot limit and the HBM budget, and queued requests
  are admitted as earlier ones finish.
"""
import numpy as np
import pytest

import oracle as O

from common import say

pytestmark = pytest.mark.gpu


def _reqs(n, seed=11, rate=50.0, steps=(10, 30), edges=(16, 32)):
    from paper_0904_0232_amd import serve
    return serve.make_requests(n, seed, rate, steps_range=steps, ppc_range=(2, 3), edges=edges)


def test_batch_graph_replay_equals_eager_steps():
    import torch
    from paper_0904_0232_amd import capi, serve
    from paper_0904_0232_amd import run as R
    req = _reqs(1, seed=3)[0]
    for nsteps in (3, 12):
        cfg = serve.request_config(req)
        parts = serve.request_particles(req)
        b = capi.grpic_batch_create(1 << 34, 4)
        rid = capi.grpic_batch_submit(b, cfg, nsteps, parts, keep_state=True)
        assert rid is not None
        it = 0
        while True:
            it += 1
            if capi.grpic_batch_step(b):
                break
        st, done, diag_b, ns, ps = capi.grpic_batch_poll(b, rid)
        assert st == capi.RUN_DONE and done == nsteps and it == nsteps
        xb, ub, spb = capi.grpic_batch_dump(b, rid, ns)
        capi.grpic_batch_destroy(b)
        # eager reference on torch's stream
        run = R.Run(serve.request_config(req))
        for s, (x, u) in enumerate(parts):
            run.load(s, x, u)
        run.step(nsteps)
        torch.cuda.synchronize()
        diag_e = run.diag()
        xe, ue, spe = run.particles()
        say("nsteps %d: batch %d slots, eager %d slots, energy %.12e vs %.12e" %
            (nsteps, ns, xe.shape[1], diag_b["energy_particles"], diag_e["energy_particles"]))
        live = spe != O.DEAD  # x and u of removed slots are unspecified
        say("   batch vs eager, live slots: max |dx| %.3e, max |du| %.3e" %
            (np.abs(xb[:, live] - xe[:, live]).max(), np.abs(ub[:, live] - ue[:, live]).max()))
        assert np.array_equal(spb, spe)
        assert np.array_equal(xb[:, live], xe[:, live]) and np.array_equal(ub[:, live], ue[:, live])
        for k in ("n_alive", "energy_particles", "lz_particles", "energy_field", "gauss_residual_max"):
            assert diag_b[k] == diag_e[k], k
        run.close()


def test_result_is_the_same_alone_and_in_the_mix():
    from paper_0904_0232_amd import serve
    reqs = _reqs(6, seed=5, rate=200.0)
    target = reqs[2]["id"]
    alone = serve.serve([dict(reqs[2], arrival=0.0)], 1 << 34, 4, keep_ids=(target,))
    mix = serve.serve(reqs, 1 << 34, 4, keep_ids=(target,))
    a, m = alone["records"][target], mix["records"][target]
    say("alone latency %.3f s, in the mix %.3f s; mix p50 %.3f p99 %.3f" %
        (a["latency"], m["latency"], mix["p50_latency_s"], mix["p99_latency_s"]))
    (xa, ua, sa), (xm, um, sm) = a["state"], m["state"]
    live = sa != O.DEAD
    assert np.array_equal(sa, sm)
    assert np.array_equal(xa[:, live], xm[:, live]) and np.array_equal(ua[:, live], um[:, live])
    assert a["diag"] == m["diag"]
    assert a["particle_steps"] == m["particle_steps"] > 0
    assert mix["n_runs"] == 6


def test_admission_by_slots_and_budget():
    from paper_0904_0232_amd import capi, serve
    reqs = _reqs(5, seed=9, rate=1000.0, steps=(5, 8), edges=(32,))
    need = max(capi.grpic_run_bytes(serve.request_config(r)) for r in reqs)
    budget = int(2.5 * need)  # room for two runs at a time
    b = capi.grpic_batch_create(budget, 8)
    ids = []
    for r in reqs:
        rid = capi.grpic_batch_submit(b, serve.request_config(r), r["steps"], serve.request_particles(r))
        ids.append(rid)
    assert ids[0] is not None and ids[1] is not None and all(i is None for i in ids[2:])
    active, used = capi.grpic_batch_stats(b)
    assert active == 2 and used <= budget
    while capi.grpic_batch_step(b) == 0:
        pass
    active, used = capi.grpic_batch_stats(b)
    assert active < 2
    capi.grpic_batch_destroy(b)
    # the loop queues the rest and admits them as memory frees up
    res = serve.serve(reqs, budget, 8)
    assert res["n_runs"] == 5
    assert all(rec["admitted"] >= rec["arrival"] - 1e-9 for rec in res["records"].values())
    say("budget-limited loop: makespan %.2f s, p50 %.3f s, p99 %.3f s" %
        (res["makespan_s"], res["p50_latency_s"], res["p99_latency_s"]))
