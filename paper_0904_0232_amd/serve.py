"""Continuous-batching request loop for independent GRPIC runs.

Requests (the serving workload: grid edge in {16, 32, 48, 64, 96}, spin
a ~ U[0, 0.99] m with m = edge/16, 2-8 particles per cell and species,
u_th ~ U[0.02, 0.2] c, 50-500 steps, FP32-mixed) arrive as a Poisson
process.  The loop admits arrived requests first-come-first-served whenever
the batch has a free slot and HBM budget (``grpic_batch_submit``), advances
every admitted run by one cycle per iteration (``grpic_batch_step``: one
replay of the captured graph of batched launches, each stage covering all
active runs), and records each request's completion latency (arrival ->
finished).  The initial particles of queued requests are generated on host
threads ahead of admission; while runs are stepping, a request whose
particles are not ready yet waits for a later iteration instead of holding
up the device.

Requests may be urgent (priority 1).  Urgent requests are admitted before
everything else; with preemption on, an urgent request that does not fit
preempts normal runs (``grpic_batch_preempt``: state saved to host memory,
slot and memory freed), the smallest first, until it fits.  Preempted runs resume (``grpic_batch_resume``) before new normal
requests are admitted, and finish exactly as if never preempted.
"""
import collections
import itertools
import math
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import capi, inputs
from . import run as R

EDGES = (16, 32, 48, 64, 96)
DT = 0.45
B0 = 0.1


def make_requests(n_runs, seed, rate, steps_range=(50, 500), ppc_range=(2, 8), edges=EDGES, urgent_frac=0.0):
    """Seeded request list; arrival times of a Poisson process of `rate` per
    second; a fraction urgent_frac of the requests is urgent (drawn from a
    stream of its own, so the requests themselves do not change with it)."""
    g = inputs.rng(seed, 7)
    gp = inputs.rng(seed, 8)
    t = 0.0
    reqs = []
    for i in range(n_runs):
        t += g.exponential(1.0 / rate)
        edge = int(edges[g.integers(len(edges))])
        m = edge / 16.0
        reqs.append(dict(
            id=i, arrival=t, edge=edge, m=m, a=float(g.uniform(0.0, 0.99)) * m,
            ppc=int(g.integers(ppc_range[0], ppc_range[1] + 1)),
            steps=int(g.integers(steps_range[0], steps_range[1] + 1)),
            u_th=float(g.uniform(0.02, 0.2)), seed=int(seed) * 100003 + i,
            priority=int(gp.uniform() < urgent_frac)))
    return reqs


def request_config(req):
    n = req["edge"]
    species = inputs.species_table(DT, req["ppc"])
    return R.make_config(n, m=req["m"], a=req["a"], dt=DT, B0=(0.0, 0.0, B0), species=species,
                         sort_every=10, capacity=2 * req["ppc"] * n ** 3, precision=capi.FP32_MIXED)


def request_particles(req):
    n = req["edge"]
    parts = inputs.uniform_plasma(req["seed"], n, n, n, req["ppc"], req["u_th"])
    return [(x, u) for _, x, u in parts]


def percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else float("nan")


def serve(requests, budget_bytes, max_slots, keep_ids=(), prefetch=8, log=None, preempt=False):
    """Run the request loop to completion.  Returns per-request records and totals."""
    b = capi.grpic_batch_create(budget_bytes, max_slots)
    pool = ThreadPoolExecutor(max_workers=prefetch)
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    waiting = collections.deque()   # arrived, not admitted (urgent ones first)
    parked = collections.deque()    # preempted runs: (run id, request, state)
    futures = {}
    active = {}
    records = {}
    n_preempted = 0

    def nbytes(r):
        return capi.grpic_run_bytes(request_config(r))

    def make_room(r):
        # preempt normal runs until the urgent request r fits, the cheapest
        # first (fewest device bytes: the save copies them to the host and
        # stalls the loop meanwhile), among equals the one with the most
        # cycles left; nothing is preempted when r would not fit beside the
        # urgent runs alone
        nonlocal n_preempted
        urgent_runs = [q for q in active.values() if q.get("priority", 0)]
        if len(urgent_runs) >= max_slots or sum(map(nbytes, urgent_runs)) + nbytes(r) > budget_bytes:
            return
        while True:
            n_active, used = capi.grpic_batch_stats(b)
            if n_active < max_slots and used + nbytes(r) <= budget_bytes:
                return
            left = {rid: q["steps"] - capi.grpic_batch_poll(b, rid)[1]
                    for rid, q in active.items() if not q.get("priority", 0)}
            if not left:
                return
            victim = min(left, key=lambda rid: (nbytes(active[rid]), -left[rid], rid))
            q = active.pop(victim)
            parked.append((victim, q, capi.grpic_batch_preempt(b, victim)))
            records[q["id"]]["preemptions"] += 1
            n_preempted += 1
            if log:
                log("run %d preempted with %d cycles left" % (q["id"], left[victim]))
    for r in requests:
        cfg = request_config(r)
        if capi.grpic_run_bytes(cfg) > budget_bytes:
            raise ValueError("request %d needs more than the whole HBM budget" % r["id"])
    t0 = time.perf_counter()
    total_psteps = 0
    iterations = 0
    t_inputs = t_submit = t_step = 0.0  # host time waiting for inputs, admitting, stepping
    try:
        while pending or waiting or active or parked:
            now = time.perf_counter() - t0
            while pending and pending[0]["arrival"] <= now:
                r = pending.popleft()
                if r.get("priority", 0):
                    # behind the urgent requests already waiting
                    k = sum(1 for q in waiting if q.get("priority", 0))
                    waiting.insert(k, r)
                else:
                    waiting.append(r)
            # a request carries its particles: the payloads of the next few
            # requests in arrival order are drawn ahead on host threads, so
            # they are ready when the requests arrive
            for q in itertools.islice(itertools.chain(waiting, pending), prefetch):
                if q["id"] not in futures:
                    futures[q["id"]] = pool.submit(request_particles, q)
            while waiting or parked:
                urgent = bool(waiting) and bool(waiting[0].get("priority", 0))
                if parked and not urgent:
                    # preempted runs go before new normal requests
                    rid, q, state = parked[0]
                    ta = time.perf_counter()
                    ok = capi.grpic_batch_resume(b, rid, state)
                    t_submit += time.perf_counter() - ta
                    if not ok:
                        break
                    parked.popleft()
                    active[rid] = q
                    continue
                for q in itertools.islice(itertools.chain(waiting, pending), prefetch):
                    if q["id"] not in futures:
                        futures[q["id"]] = pool.submit(request_particles, q)
                r = waiting[0]
                if active and not futures[r["id"]].done():
                    # the payload is still being drawn: step the active runs
                    # meanwhile instead of leaving the device idle
                    break
                if urgent and preempt:
                    make_room(r)
                ta = time.perf_counter()
                parts = futures[r["id"]].result()
                tb = time.perf_counter()
                rid = capi.grpic_batch_submit(b, request_config(r), r["steps"], parts,
                                              keep_state=r["id"] in keep_ids)
                t_inputs += tb - ta
                t_submit += time.perf_counter() - tb
                if rid is None:
                    break
                waiting.popleft()
                del futures[r["id"]]
                active[rid] = r
                records[r["id"]] = dict(r, admitted=time.perf_counter() - t0, preemptions=0)
            if active:
                ta = time.perf_counter()
                fin = capi.grpic_batch_step(b)
                t_step += time.perf_counter() - ta
                iterations += 1
                if fin:
                    tnow = time.perf_counter() - t0
                    for rid in list(active):
                        st, done, diag, nslots, ps = capi.grpic_batch_poll(b, rid)
                        if st == capi.RUN_DONE:
                            r = active.pop(rid)
                            rec = records[r["id"]]
                            rec.update(finished=tnow, latency=tnow - r["arrival"], diag=diag, particle_steps=ps)
                            total_psteps += ps
                            if r["id"] in keep_ids:
                                rec["state"] = capi.grpic_batch_dump(b, rid, nslots)
                            capi.grpic_batch_release(b, rid)
                            if log:
                                log("run %d done: edge %d, %d steps, latency %.2f s" %
                                    (r["id"], r["edge"], r["steps"], rec["latency"]))
            elif pending:
                time.sleep(max(0.0, min(0.05, pending[0]["arrival"] - (time.perf_counter() - t0))))
        makespan = time.perf_counter() - t0
    finally:
        pool.shutdown(wait=False)
        capi.grpic_batch_destroy(b)
    lat = [rec["latency"] for rec in records.values()]
    lat_u = [rec["latency"] for rec in records.values() if rec.get("priority", 0)]
    lat_n = [rec["latency"] for rec in records.values() if not rec.get("priority", 0)]
    return {
        "records": records,
        "n_runs": len(records),
        "makespan_s": makespan,
        "iterations": iterations,
        "p50_latency_s": percentile(lat, 50),
        "p99_latency_s": percentile(lat, 99),
        "urgent": {"n": len(lat_u), "p50_latency_s": percentile(lat_u, 50), "p99_latency_s": percentile(lat_u, 99)},
        "normal": {"n": len(lat_n), "p50_latency_s": percentile(lat_n, 50), "p99_latency_s": percentile(lat_n, 99)},
        "preemptions": n_preempted,
        "particle_steps": total_psteps,
        "particle_steps_per_s": total_psteps / makespan if makespan > 0 else 0.0,
        "runs_per_s": len(records) / makespan if makespan > 0 else 0.0,
        "host_s": {"waiting_for_inputs": t_inputs, "admitting": t_submit, "stepping": t_step},
    }


def one_by_one(requests):
    """The same requests run alone, one after another, each as a single run
    (``grpic_create``/``grpic_load_particles``/``grpic_step`` with its cycle
    replayed as a captured graph), the reference for the batch's throughput.
    The particles are drawn before the clock starts; each run's time covers
    creation, loading, its steps and the final diagnostics.  Returns
    particle-steps, seconds and particle-steps/s."""
    total_ps = 0
    total_s = 0.0
    for r in requests:
        parts = request_particles(r)
        t0 = time.perf_counter()
        run = R.Run(request_config(r))
        for sp, (x, u) in enumerate(parts):
            run.load(sp, x, u)
        run.step(r["steps"])
        run.diag()
        total_s += time.perf_counter() - t0
        total_ps += capi.grpic_particle_steps(run.h)
        run.close()
    return {"particle_steps": total_ps, "seconds": total_s,
            "particle_steps_per_s": total_ps / total_s if total_s > 0 else 0.0}


def main(argv=None):
    """Serve a seeded request mix and print its figures as one JSON line:
    python -m paper_0904_0232_amd.serve [--requests N] [--rate R] [--seed S]
    (rate in requests per second; a large rate makes every request arrive at
    once, which measures the loop's saturated capacity)."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=32)
    ap.add_argument("--rate", type=float, default=1e6)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--one-by-one", action="store_true",
                    help="also run the same requests alone, one after another")
    args = ap.parse_args(argv)
    reqs = make_requests(args.requests, args.seed, args.rate)
    res = serve(reqs, int(args.budget_gb * (1 << 30)), args.slots)
    res.pop("records")
    if args.one_by_one:
        res["one_by_one"] = one_by_one(reqs)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
