"""Continuous-batching request loop for independent GRPIC runs.

Requests (the serving workload: grid edge in {16, 32, 48, 64, 96}, spin
a ~ U[0, 0.99] m with m = edge/16, 2-8 particles per cell and species,
u_th ~ U[0.02, 0.2] c, 50-500 steps, FP32-mixed) arrive as a Poisson
process.  The loop admits arrived requests first-come-first-served whenever
the batch has a free slot and HBM budget (``grpic_batch_submit``), advances
every admitted run by one cycle per iteration (``grpic_batch_step``: each
run's captured cycle graph on its own stream, so runs overlap on the GPU),
and records each request's completion latency (arrival -> finished).  The
initial particles of queued requests are generated on host threads ahead of
admission.
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


def make_requests(n_runs, seed, rate, steps_range=(50, 500), ppc_range=(2, 8), edges=EDGES):
    """Seeded request list; arrival times of a Poisson process of `rate` per second."""
    g = inputs.rng(seed, 7)
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
            u_th=float(g.uniform(0.02, 0.2)), seed=int(seed) * 100003 + i))
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


def serve(requests, budget_bytes, max_slots, keep_ids=(), prefetch=8, log=None):
    """Run the request loop to completion.  Returns per-request records and totals."""
    b = capi.grpic_batch_create(budget_bytes, max_slots)
    pool = ThreadPoolExecutor(max_workers=prefetch)
    pending = collections.deque(sorted(requests, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    futures = {}
    active = {}
    records = {}
    for r in requests:
        cfg = request_config(r)
        if capi.grpic_run_bytes(cfg) > budget_bytes:
            raise ValueError("request %d needs more than the whole HBM budget" % r["id"])
    t0 = time.perf_counter()
    total_psteps = 0
    iterations = 0
    t_inputs = t_submit = t_step = 0.0  # host time waiting for inputs, admitting, stepping
    try:
        while pending or waiting or active:
            now = time.perf_counter() - t0
            while pending and pending[0]["arrival"] <= now:
                r = pending.popleft()
                waiting.append(r)
            # a request carries its particles: the payloads of the next few
            # requests in arrival order are drawn ahead on host threads, so
            # they are ready when the requests arrive
            for q in itertools.islice(itertools.chain(waiting, pending), prefetch):
                if q["id"] not in futures:
                    futures[q["id"]] = pool.submit(request_particles, q)
            while waiting:
                for q in itertools.islice(itertools.chain(waiting, pending), prefetch):
                    if q["id"] not in futures:
                        futures[q["id"]] = pool.submit(request_particles, q)
                r = waiting[0]
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
                records[r["id"]] = dict(r, admitted=time.perf_counter() - t0)
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
    return {
        "records": records,
        "n_runs": len(records),
        "makespan_s": makespan,
        "iterations": iterations,
        "p50_latency_s": percentile(lat, 50),
        "p99_latency_s": percentile(lat, 99),
        "particle_steps": total_psteps,
        "particle_steps_per_s": total_psteps / makespan if makespan > 0 else 0.0,
        "runs_per_s": len(records) / makespan if makespan > 0 else 0.0,
        "host_s": {"waiting_for_inputs": t_inputs, "admitting": t_submit, "stepping": t_step},
    }
