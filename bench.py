#!/usr/bin/env python3
"""GRPIC hot-path benchmark on one MI355X.

One step = one full GRPIC cycle (magnetic half-step, gather + RK4 push,
magnetic half-step, current deposition with removal, electric step, and the
cell sort amortised every sort_every steps) over the resident particle set.
The headline workload is the throughput configuration: Kerr a = 0.99 m on a
256^3 grid (m = 8 cells), 8 particles per cell and species (268,435,456
particles), uniform Maxwellian plasma u_th = 0.1 c plus a shell at
|R - 64| <= 2 falling in at v_r = -0.3 c, B_z = 0.1, dt = 0.45, in FP64
(value) and FP32-mixed (the "fp32_mixed" object), on synthetic seeded inputs
already in HBM when the timed region starts.  The 64^3 Kerr a = 0.95 m
workload (4,194,304 particles) is reported as a secondary key.

Prints ONE JSON line.  value = particle pushes per second over the timed
steps (live particles summed over steps / wall time).  The roofline object
prices the kernel that takes the most time (the pusher or the deposit; both
are in "rooflines") by its algorithmic FP64 operation count per particle
against the MI355X FP64 vector peak, with the average kernel time measured by
HIP events on the run's stream.  The CPU baseline times the FP64 oracle on
windows of the same workload (a 32^3 sub-box with its particles and its own
field solve, the hole placed by its centre in window coordinates): one
thread, and independent windows on all host cores.  The GPU's first cycle
is compared with the oracle's on the window interiors.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec on 1 MI355X (FP32-mixed vs FP64) + serving p50/p99 latency"
UNIT = "particle-steps/s"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

# Algorithmic FP64 operations of one particle-step of the pusher (one call of
# the RK4 step: four stages of radius quartic, Kerr-Schild gradients,
# Christoffel contraction, trilinear gather of 16 components, Lorentz term,
# paper gamma estimate and stage update, plus the final combination).  An FMA
# counts as 2, a division or square root as 1.  The breakdown is derived in
# the design notes from the kernel source.
PUSH_FLOPS_PER_PARTICLE_STEP = 2219

# Algorithmic FP64 operations of the curved-weight deposit of one particle
# (counted from the kernel source the same way): zigzag split 9; per segment
# 9 plus, for each of the 3 current directions, 59 for the flux, the
# segment-average term, the four sub-rectangles and the normalised fixed-point
# weights and 4 face-area densities (radius quartic, f, k_K, sqrt(1 + f(1 -
# k_K^2)): 41 for K = 0, 1 and 33 for K = 2); the removal test 19.  That is
# 9 + 2 (9 + 3 * 59 + 4 * 115) + 19 = 1320 per particle, with two segments
# per particle.
DEPOSIT_FLOPS_PER_PARTICLE = 1320

CSRC = os.path.join(ROOT, "paper_0904_0232_amd", "csrc")
KERNEL_SOURCES = {"fp64": ("particles.hip", "grpic_dev.h", "grpic_impl.h"),
                  "fp32": ("particles32.hip", "grpic_dev.h", "grpic_impl.h")}


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def traffic_file(precision, workload):
    return os.path.join(ROOT, "profiles", "%s_particle_kernels_%s_traffic.txt" % (precision, workload))


def kernel_source_hash(precision):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[precision]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(n_per_launch, precision, workload, key="hbm_bytes_per_particle"):
    """HBM bytes per launch of the pusher (or, with key
    "deposit_hbm_bytes_per_particle", of the deposit) from the committed
    rocprofv3 counter summary of that precision and workload, or None when
    the summary is missing or the kernel sources changed since."""
    path = traffic_file(precision, workload)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_hash(precision):
        return None
    try:
        per_particle = float(kv[key])
    except (KeyError, ValueError):
        return None
    return per_particle * n_per_launch


WINDOW = 32        # oracle window edge in cells
WINDOW_MARGIN = 8  # compared particles start and end this far inside a window


def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def window_origins(w, count):
    """Origins of `count` oracle windows of the workload: the first three at
    distance R = r_+ + 4 + WINDOW/2 from the hole along x, at n/4 along y and
    at 0.4 n along (1,1,1) (the hole's neighbourhood, the bulk with the
    infalling shell, further out); more along other directions at 0.3 n.
    Every window lies inside the grid and outside r_rm, so the oracle loads
    each window input it is given, in order."""
    import numpy as np
    n, c0 = w["n"], w["n"] / 2.0
    dirs = [(w["r_plus"] + 4.0 + WINDOW / 2.0, (1.0, 0.0, 0.0)), (n / 4.0, (0.0, 1.0, 0.0)),
            (0.4 * n, (1.0, 1.0, 1.0))]
    extra = [(-1, 0, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1), (1, -1, 0), (-1, 1, 0), (1, 1, -1), (-1, -1, 1),
             (1, 0, 1), (0, 1, -1), (-1, 0, -1), (0, -1, 1), (1, 1, 0), (-1, -1, 0)]
    dirs += [(0.3 * n, d) for d in extra]
    out = []
    for R, d in dirs[:count]:
        d = np.array(d, dtype=float) / np.linalg.norm(d)
        o = np.floor(c0 + R * d - WINDOW / 2.0).astype(int)
        o = np.clip(o, 1, n - WINDOW - 1)
        out.append(o)
    return out


def window_inputs(parts, o):
    """The inputs inside window o: per species (species, input indices,
    x in window coordinates, ucov)."""
    import numpy as np
    out = []
    for sp, x, uc in parts:
        inside = np.ones(x.shape[1], bool)
        for ax in range(3):
            inside &= (x[ax] >= o[ax]) & (x[ax] < o[ax] + WINDOW)
        idx = np.nonzero(inside)[0]
        out.append((sp, idx, x[:, idx] - o[:, None], uc[:, idx]))
    return out


def oracle_window_cycle(w, o, sel):
    """One full FP64 oracle cycle (field solve, push, deposit, removal) on
    the window at o with its inputs sel.  Returns (live particles, seconds,
    particle state after the cycle)."""
    import oracle as O
    p = O.make_params(WINDOW, m=w["m"], a=w["a"], dt=w["dt"], center=tuple(w["n"] / 2.0 - o), r_rm=w["r_rm"],
                      species=w["species"])
    s = O.Sim(p, sum(idx.size for _, idx, _, _ in sel))
    s.init_fields([0.0, 0.0, w["B0"]])
    kept = 0
    for sp, idx, x, uc in sel:
        k = s.load(sp, x, uc)
        assert k == idx.size, "an oracle window dropped an input"
        kept += k
    t0 = time.perf_counter()
    s.step(1)
    dt = time.perf_counter() - t0
    return kept, dt, s.particles()


def _window_job(args):
    w, o, sel = args
    kept, dt, _ = oracle_window_cycle(w, o, sel)
    return kept, dt


def cpu_baseline(workload, w, parts, single_windows=3, all_core_windows=16):
    """The FP64 oracle timed on windows of the workload: one thread on
    single_windows windows (their states are kept for the error check), then
    up to all_core_windows independent windows at once, one process per
    usable core (at most 16).  Returns the baseline and the windows."""
    import multiprocessing as mp

    import numpy as np
    host = host_info()
    origins = window_origins(w, max(single_windows, all_core_windows))
    windows, tot_kept, tot_s = [], 0, 0.0
    for o in origins[:single_windows]:
        sel = window_inputs(parts, o)
        kept, dt, state = oracle_window_cycle(w, o, sel)
        windows.append({"origin": o, "sel": [(sp, idx) for sp, idx, _, _ in sel], "state": state,
                        "x0": np.concatenate([x for _, _, x, _ in sel], axis=1)})
        tot_kept += kept
        tot_s += dt
        log("oracle window at %s: %d particles, %.2f s" % (list(o), kept, dt))
    out = {
        "value": tot_kept / tot_s,
        "unit": UNIT,
        "cores": 1,
        "kind": "oracle",
        "sample": "one full FP64 oracle cycle (field solve, push, deposit, removal) on %d windows of %d^3 cells "
                  "of the %s workload with their particles (%d in all, %.1f s), single thread"
                  % (single_windows, WINDOW, workload, tot_kept, tot_s),
        "host": host,
    }
    procs = max(1, min(16, host["usable_cpus"] or 1, all_core_windows))
    jobs = [(w, o, [(sp, idx, x, uc) for sp, idx, x, uc in window_inputs(parts, o)])
            for o in origins[:all_core_windows]]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        res = pool.map(_window_job, jobs, chunksize=1)
    wall = time.perf_counter() - t0
    kept = sum(k for k, _ in res)
    out["all_cores"] = {"value": kept / wall, "processes": procs, "windows": len(jobs), "particles": kept,
                        "wall_s": wall, "what": "independent oracle windows, one single-threaded process per "
                                                "usable core; wall time includes process start-up"}
    log("cpu baseline: %.4g particle-steps/s on 1 core, %.4g on %d processes" %
        (out["value"], out["all_cores"]["value"], procs))
    return out, windows


def window_errors(w, windows, state1, n_per_species):
    """Largest relative error, after the first cycle, of the GPU state
    against the oracle's windows, over the particles that start and end at
    least WINDOW_MARGIN cells inside a window (there the window's frozen
    faces do not reach the particles' fields within one cycle).  GPU slot of
    input i of species s = s * n_per_species + i (loads keep a slot for every
    input)."""
    import numpy as np
    import oracle as O
    x1, u1, sp1 = state1
    ex_max = eu_max = 0.0
    count, same = 0, True
    for win in windows:
        o = win["origin"]
        xo, uo, spo = win["state"]
        slots = np.concatenate([sp * n_per_species + idx for sp, idx in win["sel"]])
        xg = x1[:, slots] - o[:, None]
        ug = u1[:, slots]
        live = (spo != O.DEAD) & (sp1[slots] != O.DEAD)
        start_inner = np.ones(live.size, bool)
        for ax in range(3):
            start_inner &= (win["x0"][ax] >= WINDOW_MARGIN) & (win["x0"][ax] < WINDOW - WINDOW_MARGIN)
        # removal decisions of the particles that start inside the margin (the
        # window's own faces remove the others in the oracle)
        same &= bool(np.array_equal((spo != O.DEAD)[start_inner], (sp1[slots] != O.DEAD)[start_inner]))
        inner = live & start_inner
        for ax in range(3):
            inner &= (xo[ax] >= WINDOW_MARGIN) & (xo[ax] < WINDOW - WINDOW_MARGIN)
        ex = np.abs(xg[:, inner] - xo[:, inner]) / np.maximum(np.abs(xo[:, inner] + o[:, None]), 1.0)
        eu = np.abs(ug[:, inner] - uo[:, inner]) / np.maximum(np.abs(uo[:, inner]), 1.0)
        if inner.any():
            ex_max = max(ex_max, float(ex.max()))
            eu_max = max(eu_max, float(eu.max()))
        count += int(inner.sum())
    return {"x_rel": ex_max, "u_rel": eu_max, "particles": count, "same_removals": same}


def measure(workload, precision, steps, warmup, sort_every, parts, first_cycle_state=False, tile=4, repeat=True):
    """Time `steps` cycles of one run with HIP events around each kernel
    group; returns the figures of the timed region (and, with
    first_cycle_state, the particle state after the first warmup cycle,
    before any cell sort).  With repeat, the state after the warm-up is saved
    and the same cycles are timed twice more without events: replayed as
    captured graphs, and launched one by one."""
    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    w = inputs.workload_params(workload)
    ntot = sum(p[1].shape[1] for p in parts)
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=sort_every, capacity=ntot, tile=tile,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64,
                        density=w["ppc"] if w["plasma"] != "torus" else None)
    run = R.Run(cfg)
    t0 = time.perf_counter()
    for sp, x, uc in parts:
        run.load(sp, x, uc)
    log("%s %s: loaded %d particles in %.1f s" % (workload, precision, ntot, time.perf_counter() - t0))
    h = run.h
    state1 = None
    # the loaded particles are put in cell order once (after the first cycle
    # when its state is checked against the oracle by load order), so the
    # timed cycles see sorted particles whatever the warm-up length
    if first_cycle_state and warmup > 0 and (sort_every == 0 or sort_every > 1):
        capi.grpic_step(h, 1)
        state1 = run.particles()
        if sort_every > 0:
            capi.grpic_sort(h, outputs=False)
        capi.grpic_step(h, warmup - 1)
    else:
        if sort_every > 0:
            capi.grpic_sort(h, outputs=False)
        capi.grpic_step(h, warmup)
    torch.cuda.synchronize()
    ps0 = capi.grpic_particle_steps(h)
    state = run.save_state() if repeat else None
    capi.grpic_set_timing(h, True)
    capi.grpic_read_timing(h)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    capi.grpic_step(h, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = capi.grpic_read_timing(h)
    capi.grpic_set_timing(h, False)
    ps1 = capi.grpic_particle_steps(h)
    d = run.diag()
    wall = t1 - t0
    psteps = ps1 - ps0
    # the same cycles again from the same state, without kernel events: once
    # with each cycle's kernels replayed as one captured graph, once launched
    # one by one
    again = {}
    if state is not None:
        for name, graphs in (("graphs", True), ("launches", False)):
            run.load_state(state)
            capi.grpic_set_graphs(h, graphs)
            torch.cuda.synchronize()
            g0 = time.perf_counter()
            capi.grpic_step(h, steps)
            torch.cuda.synchronize()
            g1 = time.perf_counter()
            again[name] = {"value": psteps / (g1 - g0), "ms_per_step": (g1 - g0) * 1e3 / steps}
            assert capi.grpic_particle_steps(h) == ps1, "a repeat of the timed cycles did other work"
        del state
    run.close()
    what = {k: "the timed cycles again from the same state without kernel events, " + v
            for k, v in (("graphs", "each cycle's kernels replayed as one captured graph"),
                         ("launches", "kernels launched one by one"))}
    return {
        "w": w, "ntot": ntot, "wall": wall, "psteps": psteps, "value": psteps / wall,
        "ms_per_step": wall * 1e3 / steps, "timers": timers,
        "kernel_ms_per_launch": {k: (v[0] / max(v[1], 1)) for k, v in timers.items()},
        "live_end": int(sum(d["n_alive"])), "state1": state1,
        "graphs": dict(again["graphs"], what=what["graphs"]) if again else None,
        "launches": dict(again["launches"], what=what["launches"]) if again else None,
        "deposit_blocks": {"lds": d["deposit_blocks_lds"], "global": d["deposit_blocks_global"]},
        "push_blocks": {"lds": d["push_blocks_lds"], "global": d["push_blocks_global"]},
    }


KERNELS = {
    "push": ("k_push (gather + RK4 pusher)", PUSH_FLOPS_PER_PARTICLE_STEP, "hbm_bytes_per_particle"),
    "deposit": ("k_deposit (zigzag, curved face-area weights, int64 current)", DEPOSIT_FLOPS_PER_PARTICLE,
                "deposit_hbm_bytes_per_particle"),
}


def kernel_roofline(m, name, peak, with_traffic, workload, precision):
    """Algorithmic FLOP/s of one kernel over its event-timed launches
    (particles per launch = particle-steps of the timed region / launches)."""
    label, flops, tkey = KERNELS[name]
    if precision == "fp32":
        label = label.replace("k_push", "k_push32").replace("k_deposit", "k_deposit32")
    ms, n = m["timers"][name]
    avg_s = ms / 1e3 / max(n, 1)
    per_launch = m["psteps"] / max(n, 1)
    achieved = flops * per_launch / avg_s / 1e12
    return {
        "kernel": label,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": read_traffic(per_launch, precision, workload, tkey) if with_traffic else None,
        "avg_launch_ms": avg_s * 1e3,
        "flops_per_particle": flops,
        "particles_per_launch": per_launch,
    }


def rooflines(m, peak, with_traffic, workload, precision="fp64"):
    """Both particle kernels' rooflines and the one of the kernel that takes
    the most time (each launches once per cycle)."""
    both = {k: kernel_roofline(m, k, peak, with_traffic, workload, precision) for k in KERNELS}
    dominant = max(both, key=lambda k: both[k]["avg_launch_ms"])
    return both[dominant], both


def serving(args):
    """Continuous batching of independent FP32-mixed runs with Poisson
    arrivals.  A saturated probe (32 requests arriving at once) measures the
    loop's own capacity in particle-steps/s, beside the same 32 requests run
    alone one after another as single runs; the measured workload then
    arrives at 0.7 of that capacity."""
    from paper_0904_0232_amd import serve
    budget = int(args.serve_budget_gb * (1 << 30))

    def work(reqs):
        return sum(2 * r["ppc"] * r["edge"] ** 3 * r["steps"] for r in reqs) / len(reqs)

    probe_reqs = serve.make_requests(32, 1, 1e6)
    probe = serve.serve(probe_reqs, budget, args.serve_slots)
    capacity = probe["particle_steps_per_s"]
    alone = serve.one_by_one(probe_reqs)
    log("serving probe: %.4g particle-steps/s saturated; the same requests alone, one after another: %.4g" %
        (capacity, alone["particle_steps_per_s"]))
    rate = 0.7 * capacity / work(serve.make_requests(args.serve_runs, 0, 1.0))
    reqs = serve.make_requests(args.serve_runs, 0, rate)
    res = serve.serve(reqs, budget, args.serve_slots)
    return {
        "runs": res["n_runs"],
        "arrival_rate_per_s": rate,
        "p50_latency_s": res["p50_latency_s"],
        "p99_latency_s": res["p99_latency_s"],
        "runs_per_s": res["runs_per_s"],
        "particle_steps_per_s": res["particle_steps_per_s"],
        "saturated_particle_steps_per_s": capacity,
        "saturated_host_s": probe["host_s"],
        "one_by_one_particle_steps_per_s": alone["particle_steps_per_s"],
        "saturated_vs_one_by_one": capacity / alone["particle_steps_per_s"],
        "makespan_s": res["makespan_s"],
        "iterations": res["iterations"],
        "host_s": res["host_s"],
        "budget_gb": args.serve_budget_gb,
        "slots": args.serve_slots,
        "workload": "grid edge in {16,32,48,64,96}, a~U[0,0.99]m, m=edge/16, 2-8 ppc per species, "
                    "u_th~U[0.02,0.2]c, 50-500 steps, FP32-mixed, Poisson arrivals at 0.7 of the saturated "
                    "capacity (seed 0)",
    }


def preemption_study(args, n_runs=64, slots=4, urgent_frac=0.2, load=1.5):
    """Urgent requests with and without preemption: n_runs requests (50-200
    steps, otherwise the serving workload), a fraction urgent_frac of them
    urgent, arriving at `load` of the loop's saturated capacity with `slots`
    slots, so slots are contended.  Reports latency percentiles of urgent and
    normal requests in both policies."""
    from paper_0904_0232_amd import serve
    budget = int(args.serve_budget_gb * (1 << 30))

    def reqs_at(rate, seed):
        return serve.make_requests(n_runs, seed, rate, steps_range=(50, 200), urgent_frac=urgent_frac)

    probe = serve.serve(serve.make_requests(32, 1, 1e6, steps_range=(50, 200)), budget, slots)
    capacity = probe["particle_steps_per_s"]
    work = sum(2 * r["ppc"] * r["edge"] ** 3 * r["steps"] for r in reqs_at(1.0, 2)) / n_runs
    rate = load * capacity / work
    out = {"workload": "%d requests, 50-200 steps, otherwise the serving workload; %g urgent; %d slots; "
                       "Poisson arrivals at %g of the saturated capacity (seed 2)" % (n_runs, urgent_frac, slots, load),
           "saturated_particle_steps_per_s": capacity}
    for name, pre in (("fifo", False), ("preempt", True)):
        res = serve.serve(reqs_at(rate, 2), budget, slots, preempt=pre)
        out[name] = {"urgent": res["urgent"], "normal": res["normal"], "preemptions": res["preemptions"],
                     "makespan_s": res["makespan_s"], "particle_steps_per_s": res["particle_steps_per_s"]}
        log("preemption study %s: urgent p50 %.3f p99 %.3f s, normal p50 %.3f p99 %.3f s, %d preemptions" %
            (name, res["urgent"]["p50_latency_s"], res["urgent"]["p99_latency_s"], res["normal"]["p50_latency_s"],
             res["normal"]["p99_latency_s"], res["preemptions"]))
    return out


def jet_study(snapshots=(0, 50, 100, 150, 200, 250, 300, 350, 400, 450, 500)):
    """The paper's application (Sec. 6, inputs.jet_params for the readings):
    500 steps of the disk + corona workload on 64 x 64 x 128 with B^z = 30,
    in FP64 and FP32-mixed, and an FP64 control with B = 0.  The paper shows
    only pictures (a bipolar jet spiralling about z), so the check is
    qualitative: at each snapshot, the particles within 16 cells of the axis,
    more than 8 cells from the mid-plane and moving away from it faster than
    0.05 c, above and below the plane, their speeds, mean azimuthal velocity
    and median distance from the axis, the same with no field, and with an
    8-cell outer absorbing layer instead of frozen outer faces.
    Throughput is particle-steps per second of the timed steps."""
    import numpy as np
    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    w = inputs.jet_params()
    parts = inputs.jet_particles(0)
    ntot = sum(x.shape[1] for _, x, _ in parts)
    cen = np.array(w["center"])
    out = {"workload": "jet64x64x128", "particles": ntot, "m": w["m"], "a": w["a"], "c": w["c"], "dt": w["dt"],
           "runs": {}}
    for name, prec, b0, layer in (("B30_fp64", capi.FP64, w["B0"], 0.0), ("B30_fp32", capi.FP32_MIXED, w["B0"], 0.0),
                                  ("B0_fp64", capi.FP64, 0.0, 0.0), ("B30_fp64_absorbing", capi.FP64, w["B0"], 8.0)):
        cfg = R.make_config(w["nx"], ny=w["ny"], nz=w["nz"], m=w["m"], a=w["a"], c=w["c"], dt=w["dt"],
                            B0=(0.0, 0.0, b0), species=w["species"], r_rm=w["r_rm"], sort_every=8, capacity=ntot,
                            precision=prec, center=w["center"], outer_layer=layer, outer_damp=0.3 if layer else 0.0)
        r = R.Run(cfg)
        for sp, x, uc in parts:
            r.load(sp, x, uc)
        r.sort(outputs=False)
        snaps, wall, psteps, done = {}, 0.0, 0, 0
        for t in snapshots:
            if t > done:
                torch.cuda.synchronize()
                ps0 = capi.grpic_particle_steps(r.h)
                t0 = time.perf_counter()
                capi.grpic_step(r.h, t - done)
                torch.cuda.synchronize()
                wall += time.perf_counter() - t0
                psteps += capi.grpic_particle_steps(r.h) - ps0
                done = t
            x, u, sp = r.particles()
            live = sp != 0xFF
            d = x[:, live] - cen[:, None]
            v = w["c"] * u[:3, live] / u[3, live]
            rho = np.hypot(d[0], d[1])
            vout = v[2] * np.sign(d[2])
            jet = (rho < 16.0) & (np.abs(d[2]) > 8.0) & (vout > 0.05 * w["c"])
            speed = np.linalg.norm(v[:, jet], axis=0) / w["c"]
            # azimuthal velocity about +z (negative: clockwise, with the hole's frame dragging)
            vphi = (d[0, jet] * v[1, jet] - d[1, jet] * v[0, jet]) / np.maximum(rho[jet], 1e-12) / w["c"]
            snaps[str(t)] = {"live": int(live.sum()), "outflow_above": int((jet & (d[2] > 0)).sum()),
                             "outflow_below": int((jet & (d[2] < 0)).sum()),
                             "outflow_median_speed_c": float(np.median(speed)) if speed.size else None,
                             "outflow_frac_above_0.5c": float((speed > 0.5).mean()) if speed.size else None,
                             "outflow_mean_vphi_c": float(vphi.mean()) if speed.size else None,
                             "outflow_median_rho": float(np.median(rho[jet])) if speed.size else None}
        r.close()
        out["runs"][name] = {"particle_steps_per_s": psteps / wall, "ms_per_step": wall * 1e3 / done,
                             "snapshots": snaps}
        log("jet %s: %.4g particle-steps/s, %s" % (name, psteps / wall, json.dumps(snaps)))
    return out


def ablation_study(workload="kerr64", per_species=131072, T=8.0, dts=(0.4, 0.2, 0.1, 0.05), timing_steps=10):
    """The push readings side by side (FP64): the stage gamma (PAPER estimate
    or u^4/c), the RK structure (CLASSIC reading or the steps as PRINTED),
    where the field tensor is gathered (every STAGE or once per STEP) and
    the gather weights (TRILINEAR, or SPATIAL: reading B).
    For each: the observed order in coordinate time of test particles in the
    workload's frozen initial fields (positions at time T for the step sizes
    dts; order = log2 of the median ratio of successive differences, over
    particles that stay finite, inside the grid and outside R = 3m in every
    run), the distance of the finest solution from the U4 / CLASSIC /
    STAGE / TRILINEAR one (consistency: a scheme can converge to the wrong
    path) and the push kernel time per launch on the whole workload.  Also
    the Gauss-law residual after 20 cycles with CURVED and FLAT deposition
    (only FLAT conserves charge exactly)."""
    import numpy as np
    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    w = inputs.workload_params(workload)
    parts = inputs.workload_particles(workload, seed=0)
    sub = [(sp, x[:, :per_species], uc[:, :per_species]) for sp, x, uc in parts]
    nsub = sum(x.shape[1] for _, x, _ in sub)
    ntot = sum(x.shape[1] for _, x, _ in parts)
    cen = np.full(3, w["n"] / 2.0)

    def cfg(dt, gm, rk, ga, wt, cap, sort_every=0, deposit_mode=capi.DEPOSIT_CURVED):
        return R.make_config(w["n"], m=w["m"], a=w["a"], dt=dt, B0=(0.0, 0.0, w["B0"]), species=w["species"],
                             r_rm=w["r_rm"], sort_every=sort_every, capacity=cap, gamma_mode=gm, rk_mode=rk,
                             gather_mode=ga, gather_weights=wt, deposit_mode=deposit_mode)

    G = {"PAPER": capi.GAMMA_PAPER, "U4": capi.GAMMA_U4}
    K = {"CLASSIC": capi.RK_CLASSIC, "PRINTED": capi.RK_PRINTED}
    A = {"STAGE": capi.GATHER_STAGE, "STEP": capi.GATHER_STEP}
    Wt = {"TRILINEAR": capi.WEIGHTS_TRILINEAR, "SPATIAL": capi.WEIGHTS_SPATIAL}
    ref = ("U4", "CLASSIC", "STAGE", "TRILINEAR")  # first: the others are compared with it
    combos = [ref, ("U4", "CLASSIC", "STEP", "TRILINEAR"), ("U4", "PRINTED", "STAGE", "TRILINEAR"),
              ("U4", "CLASSIC", "STAGE", "SPATIAL"), ("PAPER", "CLASSIC", "STAGE", "TRILINEAR"),
              ("PAPER", "CLASSIC", "STEP", "TRILINEAR"), ("PAPER", "PRINTED", "STAGE", "TRILINEAR"),
              ("PAPER", "PRINTED", "STEP", "TRILINEAR"), ("PAPER", "CLASSIC", "STAGE", "SPATIAL")]
    out = {"workload": workload, "test_particles": nsub, "T": T, "dts": list(dts), "readings": {}}
    finest = {}
    for combo in combos:
        gm, rk, ga, wt = G[combo[0]], K[combo[1]], A[combo[2]], Wt[combo[3]]
        xs = []
        for dt in dts:
            r = R.Run(cfg(dt, gm, rk, ga, wt, nsub))
            for sp, x, uc in sub:
                r.load(sp, x, uc)
            r.push_only(int(round(T / dt)))
            xs.append(r.particles()[0])
            r.close()
        ok = np.ones(xs[0].shape[1], bool)
        for x in xs:
            ok &= np.isfinite(x).all(axis=0) & (x >= 0).all(axis=0) & (x <= w["n"]).all(axis=0)
            ok &= np.linalg.norm(x - cen[:, None], axis=0) > 3.0 * w["m"]
        d = [np.abs(xs[i] - xs[i + 1]).max(axis=0)[ok] for i in range(len(xs) - 1)]
        keep = d[-1] > 1e-13
        ratio = np.median(d[-2][keep] / d[-1][keep]) if keep.any() else float("nan")
        name = "gamma_%s/rk_%s/gather_%s/weights_%s" % combo
        entry = {"order": float(np.log2(ratio)), "particles": int(ok.sum()),
                 "median_diff_dt%g_vs_dt%g" % (dts[0], dts[1]): float(np.median(d[0])),
                 "median_diff_dt%g_vs_dt%g" % (dts[-2], dts[-1]): float(np.median(d[-1]))}
        # consistency: the finest solution against the reference one (fourth
        # order in smooth fields); a scheme can converge to the wrong path
        finest[combo] = (xs[-1], ok)
        xr, okr = finest[ref]
        both = ok & okr
        entry["median_diff_vs_reference_at_dt%g" % dts[-1]] = float(np.median(np.abs(xs[-1] - xr).max(axis=0)[both]))
        if combo[0] == "PAPER":
            r = R.Run(cfg(w["dt"], gm, rk, ga, wt, ntot, sort_every=5))
            for sp, x, uc in parts:
                r.load(sp, x, uc)
            capi.grpic_step(r.h, 10)
            capi.grpic_set_timing(r.h, True)
            capi.grpic_read_timing(r.h)
            capi.grpic_step(r.h, timing_steps)
            torch.cuda.synchronize()
            t = capi.grpic_read_timing(r.h)
            r.close()
            entry["push_ms_per_launch"] = t["push"][0] / max(t["push"][1], 1)
        out["readings"][name] = entry
        log("ablation %s: %s" % (name, json.dumps(entry)))
    for dm, dname in ((capi.DEPOSIT_CURVED, "CURVED"), (capi.DEPOSIT_FLAT, "FLAT")):
        r = R.Run(cfg(w["dt"], capi.GAMMA_PAPER, capi.RK_CLASSIC, capi.GATHER_STAGE, capi.WEIGHTS_TRILINEAR, ntot,
                      sort_every=5, deposit_mode=dm))
        for sp, x, uc in parts:
            r.load(sp, x, uc)
        capi.grpic_step(r.h, 20)
        d = r.diag()
        r.close()
        out["deposit_%s_gauss_residual_max_after_20" % dname] = d["gauss_residual_max"]
        log("ablation deposit %s: Gauss residual %.3e" % (dname, d["gauss_residual_max"]))
    return out


def precision_study(workload, checkpoints=(1, 10, 100, 300, 1000), modes=("geodesic", "push", "cycle"), n_override=None,
                    log=sys.stderr):
    """FP32-mixed against FP64 on one workload, particle identity kept (one
    cell sort at load, none afterwards).  Three runs per mode:
      A  FP64 loaded from the exact inputs,
      B  FP64 restored from C's loaded state (the inputs rounded to the
         mixed representation: FP32 offsets and velocities),
      C  FP32-mixed.
    C-A is the whole FP32-mixed error; C-B isolates the FP32 arithmetic of
    the steps; B-A is the control: how far FP64 itself carries a perturbation
    of the size of one FP32 rounding of the start (the dynamics' own
    divergence).  At every checkpoint the particles' current is also
    coarse-grained over 8^3-cell blocks (per species and net, from their
    coordinate velocities) and compared in L2.  "geodesic" runs test particles with no field, "push" test
    particles in the frozen initial fields, "cycle" the self-consistent cycle.  A particle is "regular" while its A
    path stays inside the grid and outside R = 3m."""
    import numpy as np
    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    w = inputs.workload_params(workload)
    parts = inputs.workload_particles(workload, seed=0, n_override=n_override)
    ntot = sum(p[1].shape[1] for p in parts)
    cen = np.full(3, w["n"] / 2.0)

    def cfg(prec, b0):
        return R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, b0), species=w["species"],
                             r_rm=w["r_rm"], sort_every=0, capacity=ntot,
                             precision=capi.FP32_MIXED if prec == "fp32" else capi.FP64)

    def diff(P, Q, regular):
        (x1, u1, s1), (x2, u2, s2) = P, Q
        both = (s1 != 255) & (s2 != 255)
        with np.errstate(invalid="ignore", divide="ignore"):
            ex = (np.abs(x2 - x1) / np.maximum(np.abs(x1), 1.0)).max(axis=0)
            eu = (np.abs(u2 - u1) / np.maximum(np.abs(u1), 1.0)).max(axis=0)
        e = np.where(np.isfinite(ex) & np.isfinite(eu), np.maximum(ex, eu), np.inf)
        reg = regular & both
        return {
            "alive_mismatch": int(((s1 != 255) != (s2 != 255)).sum()),
            "frac_within_1e-4": float((e[both] < 1e-4).mean()) if both.any() else None,
            "regular": int(reg.sum()),
            "regular_frac_within_1e-4": float((e[reg] < 1e-4).mean()) if reg.any() else None,
            "regular_median": float(np.median(e[reg])) if reg.any() else None,
            "regular_p99": float(np.quantile(e[reg], 0.99)) if reg.any() else None,
        }

    def jdiff(J1, J2):
        return {"l2_rel": float(np.linalg.norm(J2 - J1) / np.linalg.norm(J1)),
                "max_rel": float(np.abs(J2 - J1).max() / np.abs(J1).max())}

    def coarse_current(P, mask=None, block=8):
        """Per species and net: sum over the particles a cycle would keep
        (alive, finite, inside the grid, outside r_rm; push-only steps do not
        remove particles), and in `mask` when given, in each block^3-cell
        block of q c u^i / u^4 (c = 1)."""
        x, u, sp = P
        n = w["n"]
        nb = n // block
        with np.errstate(invalid="ignore", over="ignore"):
            fin = np.isfinite(x).all(0) & np.isfinite(u).all(0)
            xs = np.where(fin, x, -1.0)
            inside = np.all((xs >= 0) & (xs < n), axis=0)
            X, Y, Z = xs - n / 2.0
            b = X * X + Y * Y + Z * Z - w["a"] ** 2
            r = np.sqrt(0.5 * (b + np.sqrt(b * b + 4.0 * w["a"] ** 2 * Z * Z)))
        kept = (sp != 255) & fin & inside & (r > w["r_rm"])
        if mask is not None:
            kept &= mask
        idx = np.clip(np.floor(xs[:, kept] / block).astype(np.int64), 0, nb - 1)
        flat = (idx[2] * nb + idx[1]) * nb + idx[0]
        v = u[:3, kept] / u[3, kept]
        out = np.zeros((len(w["species"]) + 1, 3, nb ** 3))
        for s_, (q, _) in enumerate(w["species"]):
            sel = sp[kept] == s_
            for i in range(3):
                out[s_, i] = np.bincount(flat[sel], weights=q * v[i, sel], minlength=nb ** 3)
        out[-1] = out[:-1].sum(axis=0)
        return out

    def cdiff(J1, J2):
        return {k: float(np.linalg.norm(J2[s_] - J1[s_]) / np.linalg.norm(J1[s_]))
                for s_, k in enumerate(("electrons", "ions", "net"))}

    out = {"workload": workload, "particles": ntot}
    for mode in modes:
        b0 = 0.0 if mode == "geodesic" else w["B0"]
        c = R.Run(cfg("fp32", b0))
        a = R.Run(cfg("fp64", b0))
        for sp, x, uc in parts:
            c.load(sp, x, uc)
            a.load(sp, x, uc)
        c.sort()
        a.sort()
        b = R.Run(cfg("fp64", b0))
        b.restore_particles(*c.particles())
        runs = {"A": a, "B": b, "C": c}
        regular = None
        rows = []
        done = 0
        for target in checkpoints:
            t0 = time.perf_counter()
            for r in runs.values():
                if mode == "cycle":
                    r.step(target - done)
                else:
                    r.push_only(target - done)
            torch.cuda.synchronize()
            done = target
            st = {k: r.particles() for k, r in runs.items()}
            xa, ua, sa = st["A"]
            Rr = np.sqrt(((xa - cen[:, None]) ** 2).sum(0))
            ok = np.all((xa >= 0) & (xa < w["n"]), axis=0) & (Rr > 3.0 * w["m"]) & np.isfinite(ua).all(0) & (sa != 255)
            regular = ok if regular is None else (regular & ok)
            row = {"step": target, "alive": int((sa != 255).sum()),
                   "fp32_vs_fp64": diff(st["A"], st["C"], regular),
                   "fp32_arith": diff(st["B"], st["C"], regular),
                   "fp64_control": diff(st["A"], st["B"], regular)}
            Jc = {k: coarse_current(v) for k, v in st.items()}
            row["coarse_J_8cells"] = {"fp32_vs_fp64": cdiff(Jc["A"], Jc["C"]), "fp32_arith": cdiff(Jc["B"], Jc["C"]),
                                      "fp64_control": cdiff(Jc["A"], Jc["B"])}
            Jc = {k: coarse_current(v, regular) for k, v in st.items()}
            row["coarse_J_8cells_regular"] = {"fp32_vs_fp64": cdiff(Jc["A"], Jc["C"]),
                                              "fp32_arith": cdiff(Jc["B"], Jc["C"]),
                                              "fp64_control": cdiff(Jc["A"], Jc["B"])}
            del st, Jc
            if mode == "cycle":
                J = {k: r.fields("J") for k, r in runs.items()}
                row["J_fp32_vs_fp64"] = jdiff(J["A"], J["C"])
                row["J_fp32_arith"] = jdiff(J["B"], J["C"])
                row["J_fp64_control"] = jdiff(J["A"], J["B"])
                del J
            rows.append(row)
            print("precision %s step %d (%.1f s): %s" % (mode, target, time.perf_counter() - t0, json.dumps(row)),
                  file=log, flush=True)
        for r in runs.values():
            r.close()
        out[mode] = rows
    return out


def describe(workload, w, ntot, sort_every, tile):
    plasma = {"uniform": "uniform Maxwellian", "shell": "uniform Maxwellian plus a shell |R - n/4| <= 2 at "
              "v_r = -0.3c", "torus": "torus"}[w["plasma"]]
    return ("%s: Kerr a=%.2fm, m=%g cells, %d^3 grid, %d particles (%d ppc x 2 species), %s u_th=%gc, B_z=%g, "
            "dt=%g, curved deposit, paper gamma, sort every %d steps (tiles of %d^3 cells)"
            % (workload, w["a_frac"], w["m"], w["n"], ntot, w["ppc"], plasma, w["u_th"], w["B0"], w["dt"],
               sort_every, tile))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="shell256")
    ap.add_argument("--sort-every", type=int, default=8)
    ap.add_argument("--tile", type=int, default=4, help="edge in cells of the sort's tiles")
    ap.add_argument("--secondary", default="kerr64",
                    help="second workload timed in both precisions ('' skips it)")
    ap.add_argument("--secondary-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-windows", type=int, default=3, help="oracle windows timed on one thread")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed measurement")
    ap.add_argument("--precision", action="store_true",
                    help="also run the FP32-mixed vs FP64 precision study on the torus workload (1000 steps)")
    ap.add_argument("--jet", action="store_true",
                    help="add the paper's application (disk + corona, 64x64x128, c = 0.05): throughput and outflow")
    ap.add_argument("--ablations", action="store_true",
                    help="add the push-reading ablation study (orders, push time, CURVED/FLAT Gauss residual)")
    ap.add_argument("--precision-particles", type=int, default=0,
                    help="particles per species for the precision study (0: the full workload)")
    ap.add_argument("--serve-runs", type=int, default=256, help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--preemption", action="store_true",
                    help="add the urgent-request study (FIFO admission vs preemption, 4 slots)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the GRPIC path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_0904_0232_amd import inputs
    w = inputs.workload_params(args.workload)
    t0 = time.perf_counter()
    parts = inputs.workload_particles(args.workload, seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    nps = parts[0][1].shape[1]
    log("%s: generated %d particles in %.1f s" % (args.workload, ntot, time.perf_counter() - t0))
    # the oracle's windows first: host work only, before the GPU is touched
    cpu, windows = (None, None) if args.no_cpu_baseline else cpu_baseline(args.workload, w, parts, args.cpu_windows)

    import torch
    torch.cuda.set_device(0)

    errs = {}
    m64 = measure(args.workload, "fp64", args.steps, args.warmup, args.sort_every, parts,
                  first_cycle_state=windows is not None, tile=args.tile)
    log("fp64 %s: %.4g particle-steps/s" % (args.workload, m64["value"]))
    if windows is not None and m64["state1"] is not None:
        errs["fp64"] = window_errors(w, windows, m64["state1"], nps)
        log("fp64 error vs oracle windows: %s" % json.dumps(errs["fp64"]))
    m64["state1"] = None
    roofline, rooflines64 = rooflines(m64, FP64_PEAK_TFLOPS, True, args.workload)
    line = {
        "metric": METRIC,
        "value": m64["value"],
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": describe(args.workload, w, ntot, args.sort_every, args.tile),
            "precision": "fp64",
            "live_particles_end": m64["live_end"],
        },
        "kernel_ms_per_launch": m64["kernel_ms_per_launch"],
        "graph_replay": m64["graphs"], "launches_no_events": m64["launches"],
        "deposit_blocks": m64["deposit_blocks"], "push_blocks": m64["push_blocks"],
        "roofline": roofline,
        "rooflines": rooflines64,
        "cpu_baseline": cpu,
    }
    if not args.no_fp32:
        m32 = measure(args.workload, "fp32", args.steps, args.warmup, args.sort_every, parts,
                      first_cycle_state=windows is not None, tile=args.tile)
        log("fp32-mixed %s: %.4g particle-steps/s" % (args.workload, m32["value"]))
        if windows is not None and m32["state1"] is not None:
            errs["fp32_mixed"] = window_errors(w, windows, m32["state1"], nps)
            log("fp32-mixed error vs oracle windows: %s" % json.dumps(errs["fp32_mixed"]))
        m32["state1"] = None
        line["fp32_mixed"] = {
            "value": m32["value"], "unit": UNIT, "ms_per_step": m32["ms_per_step"], "dtype": "f32 (FP64 quartic, "
            "near-horizon metric and diagnostics)", "kernel_ms_per_launch": m32["kernel_ms_per_launch"],
            "speedup_vs_fp64": m32["value"] / m64["value"], "live_particles_end": m32["live_end"],
            "deposit_blocks": m32["deposit_blocks"], "push_blocks": m32["push_blocks"], "graph_replay": m32["graphs"],
            "launches_no_events": m32["launches"],
        }
        line["fp32_mixed"]["roofline"], line["fp32_mixed"]["rooflines"] = rooflines(m32, FP32_PEAK_TFLOPS, True,
                                                                                      args.workload, "fp32")
    if errs:
        errs["what"] = ("largest relative error after the first cycle against the FP64 oracle's windows, over the "
                        "particles at least %d cells inside a %d^3 window at the start and end of the cycle "
                        "(positions relative to max(|x|, 1 cell), four-velocities to max(|u|, c))"
                        % (WINDOW_MARGIN, WINDOW))
        line["error_vs_oracle"] = errs
    del parts, windows
    if args.secondary:
        sparts = inputs.workload_particles(args.secondary, seed=0)
        sw = inputs.workload_params(args.secondary)
        sec = {"workload": describe(args.secondary, sw, sum(p[1].shape[1] for p in sparts), args.sort_every,
                                    args.tile)}
        for prec in ("fp64", "fp32"):
            ms = measure(args.secondary, prec, args.secondary_steps, args.warmup, args.sort_every, sparts,
                         tile=args.tile)
            log("%s %s: %.4g particle-steps/s" % (args.secondary, prec, ms["value"]))
            sec[prec] = {"value": ms["value"], "ms_per_step": ms["ms_per_step"], "steps": args.secondary_steps,
                         "graph_replay": ms["graphs"], "launches_no_events": ms["launches"],
                         "kernel_ms_per_launch": ms["kernel_ms_per_launch"], "live_particles_end": ms["live_end"],
                         "roofline": rooflines(ms, FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS, False,
                                               args.secondary)[0]}
        line["secondary_" + args.secondary] = sec
        del sparts
    if args.serve_runs > 0:
        line["serving"] = serving(args)
        log("serving: p50 %.3f s p99 %.3f s" % (line["serving"]["p50_latency_s"], line["serving"]["p99_latency_s"]))
    if args.precision:
        line["precision_torus128"] = precision_study("torus128", n_override=args.precision_particles or None)
    if args.ablations:
        line["ablations_kerr64"] = ablation_study()
    if args.jet:
        line["jet"] = jet_study()
    if args.preemption:
        line["preemption"] = preemption_study(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
