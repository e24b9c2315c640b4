#!/usr/bin/env python3
"""GRPIC hot-path benchmark on one MI355X.

One step = one full GRPIC cycle (magnetic half-step, gather + RK4 push,
magnetic half-step, current deposition with removal, electric step, and the
cell sort amortised every sort_every steps) over the resident particle set.
The workload is the Kerr a = 0.95 m plasma on a 64^3 grid (m = 3 cells,
8 particles per cell and species, 4,194,304 particles, u_th = 0.1 c,
B_z = 0.1, dt = 0.45), FP64, synthetic seeded inputs already in HBM when the
timed region starts.

Prints ONE JSON line.  value = particle pushes per second over the timed
steps (live particles summed over steps / wall time).  The roofline object
prices the kernel that takes the most time (the pusher or the deposit; both
are in "rooflines") by its algorithmic FP64 operation count per particle
against the MI355X FP64 vector peak, with the average kernel time measured by
HIP events on the run's stream.  The CPU
baseline times the FP64 oracle (single thread) on a bounded sample of the
same workload.
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

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fp64_particle_kernels_kerr64_traffic.txt")
PUSH_SOURCES = [os.path.join(ROOT, "paper_0904_0232_amd", "csrc", f) for f in ("particles.hip", "grpic_dev.h")]


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def push_source_hash():
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(n_per_launch, key="hbm_bytes_per_particle"):
    """HBM bytes per launch of the pusher (or, with key
    "deposit_hbm_bytes_per_particle", of the deposit) from the committed
    rocprofv3 counter summary, or None when the summary is missing or the
    kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != push_source_hash():
        return None
    try:
        per_particle = float(kv[key])
    except (KeyError, ValueError):
        return None
    return per_particle * n_per_launch


def cpu_baseline(workload, sample_per_species):
    """The FP64 oracle (one thread) timed on one cycle of a sample of the
    workload: the first sample_per_species particles of each species.
    Returns the figures and the oracle's particle state after the cycle."""
    import oracle as O
    from paper_0904_0232_amd import inputs
    w = inputs.workload_params(workload)
    parts = inputs.workload_particles(workload, seed=0)
    p = O.make_params(w["n"], m=w["m"], a=w["a"], dt=w["dt"], r_rm=w["r_rm"], species=w["species"])
    s = O.Sim(p, 2 * sample_per_species)
    s.init_fields([0.0, 0.0, w["B0"]])
    kept = 0
    for sp, x, uc in parts:
        kept += s.load(sp, x[:, :sample_per_species], uc[:, :sample_per_species])
    t0 = time.perf_counter()
    s.step(1)
    dt = time.perf_counter() - t0
    return {
        "value": kept / dt,
        "unit": UNIT,
        "cores": 1,
        "kind": "oracle",
        "sample": "one full FP64 oracle cycle (64^3 field solve + push/deposit) of the first %d particles "
                  "per species of the %s workload (%d live), %.1f s" % (sample_per_species, workload, kept, dt),
    }, s.particles()


def error_vs_oracle(workload, precision, sort_every, sample_per_species, oracle_state):
    """Largest relative error, after the first cycle, of the GPU state against
    the oracle's for the oracle's sample (the first sample_per_species inputs
    of each species).  Positions after one cycle depend only on the initial
    fields, so the oracle's smaller particle set does not matter."""
    import numpy as np
    import oracle as O
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R
    w = inputs.workload_params(workload)
    parts = inputs.workload_particles(workload, seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=sort_every, capacity=ntot,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    run = R.Run(cfg)
    slots, off = [], 0
    for sp, x, uc in parts:
        run.load(sp, x, uc)
        slots.append(off + np.arange(min(sample_per_species, x.shape[1])))
        off += x.shape[1]
    sp0 = run.particles()[2]
    run.step(1)
    x1, u1, sp1 = run.particles()
    run.close()
    slots = np.concatenate(slots)
    slots = slots[sp0[slots] != O.DEAD]  # the oracle keeps the same inputs, in input order
    xo, uo, spo = oracle_state
    live_o = spo != O.DEAD
    same_removal = bool(np.array_equal(sp1[slots] != O.DEAD, live_o))
    both = (sp1[slots] != O.DEAD) & live_o
    ex = np.abs(x1[:, slots][:, both] - xo[:, both]) / np.maximum(np.abs(xo[:, both]), 1.0)
    eu = np.abs(u1[:, slots][:, both] - uo[:, both]) / np.maximum(np.abs(uo[:, both]), 1.0)
    return {"x_rel": float(ex.max()), "u_rel": float(eu.max()), "particles": int(both.sum()),
            "same_removals": same_removal}


def measure(workload, precision, steps, warmup, sort_every):
    """Time `steps` cycles of one run; returns the figures of the timed region."""
    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    w = inputs.workload_params(workload)
    parts = inputs.workload_particles(workload, seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=sort_every, capacity=ntot,
                        precision=capi.FP32_MIXED if precision == "fp32" else capi.FP64)
    run = R.Run(cfg)
    for sp, x, uc in parts:
        run.load(sp, x, uc)
    del parts
    h = run.h
    capi.grpic_step(h, warmup)
    torch.cuda.synchronize()
    ps0 = capi.grpic_particle_steps(h)
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
    run.close()
    wall = t1 - t0
    psteps = ps1 - ps0
    return {
        "w": w, "ntot": ntot, "wall": wall, "psteps": psteps, "value": psteps / wall,
        "ms_per_step": wall * 1e3 / steps, "timers": timers,
        "kernel_ms_per_launch": {k: (v[0] / max(v[1], 1)) for k, v in timers.items()},
        "live_end": int(sum(d["n_alive"])),
    }


KERNELS = {
    "push": ("k_push (gather + RK4 pusher)", PUSH_FLOPS_PER_PARTICLE_STEP, "hbm_bytes_per_particle"),
    "deposit": ("k_deposit (zigzag, curved face-area weights, int64 current)", DEPOSIT_FLOPS_PER_PARTICLE,
                "deposit_hbm_bytes_per_particle"),
}


def kernel_roofline(m, name, peak, with_traffic):
    """Algorithmic FLOP/s of one kernel over its event-timed launches
    (particles per launch = particle-steps of the timed region / launches)."""
    label, flops, tkey = KERNELS[name]
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
        "traffic": read_traffic(per_launch, tkey) if with_traffic else None,
        "avg_launch_ms": avg_s * 1e3,
        "flops_per_particle": flops,
        "particles_per_launch": per_launch,
    }


def rooflines(m, peak, with_traffic):
    """Both particle kernels' rooflines and the one of the kernel that takes
    the most time (each launches once per cycle)."""
    both = {k: kernel_roofline(m, k, peak, with_traffic) for k in KERNELS}
    dominant = max(both, key=lambda k: both[k]["avg_launch_ms"])
    return both[dominant], both


def serving(args):
    """Continuous batching of independent FP32-mixed runs with Poisson
    arrivals.  A saturated probe (32 requests arriving at once) measures the
    loop's own capacity in particle-steps/s; the measured workload then
    arrives at 0.7 of that capacity."""
    from paper_0904_0232_amd import serve
    budget = int(args.serve_budget_gb * (1 << 30))

    def work(reqs):
        return sum(2 * r["ppc"] * r["edge"] ** 3 * r["steps"] for r in reqs) / len(reqs)

    probe = serve.serve(serve.make_requests(32, 1, 1e6), budget, args.serve_slots)
    capacity = probe["particle_steps_per_s"]
    log("serving probe: %.4g particle-steps/s saturated" % capacity)
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
                            B0=(0.0, 0.0, b0), species=w["species"], r_rm=w["r_rm"], sort_every=5, capacity=ntot,
                            precision=prec, center=w["center"], outer_layer=layer, outer_damp=0.3 if layer else 0.0)
        r = R.Run(cfg)
        for sp, x, uc in parts:
            r.load(sp, x, uc)
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
    divergence).  "geodesic" runs test particles with no field, "push" test
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
            del st
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="kerr64")
    ap.add_argument("--sort-every", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=3 << 19, help="particles per species for the oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-mixed measurement")
    ap.add_argument("--scale", action="store_true",
                    help="also time the 256^3 throughput workload (268M particles) in both precisions")
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

    import torch
    torch.cuda.set_device(0)

    m64 = measure(args.workload, "fp64", args.steps, args.warmup, args.sort_every)
    log("fp64 %s: %.4g particle-steps/s" % (args.workload, m64["value"]))
    w = m64["w"]
    roofline, rooflines64 = rooflines(m64, FP64_PEAK_TFLOPS, True)
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
            "workload": "%s: Kerr a=%.2fm, m=%g cells, %d^3 grid, %d particles (%d ppc x 2 species), "
                        "uniform Maxwellian u_th=%gc, B_z=%g, dt=%g, curved deposit, paper gamma, "
                        "sort every %d steps" % (args.workload, w["a_frac"], w["m"], w["n"], m64["ntot"], w["ppc"],
                                                 w["u_th"], w["B0"], w["dt"], args.sort_every),
            "precision": "fp64",
            "live_particles_end": m64["live_end"],
        },
        "kernel_ms_per_launch": m64["kernel_ms_per_launch"],
        "roofline": roofline,
        "rooflines": rooflines64,
        "cpu_baseline": None,
    }
    if not args.no_fp32:
        m32 = measure(args.workload, "fp32", args.steps, args.warmup, args.sort_every)
        log("fp32-mixed %s: %.4g particle-steps/s" % (args.workload, m32["value"]))
        line["fp32_mixed"] = {
            "value": m32["value"], "unit": UNIT, "ms_per_step": m32["ms_per_step"], "dtype": "f32 (FP64 quartic, "
            "near-horizon metric and diagnostics)", "kernel_ms_per_launch": m32["kernel_ms_per_launch"],
            "speedup_vs_fp64": m32["value"] / m64["value"], "live_particles_end": m32["live_end"],
        }
        line["fp32_mixed"]["roofline"], line["fp32_mixed"]["rooflines"] = rooflines(m32, FP32_PEAK_TFLOPS, False)
    if args.serve_runs > 0:
        line["serving"] = serving(args)
        log("serving: p50 %.3f s p99 %.3f s" % (line["serving"]["p50_latency_s"], line["serving"]["p99_latency_s"]))
    if args.scale:
        scale = {}
        for prec in ("fp32", "fp64"):
            # warm up past the first cell sort (loaded particles are in
            # generation order), as the main measurement does
            ms = measure("shell256", prec, 100, max(2, args.sort_every), args.sort_every)
            log("shell256 %s: %.4g particle-steps/s" % (prec, ms["value"]))
            scale[prec] = {"value": ms["value"], "ms_per_step": ms["ms_per_step"], "particles": ms["ntot"],
                           "kernel_ms_per_launch": ms["kernel_ms_per_launch"], "steps": 100,
                           "warmup": max(2, args.sort_every)}
        line["throughput_scale_shell256"] = scale
    if args.precision:
        line["precision_torus128"] = precision_study("torus128", n_override=args.precision_particles or None)
    if args.ablations:
        line["ablations_kerr64"] = ablation_study()
    if args.jet:
        line["jet"] = jet_study()
    if args.preemption:
        line["preemption"] = preemption_study(args)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], ostate = cpu_baseline(args.workload, args.cpu_sample)
        log("cpu baseline: %.4g particle-steps/s" % line["cpu_baseline"]["value"])
        errs = {"fp64": error_vs_oracle(args.workload, "fp64", args.sort_every, args.cpu_sample, ostate)}
        if not args.no_fp32:
            errs["fp32_mixed"] = error_vs_oracle(args.workload, "fp32", args.sort_every, args.cpu_sample, ostate)
        errs["what"] = ("largest relative error after the first cycle against the FP64 oracle, on the oracle's "
                        "sample (positions relative to max(|x|, 1 cell), four-velocities to max(|u|, c))")
        line["error_vs_oracle"] = errs
        log("error vs oracle: %s" % json.dumps(errs))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
