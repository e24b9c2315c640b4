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
prices the dominant kernel (the pusher) by its algorithmic FP64 operation
count per particle-step against the MI355X FP64 vector peak, with the
average kernel time measured by HIP events on the run's stream.  The CPU
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
HBM_PEAK_GBS = 8000.0

# Algorithmic FP64 operations of one particle-step of the pusher (one call of
# the RK4 step: four stages of radius quartic, Kerr-Schild gradients,
# Christoffel contraction, trilinear gather of 16 components, Lorentz term,
# paper gamma estimate and stage update, plus the final combination).  An FMA
# counts as 2, a division or square root as 1.  The breakdown is derived in
# the design notes from the kernel source.
PUSH_FLOPS_PER_PARTICLE_STEP = 2219

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_push_kerr64_traffic.txt")
PUSH_SOURCES = [os.path.join(ROOT, "paper_0904_0232_amd", "csrc", f) for f in ("particles.hip", "grpic_dev.h")]


def push_source_hash():
    h = hashlib.sha256()
    for f in PUSH_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(n_per_launch):
    """HBM bytes per push launch from the committed rocprofv3 counter summary,
    or None when the summary is missing or the kernel source changed since."""
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
        per_particle = float(kv["hbm_bytes_per_particle"])
    except (KeyError, ValueError):
        return None
    return per_particle * n_per_launch


def cpu_baseline(workload, sample_per_species):
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
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="kerr64")
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=1 << 20, help="particles per species for the oracle timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the GRPIC path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not a measured path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0904_0232_amd import capi, inputs
    from paper_0904_0232_amd import run as R

    torch.cuda.set_device(0)
    w = inputs.workload_params(args.workload)
    parts = inputs.workload_particles(args.workload, seed=0)
    ntot = sum(p[1].shape[1] for p in parts)
    cfg = R.make_config(w["n"], m=w["m"], a=w["a"], dt=w["dt"], B0=(0.0, 0.0, w["B0"]), species=w["species"],
                        r_rm=w["r_rm"], sort_every=args.sort_every, capacity=ntot)
    run = R.Run(cfg)
    for sp, x, uc in parts:
        run.load(sp, x, uc)
    h = run.h
    capi.grpic_step(h, args.warmup)
    torch.cuda.synchronize()
    ps0 = capi.grpic_particle_steps(h)
    capi.grpic_set_timing(h, True)
    capi.grpic_read_timing(h)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    capi.grpic_step(h, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timers = capi.grpic_read_timing(h)
    capi.grpic_set_timing(h, False)
    ps1 = capi.grpic_particle_steps(h)
    wall = t1 - t0
    psteps = ps1 - ps0
    value = psteps / wall
    d = run.diag()

    push_ms, push_n = timers["push"]
    avg_push_s = push_ms / 1e3 / max(push_n, 1)
    per_launch = psteps / max(push_n, 1)
    flops_per_launch = PUSH_FLOPS_PER_PARTICLE_STEP * per_launch
    achieved = flops_per_launch / avg_push_s / 1e12
    traffic = read_traffic(per_launch)
    roofline = {
        "kernel": "k_push (gather + RK4 pusher)",
        "bound": "alu",
        "achieved": achieved,
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": traffic,
        "avg_launch_ms": avg_push_s * 1e3,
        "flops_per_particle_step": PUSH_FLOPS_PER_PARTICLE_STEP,
    }
    per_step = {k: (v[0] / max(v[1], 1)) for k, v in timers.items()}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "%s: Kerr a=%.2fm, m=%g cells, %d^3 grid, %d particles (%d ppc x 2 species), "
                        "uniform Maxwellian u_th=%gc, B_z=%g, dt=%g, curved deposit, paper gamma, "
                        "sort every %d steps" % (args.workload, w["a_frac"], w["m"], w["n"], ntot, w["ppc"],
                                                 w["u_th"], w["B0"], w["dt"], args.sort_every),
            "precision": "fp64",
            "live_particles_end": int(sum(d["n_alive"])),
        },
        "kernel_ms_per_launch": per_step,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    run.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_sample)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
