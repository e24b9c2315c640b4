"""Host-side pieces of bench.py (no GPU): the roofline arithmetic of the
JSON line, the committed traffic summaries it reads, the workload
description, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _fake_measure(push_ms=26.0, deposit_ms=18.0, launches=10, particles=2.5e8):
    return {"timers": {"push": (push_ms * launches, launches), "deposit": (deposit_ms * launches, launches),
                       "fields": (2.0 * 3 * launches, 3 * launches), "sort": (17.0 * 2, 2)},
            "psteps": particles * launches}


def test_roofline_is_algorithmic_flops_over_launch_time():
    m = _fake_measure()
    dom, both = bench.rooflines(m, bench.FP64_PEAK_TFLOPS, False, "shell256", "fp64")
    assert dom["kernel"].startswith("k_push") and dom is both["push"]
    want = bench.PUSH_FLOPS_PER_PARTICLE_STEP * 2.5e8 / 26.0e-3 / 1e12
    assert abs(dom["achieved"] - want) < 1e-9 * want
    assert abs(dom["frac"] - want / 78.6) < 1e-12
    assert dom["bound"] == "alu" and dom["unit"] == "TFLOP/s" and dom["traffic"] is None
    dep = both["deposit"]
    assert abs(dep["achieved"] - bench.DEPOSIT_FLOPS_PER_PARTICLE * 2.5e8 / 18.0e-3 / 1e12) < 1e-6
    # the dominant kernel is the one with the longest launches
    dom2, _ = bench.rooflines(_fake_measure(push_ms=10.0, deposit_ms=18.0), 157.3, False, "shell256", "fp32")
    assert dom2["kernel"].startswith("k_deposit32")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_traffic_summaries_parse(precision):
    path = bench.traffic_file(precision, "shell256")
    assert os.path.exists(path), path
    kv = {}
    with open(path) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    for k in ("source_sha", "fetch_scale", "write_scale", "hbm_bytes_per_particle", "deposit_hbm_bytes_per_particle"):
        assert k in kv, k
    assert float(kv["hbm_bytes_per_particle"]) > 0 and float(kv["deposit_hbm_bytes_per_particle"]) > 0
    # read_traffic scales the per-particle bytes when the kernel sources match
    # the measured build, and gives None otherwise
    t = bench.read_traffic(2.0, precision, "shell256")
    if kv["source_sha"] == bench.kernel_source_hash(precision):
        assert t == pytest.approx(2.0 * float(kv["hbm_bytes_per_particle"]))
    else:
        assert t is None
    assert bench.read_traffic(1.0, precision, "no_such_workload") is None


def test_describe_names_the_workload_and_its_sizes():
    from paper_0904_0232_amd import inputs
    w = inputs.workload_params("shell256")
    text = bench.describe("shell256", w, 268435456, 5, 4)
    assert text.startswith("shell256:") and "256^3" in text and "268435456" in text and "4^3" in text


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
