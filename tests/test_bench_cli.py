"""The bench's driver-facing output: the last stdout line is a short JSON
record with the headline, its roofline and the CPU baseline (the full record
goes to a file), and more than one GPU is refused.  CPU only."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

REQUIRED = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "settle_s", "ms_per_step", "dtype",
            "config", "roofline", "cpu_baseline", "bf16_mfma_vs_fp32")


def _full_record():
    variant = {"ms_per_step": 0.25, "subcarriers_per_s": 1.5e8, "call_ms_mean": 0.245,
               "call_ms_median_single": 0.26, "call_ms_p10_single": 0.25, "call_ms_p90_single": 0.27,
               "alg_GBps": 5500.0, "hbm_frac": 0.69, "fp64_routed": 0,
               "parity_max_rel_err_z": 1.0e-6, "parity_max_sigma2_db": 1e-6,
               "frac_of_read_ceiling": 0.9}
    variants = {f"{m}_{p}": dict(variant) for m, p in bench.VARIANTS}
    other = {f"workload_{k}": dict(variant, extra="x" * 200) for k in range(120)}
    return {
        "metric": "equalized subcarriers/s @B=256,U=16,C=8: FP32 vs BF16-MFMA; % HBM roofline",
        "value": 1.5e8, "unit": "subcarriers/s", "n_gpus": 1, "steps": 20, "warmup": 5, "settle_s": 0.2,
        "ms_per_step": 0.25, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "PD L-MMSE, B=256 antennas in C=8 clusters of 32, U=16, 38400 systems",
                   "B": 256, "C": 8, "U": 16, "systems_per_step": 38400, "form": "pd_fp32"},
        "roofline": {"bound": "hbm", "achieved": 5500.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.69,
                     "traffic": 1.3449e9, "kernel": "eq_forward_kernel<16, FP32, PD>",
                     "alg_bytes_per_launch": 1344307200, "alg_bytes_per_system": 35008,
                     "read_ceiling_GBps": 6200.0, "frac_of_read_ceiling": 0.89},
        "variants": variants,
        "bf16_mfma_vs_fp32": {m: {"form": f"{m}_bf16x3", "speedup": 1.05, "hbm_frac": 0.72,
                                  "frac_of_read_ceiling": 0.93, "parity_max_rel_err_z": 5e-6,
                                  "fp32_parity_max_rel_err_z": 1e-6} for m in ("pd", "fd")},
        "other_workloads": other,
        "cpu_baseline": {"value": 3.0e5, "unit": "subcarriers/s", "cores": 16, "kind": "oracle",
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor",
                         "sample": "PD L-MMSE complex128 NumPy oracle, 16 processes x 1 thread " + "x" * 100},
    }


def test_compact_line_is_short_and_complete():
    full = _full_record()
    assert len(json.dumps(full)) > 20000
    line = json.dumps(bench.compact_record(full, os.path.join(ROOT, "gpurun_out", "bench_full.json")))
    assert "\n" not in line
    # the driver keeps the last 2,000 characters of the output
    assert len(line) < 1950, len(line)
    rec = json.loads(line)
    for k in REQUIRED:
        assert k in rec, k
    assert "workload" in rec["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rec["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample", "cpu_model"):
        assert k in rec["cpu_baseline"], k
    assert "other_workloads" not in rec and "variants" not in rec
    assert set(rec["forms"]) == {f"{m}_{p}" for m, p in bench.VARIANTS}
    assert rec["full_record"] == "gpurun_out/bench_full.json"


def test_cpu_cores_capped():
    n = bench.cpu_cores()
    assert 1 <= n <= 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "--gpus must be 1" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes():
    # read H (B U complex64) and y once, write z (complex64) and sigma2 (float32)
    assert bench.bytes_per_system(256, 16) == 256 * 16 * 8 + 256 * 8 + 16 * 8 + 16 * 4 == 35008
    assert bench.bytes_per_system(1024, 32) == 270720
    # several vectors: S receive vectors in, S estimates out, one sigma2 row
    assert bench.bytes_per_system_sym(256, 16, 14) == 256 * 16 * 8 + 14 * 256 * 8 + 14 * 16 * 8 + 16 * 4 == 63296
