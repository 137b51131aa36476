"""bench.py's command line on the CPU: more than one GPU is refused with a
message (this build measures one GPU; the batches shard by ket-pair blocks)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _full_record_fixture():
    """A full bench record with every leg, at the sizes the real run produces
    (long floats everywhere), for the compact-line test."""
    import math
    f = lambda i: math.pi * 1e3 / (i + 7) + 1e-9 * i        # 17-digit floats
    names_hl = ["(ff|ff)", "(gg|gg)", "(s|dd)", "(p|dd)", "(d|dd)", "(f|dd)", "(g|dd)", "(h|dd)", "(i|dd)",
                "(hh|hh)", "(ii|ii)"]
    names_sp = ["(ss|ss)", "(ps|ss)", "(ps|ps)", "(pp|ss)", "(pp|ps)", "(pp|pp)"]
    leg = lambda i: {"shellsets": 65536, "ms_per_call": f(i), "kernel_ms": f(i + 1), "shellsets_per_s": f(i + 2),
                     "kernel_tflops": f(i + 3), "pct_fp64_peak": f(i + 4), "hbm_frac": f(i + 5),
                     "out_write_GB_per_s": f(i + 6), "variant": 2, "tuning_ms": {"1": f(i), "2": f(i + 1)}}
    extras = {"gradient": leg(0), "high_l": {n: leg(i) for i, n in enumerate(names_hl)},
              "sp_classes": {n: leg(i) for i, n in enumerate(names_sp)},
              "sp_hbm": {n: leg(i) for i, n in enumerate(names_sp)},
              "digest": {n: leg(i) for i, n in enumerate(names_sp + ["(dd|dd) K=3", "(pd|dd) K=3"])},
              "one_body": {n: leg(i) for i, n in enumerate(["(s|s)", "(p|p)", "(d|p)", "(d|d)", "(f|f)"])},
              "nuclear": {f"({a}|{b}) K={k}": leg(i) for i, (a, b, k) in enumerate(
                  [(a, b, k) for k in (1, 5) for a, b in ["ss", "ps", "pp", "ds", "dp", "dd", "fs", "fp", "ff"]])}}
    cluster = {"workload": "x" * 300, "quartets": 19111359, "plain_ms": f(1), "plain_tuned_ms": f(2),
               "fused_ms": f(3), "fused_speedup": f(4), "fusion_only_speedup": f(5), "pct_fp64_peak_fused": f(6),
               "fused_tuning": {f"c{i}": {"variant": 1, "ms": {"0": f(i)}} for i in range(21)},
               "parity_sample": {"checked": 368036, "failed": 0, "passed_only_by_QQ_clause": 3,
                                 "max_err_over_QQ": f(7), "reference": "__float128 oracle"}}
    per_class = {n: {"shellsets": 65536, "kernel_ms": f(i), "algorithmic_gflop": f(i + 1), "kernel_tflops": f(i + 2),
                     "pct_fp64_peak": f(i + 3), "shellsets_per_s_kernel": f(i + 4)}
                 for i, n in enumerate(["(dd|dd)", "(pd|dd)"])}
    return {
        "metric": "FP64 ERI shellsets/s + % FP64 peak per L-class; fused-batch vs per-class speedup",
        "value": f(0), "unit": "shellsets/s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": f(1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "y" * 200, "classes": ["(dd|dd)", "(pd|dd)"], "shellsets_per_step": 131072},
        "step_tflops_algorithmic": f(2), "step_pct_fp64_peak": f(3), "per_class": per_class,
        "tuning": {"(dd|dd)": {"variant": 2, "ms": {"1": f(1)}}},
        "roofline": {"bound": "mfma", "achieved": f(4), "peak": 78.6, "unit": "TFLOP/s", "frac": f(5),
                     "traffic": 9.1e8, "kernel": "eri_mfma_kernel (dd|dd) K=3, 65,536 shellsets per launch",
                     "flops_per_launch": f(6)},
        "cpu_baseline": {"value": f(7), "unit": "shellsets/s", "cores": 16, "kind": "oracle", "cpu_model": "z" * 48,
                         "sample": "224x224 shellsets of each class (first pairs of the workload), 100352 shellsets, "
                                   "15.3 s",
                         "single_thread": {"value": f(8), "cores": 1, "sample": "24x24 shellsets of each class"}},
        "parity_sample": {"checked": 50331648, "failed": 0, "max_abs_err": f(9), "max_rel_err_above_atol": f(10),
                          "tolerance": "t" * 60},
        "extras": extras, "mixed_cluster": cluster, "wall_s_timed": f(11)}


def test_compact_line_fits_and_keeps_the_headline():
    """The driver keeps only the tail of stdout: the printed line must stay
    well under 4 KB with every leg present, and keep the headline keys."""
    sys.path.insert(0, ROOT)
    import bench
    rec = bench.compact_record(_full_record_fixture(), "gpurun_out/bench_detail.json")
    line = json.dumps(rec, separators=(",", ":"))
    assert len(line) <= 4096, len(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "per_class", "mixed_cluster"):
        assert k in rec, k
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rec["roofline"], k
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in rec["cpu_baseline"], k
    assert rec["cpu_baseline"]["single_thread"]["cores"] == 1
    assert rec["mixed_cluster"]["parity"]["passed_only_by_QQ_clause"] == 3
    assert json.loads(line) == rec
