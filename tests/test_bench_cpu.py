"""bench.py's host-side bookkeeping: the profile summary built from
rocprofv3 CSV files (synthetic files with known durations and counters
here), and the refusal of more than one GPU."""
from __future__ import annotations

import csv
import json
import os
import subprocess
import sys

import bench

BLOCK = "void pm::ntt_block_kernel<true, 4, 256>(pm::NttLaunch)"
PW = "void pm::pointwise_mfma_kernel<256>(pm::PointwiseLaunch)"


def write_csv(path, fields, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_summary_averages_the_steady_steps_and_scales_the_counters(tmp_path):
    steps, warmup, steps_pmc = 20, 100, 3
    total = warmup + 2 * steps          # warm-up, timed loop, distribution loop
    trace, t = [], 0
    for s in range(total):
        steady = s >= total - 2 * steps
        for name, per_step, us in ((BLOCK, 2, 50 if steady else 100),
                                   (PW, 1, 30 if steady else 70)):
            for _ in range(per_step):
                trace.append({"Kernel_Name": name, "Start_Timestamp": t,
                              "End_Timestamp": t + us * 1000})
                t += us * 1000 + 500
    root = tmp_path / "out"
    write_csv(str(root / "st" / "st_kernel_trace.csv"),
              ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], trace)
    stats = []
    for name in (BLOCK, PW):
        d = [r["End_Timestamp"] - r["Start_Timestamp"] for r in trace if r["Kernel_Name"] == name]
        stats.append({"Name": name, "Calls": len(d), "AverageNs": sum(d) / len(d),
                      "TotalDurationNs": sum(d)})
    write_csv(str(root / "st" / "st_kernel_stats.csv"),
              ["Name", "Calls", "AverageNs", "TotalDurationNs"], stats)
    # counter runs: 1 + 2 (steps_pmc - 1) = 5 steps, the block kernel twice a step
    pmc_steps = 1 + 2 * (steps_pmc - 1)
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    write_csv(str(root / "f" / "f_counter_collection.csv"), fields,
              [{"Kernel_Name": BLOCK, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0}]
              * (2 * pmc_steps))
    write_csv(str(root / "w" / "w_counter_collection.csv"), fields,
              [{"Kernel_Name": BLOCK, "Counter_Name": "WRITE_SIZE", "Counter_Value": 500.0}]
              * (2 * pmc_steps))
    cal_bytes = 3 * (256 << 20) * 4
    copy = "copyBuffer"
    write_csv(str(root / "cf" / "cf_counter_collection.csv"), fields,
              [{"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE",
                "Counter_Value": cal_bytes / 2 / 1024}])
    write_csv(str(root / "cw" / "cw_counter_collection.csv"), fields,
              [{"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE",
                "Counter_Value": cal_bytes / 1024}])

    out = tmp_path / "profiles"
    bench.summarize_profiles(str(root), steps, warmup, steps_pmc, "tst", out_dir=str(out))
    t = json.load(open(out / "tst_traffic.json"))
    assert abs(t["fetch_scale"] - 2.0) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    # per step: 2 dispatches x (1000 KiB x 2 + 500 KiB x 1)
    assert abs(t["bytes_per_step"]["ntt_fwd"] - 2 * (2000 + 500) * 1024) < 1e-6
    assert "pointwise" not in t["bytes_per_step"]
    assert abs(t["device_ms_per_step"]["ntt_fwd"] - 0.100) < 1e-9
    assert abs(t["device_ms_per_step"]["pointwise"] - 0.030) < 1e-9
    md = open(out / "tst_kernels.md").read()
    row = [ln for ln in md.splitlines() if BLOCK in ln][0].split("|")
    assert int(row[2]) == 2 * total and float(row[4]) == 50.0   # calls, timed avg us
    assert t["source_hash"] == bench.source_hash()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_product_floor_matches_the_path_roofline_and_counts_lazy_butterflies():
    from paper_1905_04356_amd import binding as Bd
    p, m, n, k, d = 2013265921, 64, 64, 32, 4096
    plan = Bd.pm_plan(p, m, n, k, d, 4)
    kernels = {}
    for kind in ("ntt_fwd", "pointwise", "ntt_inv"):
        b, o = bench.kernel_work(kind, plan, p, m, n, k, d, 4)
        kernels[kind] = {"algorithmic_bytes": b, "ops": o}
    path = bench.path_roofline(kernels, plan, 1.0)
    assert abs(bench.product_floor_us(plan, m, n, k, d) - path["floor_us"]) < 1e-6
    assert bench.butterfly_ops(plan) == (10, 11)          # q >= 2^30: canonical
    lazy = Bd.pm_plan(998244353, m, n, k, d, 4)
    assert bench.butterfly_ops(lazy) == (8, 10)
    # three-quarter points lower the floor's bytes
    tr = Bd.pm_plan(998244353, 16, 16, 16, 1500, 4)
    assert tr.num_points == 3 << (tr.log2_len - 2)
    full = bench.product_floor_us(tr, 16, 16, 16, 1500)
    assert 0 < full < bench.product_floor_us(Bd.pm_plan(998244353, 16, 16, 16, 2040, 4),
                                             16, 16, 16, 2040)
