"""Benchmark: polynomial-matrix products mod p on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2]

A step is one full product A(x) B(x) mod p through the C ABI (forward
transforms, pointwise matrix products, inverse transform, and Chinese
remaindering when the modulus needs it), on inputs already resident in HBM.
The default workload is the PM-basis-shaped product of the paper's
multiplication experiments scaled to one GPU: A 64x64, B 64x32, degree < 4096,
p = 2013265921, uint32 residues.

Prints one JSON line with throughput in m*n*k*d coefficient-MACs per second,
per-kernel device times measured with HIP events on the library's stream, the
roofline of the dominant kernel, and the CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts.
HBM_PEAK_GBS = 8000.0
INT8_MFMA_PEAK_TOPS = 5000.0          # dense int8, 5.0 POP/s
CUS, LANES, CLOCK_GHZ = 256, 64, 2.4
VALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0   # 39.3 T 32-bit lane-ops/s

# 32-bit VALU operations of one radix-2 butterfly with canonical residues and
# Shoup multiplication: modular add (add, sub, min), modular difference
# (sub, add), product by the twiddle (mul_hi, mul_lo, mul_lo, sub) and its
# final correction (sub, min).
OPS_PER_BUTTERFLY = 11

WORKLOADS = {
    # name: (p, m, n, k, d, elem dtype)
    "c1": (998244353, 8, 8, 8, 256, "u32"),
    "c2": (2013265921, 64, 64, 32, 4096, "u32"),
    "c4": (None, 32, 32, 32, 2048, "u64"),   # seeded 60-bit prime
}


def workload_params(name):
    from paper_1905_04356_amd import inputs as I
    p, m, n, k, d, dt = WORKLOADS[name]
    if p is None:
        p = I.seeded_prime_60(4)
    return p, m, n, k, d, dt


def kernel_work(kind, plan, p, m, n, k, d, eb):
    """Algorithmic work of all launches of one kernel kind in one product:
    (bytes, ops, ops_unit, peak, bound)."""
    L = 1 << plan.log2_len
    r = plan.num_primes
    logL = plan.log2_len
    if kind == "ntt_fwd":
        E = m * n + n * k
        byts = eb * d * E + 4 * L * E * r
        ops = OPS_PER_BUTTERFLY * (L // 2) * logL * E * r
        return byts, ops
    if kind == "ntt_inv":
        E = m * k
        out_b = eb if plan.mode == 0 else 4
        byts = 4 * L * E * r + out_b * (2 * d - 1) * E * r
        ops = OPS_PER_BUTTERFLY * (L // 2) * logL * E * r
        return byts, ops
    if kind == "pointwise":
        byts = 4 * L * (m * n + n * k + m * k) * r
        macs = L * m * n * k * r
        return byts, macs
    if kind == "crt":
        cnt = (2 * d - 1) * m * k
        return 4 * r * cnt + eb * cnt, cnt
    return 0, 0


def roofline_for(kind, byts, ops, seconds, plan):
    if kind in ("ntt_fwd", "ntt_inv"):
        achieved = ops / seconds / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "Tops/s (32-bit VALU lane-ops)", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": None, "kernel": kind,
                "hbm_GBs": byts / seconds / 1e9,
                "hbm_frac": byts / seconds / 1e9 / HBM_PEAK_GBS}
    if kind == "pointwise":
        if plan.pointwise == 1:
            achieved = 32.0 * ops / seconds / 1e12   # 16 int8 limb products, 2 ops each
            return {"bound": "mfma", "achieved": achieved, "peak": INT8_MFMA_PEAK_TOPS,
                    "unit": "TOP/s (int8)", "frac": achieved / INT8_MFMA_PEAK_TOPS,
                    "traffic": None, "kernel": kind,
                    "hbm_GBs": byts / seconds / 1e9,
                    "hbm_frac": byts / seconds / 1e9 / HBM_PEAK_GBS}
        achieved = byts / seconds / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kind,
                "mod_macs_per_s": ops / seconds}
    achieved = byts / seconds / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": kind}


def cpu_baseline(p, A, B, m, n, k, d, target_s):
    """The oracle's schoolbook on whole output entries of the same product,
    scaled to the metric's unit (m*n*k*d per full product)."""
    from oracle import oracle as O
    from paper_1905_04356_amd import inputs as I
    threads = min(16, O.host_threads())
    pairs = I.sample_pairs(12345, m, k, m * k)
    t0 = time.perf_counter()
    O.polymatmul_entries(p, A, B, pairs[:threads], threads=threads)
    t_probe = time.perf_counter() - t0
    want = int(threads * max(1.0, target_s / max(t_probe, 1e-3)))
    count = max(threads, min(m * k, (want // threads) * threads))
    t0 = time.perf_counter()
    O.polymatmul_entries(p, A, B, pairs[:count], threads=threads)
    dt = time.perf_counter() - t0
    return {"value": count * n * d / dt, "unit": "coefficient-MAC/s (m*n*k*d per product)",
            "cores": threads, "kind": "oracle",
            "sample": f"{count} of {m * k} whole output entries (all {2 * d - 1} coefficients, "
                      f"schoolbook) of the same product, {dt:.2f} s wall",
            "seconds": dt}


def bench_batched(steps, warmup, seed=3, count=512, p=998244353):
    """Config 3: `count` products with the batched shape rule, all in one
    batched call per step, against one pm_mul call per product on the same
    stream (same inputs, outputs, device)."""
    import torch

    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat

    dev = torch.device("cuda:0")
    shapes = I.batched_shapes(seed, count)
    As = [I.polymat_torch(seed, i, I.TENSOR_A, p, d, m, n, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    Bs = [I.polymat_torch(seed, i, I.TENSOR_B, p, d, n, k, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    outs = [torch.empty((2 * d - 1, m, k), dtype=torch.uint32, device=dev)
            for (m, n, k, d) in shapes]
    work = float(sum(m * n * k * d for (m, n, k, d) in shapes))
    stream = torch.cuda.current_stream()
    wsb = polymat.Workspace(dev)
    for _ in range(warmup):
        polymat.mul_batched(p, As, Bs, outs, workspace=wsb, stream=stream)
    torch.cuda.synchronize()
    Bd.pm_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        polymat.mul_batched(p, As, Bs, outs, workspace=wsb, stream=stream)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    kb = Bd.pm_profile_end()
    batched_ws = wsb.buf.numel()
    del wsb
    wss = polymat.Workspace(dev)
    for _ in range(warmup):
        for A, B, C in zip(As, Bs, outs):
            polymat.mul(p, A, B, out=C, workspace=wss, stream=stream)
    torch.cuda.synchronize()
    Bd.pm_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        for A, B, C in zip(As, Bs, outs):
            polymat.mul(p, A, B, out=C, workspace=wss, stream=stream)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / steps
    ks = Bd.pm_profile_end()
    return {"workload": f"{count} products, (m,k) uniform over pairs of {{4..128}} with k<=m, "
                        f"n uniform, degrees log-uniform in [32, 8192], mod {p}, seed {seed}",
            "value": work / t_b, "unit": "coefficient-MAC/s", "ms_per_batch": t_b * 1e3,
            "device_ms_per_batch": kb["batched"][0] / steps,
            "one_per_call_value": work / t_s, "one_per_call_ms": t_s * 1e3,
            "speedup_vs_one_per_call": t_s / t_b, "sum_mnkd": work,
            "batched_workspace_GB": batched_ws / 1e9, "steps": steps, "warmup": warmup,
            "batched_kernel_ms": {kk: v[0] / steps for kk, v in kb.items() if v[1]},
            "one_per_call_kernel_ms": {kk: v[0] / steps for kk, v in ks.items() if v[1]}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build runs every product on a single "
              "MI355X and has no multi-GPU path (see the sharding design).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat

    p, m, n, k, d, dt = workload_params(args.workload)
    npdt = np.uint32 if dt == "u32" else np.uint64
    eb = 4 if dt == "u32" else 8
    plan = Bd.pm_plan(p, m, n, k, d, eb)
    A = I.polymat(2, 0, I.TENSOR_A, p, d, m, n, npdt)
    B = I.polymat(2, 0, I.TENSOR_B, p, d, n, k, npdt)
    dev = torch.device("cuda:0")
    tA = torch.from_numpy(A).to(dev)
    tB = torch.from_numpy(B).to(dev)
    tC = torch.empty((2 * d - 1, m, k), dtype=tA.dtype, device=dev)
    ws = polymat.Workspace(dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream)
    torch.cuda.synchronize()

    Bd.pm_profile_begin()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstats = Bd.pm_profile_end()

    wall = t1 - t0
    work = float(m) * n * k * d
    value = work * args.steps / wall
    kernels = {}
    for kind, (ms, launches) in kstats.items():
        if launches == 0:
            continue
        byts, ops = kernel_work(kind, plan, p, m, n, k, d, eb)
        sec = ms / 1e3 / args.steps           # device seconds per product
        kernels[kind] = {"ms_per_step": ms / args.steps, "launches_per_step":
                         launches / args.steps, "algorithmic_bytes": byts,
                         "ops": ops}
        kernels[kind]["roofline"] = roofline_for(kind, byts, ops, sec, plan)
    dominant = max(kernels, key=lambda kk: kernels[kk]["ms_per_step"])
    roof = dict(kernels[dominant]["roofline"])

    out = {
        "metric": "polymatrix mul mod p: m*n*k*d coefficient-MACs/s",
        "value": value,
        "unit": "coefficient-MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "device_ms_per_step": ev0.elapsed_time(ev1) / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic: seeded uniform residues in [0, p) (splitmix64)",
        "config": {"workload": f"{m}x{n}.{n}x{k} polynomial matrices, degree<{d}, mod {p}",
                   "p": p, "m": m, "n": n, "k": k, "d": d,
                   "L": 1 << plan.log2_len, "mode": "direct" if plan.mode == 0 else "crt",
                   "primes": plan.num_primes,
                   "pointwise": "mfma_int8" if plan.pointwise == 1 else "valu"},
        "roofline": roof,
        "kernels": kernels,
    }
    del tA, tB, tC, ws
    torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(args.batched_steps, 1)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, A, B, m, n, k, d, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
