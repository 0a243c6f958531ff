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
XCDS = 8
VALU_PEAK_TOPS = CUS * LANES * CLOCK_GHZ / 1000.0   # 39.3 T 32-bit lane-ops/s

PROFILE_EVERY = 4        # kernel timing on every 4th step of the timed loop

# 32-bit VALU operations of one radix-2 butterfly with canonical residues
# (q may exceed 2^30, so no lazy reduction) and Shoup multiplication, whose
# product a*w - floor(a*w'/2^32)*q mod 2^32 takes mul_hi, mul_lo and one
# v_mad_u64_u32 (with 2^32 - q), plus the final correction (sub, min):
#   forward (DIF): modular add (add, sub, min), difference plus q (sub, add),
#     product (3) and correction (2): 10;
#   inverse (DIT): product (3), correction (2), modular add (3), modular
#     difference (sub, add, min): 11.
OPS_FWD_BUTTERFLY = 10
OPS_INV_BUTTERFLY = 11

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


def garner_ops(r):
    """VALU instructions of one reconstruction from r residues: r (r-1) / 2
    Garner steps (Barrett correction 3, modular difference 3, Shoup product
    5) and the sum of r digit products mod p (about 12 each)."""
    return 11 * r * (r - 1) // 2 + 12 * r


def butterfly_ops(plan):
    """VALU operations per forward and inverse butterfly: Shoup's butterflies
    on canonical residues (10, 11), or Harvey's lazy ones (8, 10) where every
    prime of the plan is below 2^30."""
    if all(2 * plan.primes[i] - 1 <= 0x7F7F7F7F for i in range(plan.num_primes)):
        return 8, 10
    return OPS_FWD_BUTTERFLY, OPS_INV_BUTTERFLY


def kernel_work(kind, plan, p, m, n, k, d, eb, crt_folded=False):
    """Algorithmic work of all launches of one kernel kind in one product:
    (bytes, ops). crt_folded: CRT mode with the reconstruction done by the
    last inverse pass (no residue arrays; its operations count there)."""
    L = 1 << plan.log2_len
    r = plan.num_primes
    logL = plan.log2_len
    of, oi = butterfly_ops(plan)
    if kind == "ntt_fwd":
        E = m * n + n * k
        byts = eb * d * E + 4 * L * E * r
        ops = of * (L // 2) * logL * E * r
        return byts, ops
    if kind == "ntt_inv":
        E = m * k
        if crt_folded:
            byts = 4 * L * E * r + eb * (2 * d - 1) * E
            ops = oi * (L // 2) * logL * E * r + garner_ops(r) * (2 * d - 1) * E
            return byts, ops
        out_b = eb if plan.mode == 0 else 4
        byts = 4 * L * E * r + out_b * (2 * d - 1) * E * r
        ops = oi * (L // 2) * logL * E * r
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


def path_roofline(kernels, plan, device_ms):
    """Roofline of the whole path: the sum over kernel kinds of the larger of
    (algorithmic bytes at peak HBM bandwidth) and (algorithmic operations at
    the peak of the unit that executes them), against the measured device
    time of one product."""
    floor_s = 0.0
    for kind, kk in kernels.items():
        t_hbm = kk["algorithmic_bytes"] / (HBM_PEAK_GBS * 1e9)
        if kind in ("ntt_fwd", "ntt_inv"):
            t_ops = kk["ops"] / (VALU_PEAK_TOPS * 1e12)
        elif kind == "pointwise" and plan.pointwise == 1:
            t_ops = 32.0 * kk["ops"] / (INT8_MFMA_PEAK_TOPS * 1e12)
        else:
            t_ops = 0.0
        floor_s += max(t_hbm, t_ops)
    return {"floor_us": floor_s * 1e6, "measured_us": device_ms * 1e3,
            "frac": floor_s * 1e6 / (device_ms * 1e3)}


def product_floor_us(plan, m, n, k, d, eb=4):
    """The path floor of one product (as path_roofline) at the points its
    plan evaluates: 3L/4 for three-quarter transforms, 2^j for the wrapped
    form (its short top product left out); butterflies at Harvey's lazy
    counts (8 forward, 10 inverse) where every prime is below 2^30; in CRT
    mode the reconstruction is taken as folded into the last inverse pass
    (its operations there, no residue arrays)."""
    logL = plan.wrap_log2_len or plan.log2_len
    L = 1 << logL
    pts = L if plan.wrap_log2_len else plan.num_points
    r = plan.num_primes
    of, oi = butterfly_ops(plan)
    bfly = (L // 2) * logL * pts / L          # butterflies per transform
    ef, ei, ep = m * n + n * k, m * k, m * n + n * k + m * k
    hbm, valu = HBM_PEAK_GBS * 1e3, VALU_PEAK_TOPS * 1e6   # bytes, ops per us
    cnt = (2 * d - 1) * ei
    garner = garner_ops(r) * cnt if plan.mode == 1 else 0
    t = max((eb * d * ef + 4 * pts * ef * r) / hbm, of * bfly * ef * r / valu)
    t += max((4 * pts * ei * r + eb * cnt) / hbm, (oi * bfly * ei * r + garner) / valu)
    pw_ops = 32.0 * pts * m * n * k * r / (INT8_MFMA_PEAK_TOPS * 1e6) if plan.pointwise == 1 else 0
    t += max(4 * pts * ep * r / hbm, pw_ops)
    return t


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
    macs = count * n * d * d            # schoolbook: d^2 coefficient MACs per (i, l, j)
    return {"value": count * n * d / dt, "unit": "coefficient-MAC/s (m*n*k*d per product)",
            "cores": threads, "kind": "oracle",
            "sample": f"{count} of {m * k} whole output entries (all {2 * d - 1} coefficients, "
                      f"schoolbook) of the same product, {dt:.2f} s wall",
            "seconds": dt, "schoolbook_mac_per_s": macs / dt,
            "extrapolated_full_product_s": dt * (m * k) / count}


def bench_middle(steps=10, warmup=2, seed=6, p=2013265921, m=64, n=64, k=32, c=4096,
                 dd=4096):
    """Residual of Algorithm PM-Basis at order c + dd: an m x m basis of degree
    <= c times the m x n series truncated at order c + dd, coefficients
    c .. c + dd - 1 (the paper's MiddleProduct).  pm_middle against the whole
    product of the same operands (both padded to c + dd coefficients) and a
    slice, on the same stream; outputs compared."""
    import torch
    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    P1 = I.polymat_torch(seed, 0, I.TENSOR_A, p, c + 1, m, n, dev)
    F = I.polymat_torch(seed, 0, I.TENSOR_B, p, c + dd, n, k, dev)
    P1pad = torch.zeros((c + dd, m, n), dtype=P1.dtype, device=dev)
    P1pad[:c + 1] = P1
    ws = polymat.Workspace(dev)
    out = torch.empty((dd, m, k), dtype=P1.dtype, device=dev)
    full = torch.empty((2 * (c + dd) - 1, m, k), dtype=P1.dtype, device=dev)

    def run_mid():
        polymat.middle(p, P1, F, c, dd, out=out, workspace=ws, stream=stream)

    def run_full():
        polymat.mul(p, P1pad, F, out=full, workspace=ws, stream=stream)
        return full[c:c + dd]

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    t_mid = timed(run_mid)
    t_full = timed(run_full)
    same = bool(torch.equal(out, run_full()))
    torch.cuda.synchronize()
    plan_mid = Bd.pm_middle_plan(p, m, n, k, c + 1, c + dd, c, dd, 4)
    plan_full = Bd.pm_plan(p, m, n, k, c + dd, 4)
    del P1, F, P1pad, out, full, ws
    return {"workload": f"PM-Basis residual: {m}x{n} basis of degree <= {c} times {n}x{k} "
                        f"series of order {c + dd}, coefficients {c}..{c + dd - 1}, mod {p}",
            "middle_ms": t_mid, "whole_product_then_slice_ms": t_full,
            "speedup": t_full / t_mid, "middle_L": 1 << plan_mid.log2_len,
            "whole_L": 1 << plan_full.log2_len, "outputs_equal": same}


def bench_pmbasis(p=786433, seed=7):
    """Algorithm PM-Basis (approximant bases) driven through the GPU middle
    products, on the two table sizes of the paper that fit transforms of at
    most 2^15 points, mod a 20-bit FFT prime (786433 = 3 2^18 + 1), zero
    shift, F seeded uniform; one warm-up run, then one timed run each."""
    import torch
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import pmbasis as PB
    dev = torch.device("cuda")
    rows = []
    for (m, n, sigma, T) in [(32, 16, 8192, 8), (128, 64, 2048, 1)]:
        F = I.polymat_torch(seed, 0, I.TENSOR_A, p, sigma, m, n, dev)
        PB.PMBasis(p, T)(F[:64], 64, [0] * m)
        pm = PB.PMBasis(p, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, rd = pm(F, sigma, [0] * m)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rows.append({"m": m, "n": n, "order": sigma, "threshold": T, "seconds": dt,
                     "leaf_seconds": pm.leaf_seconds, "leaves": pm.leaves,
                     "basis_degree": int(P.shape[0]) - 1})
        del F, P
    # sixteen independent instances in lockstep (batched windows, leaves on
    # the device, one workgroup per instance) against the same with leaves on
    # a host thread pool and against one run after another
    m, n, sigma, T, K = 32, 16, 2048, 8, 16
    Fs = [I.polymat_torch(seed + 1 + i, 0, I.TENSOR_A, p, sigma, m, n, dev) for i in range(K)]
    PB.PMBasisMany(p, T)([F[:64] for F in Fs], 64, [[0] * m] * K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    PB.PMBasisMany(p, T)(Fs, sigma, [[0] * m] * K)
    torch.cuda.synchronize()
    t_many = time.perf_counter() - t0
    t0 = time.perf_counter()
    PB.PMBasisMany(p, T, device_leaf_min=1 << 30)(Fs, sigma, [[0] * m] * K)
    torch.cuda.synchronize()
    t_many_host = time.perf_counter() - t0
    t0 = time.perf_counter()
    for F in Fs:
        PB.PMBasis(p, T)(F, sigma, [0] * m)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    del Fs
    return {"workload": f"PM-Basis, F m x n of order sigma, mod {p}, zero shift", "runs": rows,
            "lockstep": {"instances": K, "m": m, "n": n, "order": sigma, "threshold": T,
                         "lockstep_seconds": t_many, "lockstep_host_leaves_seconds": t_many_host,
                         "one_after_another_seconds": t_seq}}


def bench_newton(p=2013265921, n=32, da=2049, N=4096, rhs=64, seed=8):
    """Truncated inverse S = A^{-1} mod x^N by Newton iteration (GPU middle
    products), then S as a multiplier class: `rhs` products S b_i
    (b_i: n x 1, N coefficients) in one batched call with S's evaluations
    computed once, against the same batch transforming S every time."""
    import torch
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import newton
    from paper_1905_04356_amd import polymat
    dev = torch.device("cuda")
    A = I.polymat_torch(seed, 0, I.TENSOR_A, p, da, n, n, dev)
    newton.truncated_inverse(p, A[:8], 64)               # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Sx = newton.truncated_inverse(p, A, N)
    torch.cuda.synchronize()
    t_inv = time.perf_counter() - t0
    Bs = [I.polymat_torch(seed, 1 + i, I.TENSOR_B, p, N, n, 1, dev) for i in range(rhs)]
    ws = polymat.Workspace(dev)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3

    t_eval = timed(lambda: newton.evaluations(p, Sx), reps=1)
    Se = newton.evaluations(p, Sx)
    t_reuse = timed(lambda: polymat.mul_batched(p, [Sx] * rhs, Bs, workspace=ws,
                                                A_evals=[Se] * rhs))
    t_plain = timed(lambda: polymat.mul_batched(p, [Sx] * rhs, Bs, workspace=ws))
    del A, Sx, Bs, Se, ws
    return {"workload": f"truncated inverse of a {n}x{n} matrix of degree < {da} mod x^{N}, "
                        f"mod {p}; then {rhs} products by it ({n}x1 right sides)",
            "newton_s": t_inv, "eval_once_ms": t_eval, "products_reusing_evals_ms": t_reuse,
            "products_transforming_S_ms": t_plain, "reuse_speedup": t_plain / t_reuse}


def bench_vdm(p=1000000007, seed=9, reps=10):
    """Products mod a prime without roots of unity of the needed order
    (10^9 + 7: 2 is the only power of 2 dividing p - 1): Vandermonde
    evaluation/interpolation on the matrix cores (pm_mul_vdm_u32) and
    evaluation/interpolation at a geometric progression (pm_mul_geo_u32)
    against the three-prime CRT transforms (a one-product pm_mul_batched
    call, which always takes the transforms), same operands, outputs
    compared."""
    import torch
    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for (m, n, k, d) in [(32, 32, 32, 16), (32, 32, 32, 64), (128, 128, 128, 64),
                         (32, 32, 32, 256), (128, 128, 128, 256), (32, 32, 32, 1024),
                         (128, 128, 128, 1024)]:
        A = I.polymat_torch(seed, 0, I.TENSOR_A, p, d, m, n, dev)
        B = I.polymat_torch(seed, 0, I.TENSOR_B, p, d, n, k, dev)
        ws = polymat.Workspace(dev)
        outv = torch.empty((2 * d - 1, m, k), dtype=A.dtype, device=dev)
        outc = torch.empty_like(outv)
        outg = torch.empty_like(outv)
        plan = Bd.pm_plan(p, m, n, k, d, 4)

        def timed(fn):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        t_v = timed(lambda: polymat.mul_vdm(p, A, B, out=outv, workspace=ws, stream=stream))
        t_c = timed(lambda: polymat.mul_batched(p, [A], [B], [outc], workspace=ws,
                                                stream=stream))
        t_g = timed(lambda: polymat.mul_geo(p, A, B, out=outg, workspace=ws, stream=stream))
        rows.append({"m": m, "n": n, "k": k, "d": d, "vandermonde_ms": t_v, "crt_ms": t_c,
                     "geometric_ms": t_g,
                     "crt_primes": plan.num_primes, "crt_L": 1 << plan.log2_len,
                     "outputs_equal": bool(torch.equal(outv, outc) and torch.equal(outg, outc))})
        del A, B, ws, outv, outc, outg
    return {"workload": f"products mod {p} (no 2^k-th roots of unity for k > 1): Vandermonde "
                        "evaluation on the matrix cores and evaluation at a geometric "
                        "progression vs three-prime CRT", "runs": rows}


def bench_wrap(p=998244353, seed=10, reps=10):
    """Degrees where 2d - 1 lies just above a power of two: pm_mul, which takes
    the wrapped form (cyclic product on 2^j points, short product for the
    top coefficients, correction) when the top is small and the product
    large, against the plain 2^(j+1)-point transforms (pm_middle over the
    whole window), same operands, outputs compared."""
    import torch
    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for (m, n, k, d) in [(64, 64, 32, 1100), (64, 64, 32, 2100), (64, 64, 32, 2500),
                         (128, 128, 64, 1100), (128, 128, 64, 2100), (32, 32, 32, 2100)]:
        A = I.polymat_torch(seed, 0, I.TENSOR_A, p, d, m, n, dev)
        B = I.polymat_torch(seed, 0, I.TENSOR_B, p, d, n, k, dev)
        ws = polymat.Workspace(dev)
        ow = torch.empty((2 * d - 1, m, k), dtype=A.dtype, device=dev)
        op = torch.empty_like(ow)

        def timed(fn):
            fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        t_w = timed(lambda: polymat.mul(p, A, B, out=ow, workspace=ws, stream=stream))
        t_p = timed(lambda: polymat.middle(p, A, B, 0, 2 * d - 1, out=op, workspace=ws,
                                           stream=stream))
        # in direct mode only the wrap's correction kernel is timed as CRT
        Bd.pm_profile_begin()
        polymat.mul(p, A, B, out=ow, workspace=ws, stream=stream)
        wrapped = Bd.pm_profile_end()["crt"][1] > 0
        rows.append({"m": m, "n": n, "k": k, "d": d,
                     "pm_mul_path": "wrapped" if wrapped else "plain",
                     "pm_mul_ms": t_w, "plain_ms": t_p,
                     "outputs_equal": bool(torch.equal(ow, op))})
        del A, B, ws, ow, op
    return {"workload": f"products mod {p} with 2d - 1 just above a power of two", "runs": rows}


def bench_batched(steps, warmup, seed=3, count=512, p=998244353, settle_s=1.0):
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
    settle(lambda: polymat.mul_batched(p, As, Bs, outs, workspace=wsb, stream=stream), settle_s)
    Bd.pm_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        polymat.mul_batched(p, As, Bs, outs, workspace=wsb, stream=stream)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    kb = Bd.pm_profile_end()
    batched_ws = wsb.buf.numel()
    del wsb
    # a marker kernel between the batched calls and the single calls, so that
    # a kernel trace of this run can be split (the batched calls also launch
    # single-product kernels for their largest products)
    mark = torch.zeros(64, dtype=torch.uint32, device=dev)
    Bd.pm_neg_mod(p, mark.data_ptr(), mark.data_ptr(), 64, 4, int(stream.cuda_stream))
    torch.cuda.synchronize()
    wss = polymat.Workspace(dev)
    for _ in range(warmup):
        for A, B, C in zip(As, Bs, outs):
            polymat.mul(p, A, B, out=C, workspace=wss, stream=stream)
    torch.cuda.synchronize()

    def singles():
        for A, B, C in zip(As, Bs, outs):
            polymat.mul(p, A, B, out=C, workspace=wss, stream=stream)
    settle(singles, settle_s)
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
            "device_ms_per_batch": sum(v[0] for v in kb.values()) / steps,
            "one_per_call_value": work / t_s, "one_per_call_ms": t_s * 1e3,
            "speedup_vs_one_per_call": t_s / t_b, "sum_mnkd": work,
            "batched_workspace_GB": batched_ws / 1e9, "steps": steps, "warmup": warmup,
            "batched_kernel_ms": {kk: v[0] / steps for kk, v in kb.items() if v[1]},
            "one_per_call_kernel_ms": {kk: v[0] / steps for kk, v in ks.items() if v[1]},
            "path": batch_path(p, shapes, sum(v[0] for v in kb.values()) / steps,
                               sum(v[0] for v in ks.values()) / steps)}


def batch_path(p, shapes, device_ms_batched, device_ms_single):
    """The sum of the products' path floors against the device time of one
    batched call and of the single calls."""
    from paper_1905_04356_amd import binding as Bd
    floor_us = sum(product_floor_us(Bd.pm_plan(p, m, n, k, d, 4), m, n, k, d)
                   for (m, n, k, d) in shapes)
    return {"floor_ms": floor_us / 1e3, "frac": floor_us / 1e3 / device_ms_batched,
            "frac_one_per_call": floor_us / 1e3 / device_ms_single,
            "floor": "per product: sum over kernel kinds of max(algorithmic bytes at "
                     "8 TB/s, operations at the unit's peak), at the plan's points"}


KERNEL_KIND_OF = (  # rocprofv3 kernel-name fragment -> kind of the C ABI's timing
    ("ntt_col_fwd_kernel", "ntt_fwd"), ("ntt_col_fwd_mp_kernel", "ntt_fwd"),
    ("ntt_col_inv_crt_kernel", "ntt_inv"), ("ntt_block_kernel<true", "ntt_fwd"),
    ("ntt_fwd_pair_kernel", "ntt_fwd"), ("ntt_block_pair_kernel", "ntt_fwd"),
    ("ntt_col_fwd_pair_kernel", "ntt_fwd"), ("ntt_block_regc_pair_kernel", "ntt_fwd"),
    ("ntt_block_regc_kernel<true", "ntt_fwd"), ("ntt_block_regc_kernel<false", "ntt_inv"),
    ("ntt_fwd_kernel", "ntt_fwd"), ("pointwise", "pointwise"),
    ("ntt_block_kernel<false", "ntt_inv"), ("ntt_col_inv_kernel", "ntt_inv"),
    ("ntt_inv_kernel", "ntt_inv"), ("crt_kernel", "crt"), ("batch_kernel", "batched"))


def kind_of(name):
    for frag, kind in KERNEL_KIND_OF:
        if frag in name:
            return kind
    return None


def source_hash():
    """Hash of the library sources, so counters taken on older kernels are
    not reused."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_04356_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + fh.read())
    return h.hexdigest()[:16]


def summarize_profiles(root, steps_stats, warmup_stats, steps_pmc, workload, out_dir=None):
    """Turn rocprofv3 CSV output under `root` (st/: --kernel-trace --stats,
    f/ and w/: --pmc FETCH_SIZE / WRITE_SIZE of the benchmark, cf/ and cw/:
    the same counters on the calibration copy) into profiles/ summaries.
    Besides the --stats averages over every call (warm-up included), each
    kernel's average over the dispatches of the steady-state steps (the
    steps_stats timed steps and the steps_stats steps of the per-step
    distribution loop after them: its last 2 steps_stats / (warmup_stats +
    2 steps_stats) calls, from the trace) is the figure that bench.py's
    kernel timing measures."""
    import collections
    import csv

    def rows(sub, name):
        import glob
        files = glob.glob(os.path.join(root, sub, f"*{name}*.csv"))
        return list(csv.DictReader(open(files[0]))) if files else []

    total_steps = warmup_stats + 2 * steps_stats    # warm-up, timed, distribution loop
    steady_steps = 2 * steps_stats
    trace = collections.defaultdict(list)
    for r in rows("st", "kernel_trace"):
        trace[r["Kernel_Name"]].append((int(r["Start_Timestamp"]),
                                        int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    stats = rows("st", "kernel_stats")
    per_kind = collections.defaultdict(lambda: [0.0, 0])
    lines = []
    for r in stats:
        kd = kind_of(r["Name"])
        calls = int(r["Calls"])
        durs = [dn for _, dn in sorted(trace.get(r["Name"], []))]
        timed = durs[len(durs) - len(durs) * steady_steps // total_steps:] if durs else []
        avg_timed = sum(timed) / len(timed) / 1e3 if timed else float("nan")
        lines.append((r["Name"], calls, float(r["AverageNs"]) / 1e3, avg_timed,
                      float(r["TotalDurationNs"]) / 1e6, kd))
        if kd and timed:
            per_kind[kd][0] += sum(timed) / 1e6
            per_kind[kd][1] += len(timed)

    def counter(sub, cname):
        out = collections.defaultdict(float)
        for r in rows(sub, "counter_collection"):
            if r["Counter_Name"] == cname:
                out[r["Kernel_Name"]] += float(r["Counter_Value"]) * 1024.0  # KiB -> bytes
        return out

    # the calibration run also fills its source tensor; only the copies count
    cal_bytes = 3 * (256 << 20) * 4
    cf = sum(v for k, v in counter("cf", "FETCH_SIZE").items() if "copy" in k.lower())
    cw = sum(v for k, v in counter("cw", "WRITE_SIZE").items() if "copy" in k.lower())
    fscale = cal_bytes / cf if cf else None
    wscale = cal_bytes / cw if cw else None
    fetch, write = counter("f", "FETCH_SIZE"), counter("w", "WRITE_SIZE")
    # the counter runs: 1 warm-up step, steps_pmc - 1 timed steps and as many
    # distribution-loop steps
    pmc_total_steps = 1 + 2 * (steps_pmc - 1)
    traffic = collections.defaultdict(float)
    for name, v in fetch.items():
        if kind_of(name) and fscale:
            traffic[kind_of(name)] += v * fscale / pmc_total_steps
    for name, v in write.items():
        if kind_of(name) and wscale:
            traffic[kind_of(name)] += v * wscale / pmc_total_steps
    wflag = "" if workload == "c2" else f" --workload {workload}"
    cmd_st = (f"rocprofv3 --kernel-trace --stats --output-format csv -d {root}/st -o st -- "
              f"python3 bench.py --steps {steps_stats} --warmup {warmup_stats} --no-cpu-baseline "
              "--no-batched --no-middle --no-pmbasis --no-extra --serving-seconds 0 --settle-seconds 0"
              + wflag)
    md = [f"# Kernel profile: {workload}", "",
          "Command (from the repository root, on one MI355X):", "", "```", cmd_st, "```", "",
          f"`avg us` is rocprofv3's --stats average over all calls ({warmup_stats} warm-up "
          f"steps, {steps_stats} timed steps and the {steps_stats} steps of bench.py's "
          "per-step distribution loop); `timed avg us` averages, from the kernel trace, only "
          f"the dispatches of the last {steady_steps} steps, after the clocks have ramped up.",
          "",
          "| kernel | calls | avg us | timed avg us | total ms | kind |",
          "|---|---|---|---|---|---|"]
    for name, calls, avg, avg_t, tot, kd in sorted(lines, key=lambda x: -x[4]):
        md.append(f"| `{name}` | {calls} | {avg:.1f} | {avg_t:.1f} | {tot:.3f} | {kd} |")
    md += ["", f"Per steady-state step (last {steady_steps} steps):", "",
           "| kind | device ms per step |", "|---|---|"]
    for kd, (tot, calls) in sorted(per_kind.items()):
        md.append(f"| {kd} | {tot / steady_steps:.4f} |")
    md += ["", "## HBM traffic (rocprofv3 --pmc)", "",
           "Commands:", "", "```"]
    for sub, c in (("f", "FETCH_SIZE"), ("w", "WRITE_SIZE")):
        md.append(f"timeout -s KILL 90 rocprofv3 --pmc {c} --output-format csv -d {root}/{sub} "
                  f"-o {sub} -- python3 bench.py --steps {steps_pmc - 1} --warmup 1 "
                  "--no-cpu-baseline --no-batched --no-middle --no-pmbasis --no-extra --serving-seconds 0 "
                  "--settle-seconds 0" + wflag)
    for sub, c in (("cf", "FETCH_SIZE"), ("cw", "WRITE_SIZE")):
        md.append(f"timeout -s KILL 90 rocprofv3 --pmc {c} --output-format csv -d {root}/{sub} "
                  f"-o {sub} -- python3 bench.py --calibration-copy")
    md += ["```", "",
           f"Calibration: a plain copy of 3 x 1 GiB reads back FETCH_SIZE x {fscale:.3f} and "
           f"WRITE_SIZE x {wscale:.3f} of the bytes it moves; these factors scale the kernels' "
           "counters below.", "", "| kind | HBM bytes per step (fetch + write, scaled) |",
           "|---|---|"]
    for kd, b in sorted(traffic.items()):
        md.append(f"| {kd} | {b / 1e6:.1f} MB |")
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, f"{workload}_kernels.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    with open(os.path.join(out_dir, f"{workload}_traffic.json"), "w") as f:
        json.dump({"source_hash": source_hash(), "fetch_scale": fscale, "write_scale": wscale,
                   "bytes_per_step": dict(traffic),
                   "device_ms_per_step": {k: v[0] / steady_steps
                                          for k, v in per_kind.items()}}, f, indent=1)
    print("wrote profiles for", workload)


COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "SQ_INSTS_LDS",
            "SQ_LDS_BANK_CONFLICT", "SQ_INSTS_SALU", "SQ_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def summarize_counters(root, workload, steps_pmc=3):
    """profiles/<workload>_counters.md from one rocprofv3 --pmc run of
    bench.py under root/vc/ (the COUNTERS above): per kernel and per step,
    waves, VALU and LDS instructions, LDS bank conflicts, and the derived
    VALU busy fraction (SQ_ACTIVE_INST_VALU x 4 cycles per wave-instruction
    over the SIMDs' busy cycles) and VALU lane-operations per butterfly for
    the transform kernels."""
    import collections
    import csv
    import glob
    from paper_1905_04356_amd import binding as Bd
    files = glob.glob(os.path.join(root, "vc", "*counter_collection*.csv"))
    rows = list(csv.DictReader(open(files[0])))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    dur = collections.defaultdict(float)
    seen = set()
    for r in rows:
        name = r["Kernel_Name"]
        if "pm::" not in name:
            continue
        per[name][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[name].add(r["Dispatch_Id"])
        key = (name, r["Dispatch_Id"])
        if key not in seen and r.get("Start_Timestamp") and r.get("End_Timestamp"):
            seen.add(key)
            dur[name] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    steps = 1 + 2 * (steps_pmc - 1)
    p, m, n, k, d, dt = workload_params(workload)
    plan = Bd.pm_plan(p, m, n, k, d, 4 if dt == "u32" else 8)
    L, logL, r_ = 1 << plan.log2_len, plan.log2_len, plan.num_primes
    split = 4 if logL >= 11 else 0
    bfly = {"col_fwd": split * (L // 2) * (m * n + n * k) * r_,
            "block_fwd": (logL - split) * (L // 2) * (m * n + n * k) * r_,
            "block_inv": (logL - split) * (L // 2) * m * k * r_,
            "col_inv": split * (L // 2) * m * k * r_}

    def role(name):
        if "ntt_col_fwd" in name:
            return "col_fwd"
        if "ntt_col_inv" in name:
            return "col_inv"
        if "ntt_block" in name:
            return "block_fwd" if "<true" in name or "_pair_" in name else "block_inv"
        return None

    simds = CUS * 4
    cmd = ("timeout -s KILL 90 rocprofv3 --pmc " + " ".join(COUNTERS) +
           " --output-format csv -d gpurun_out/vc -o vc -- python3 bench.py --steps "
           f"{steps_pmc - 1} --warmup 1 --workload {workload} --no-cpu-baseline --no-batched "
           "--no-middle --no-pmbasis --no-extra --serving-seconds 0 --settle-seconds 0")
    md = [f"# Instruction counters: {workload}", "",
          "Command (from the repository root, on one MI355X):", "", "```", cmd, "```", "",
          f"Sums over the {steps} steps of the run, divided by {steps} (per step). "
          "GRBM_GUI_ACTIVE is summed over the 8 XCDs (it reads about 8 x 2.4 GHz x "
          "duration), so one XCD's busy cycles are GRBM_GUI_ACTIVE / 8. "
          "VALU busy = SQ_ACTIVE_INST_VALU x 4 / (SIMDs x GRBM_GUI_ACTIVE / 8), SIMDs = "
          f"{simds} (a wave's VALU instruction holds its SIMD for 4 cycles); the clock "
          "column is GRBM_GUI_ACTIVE / 8 / duration. "
          "VALU lane-ops per butterfly = SQ_INSTS_VALU x 64 / butterflies (transform "
          "kernels; the butterflies of both operands, or of C, per step).", "",
          "| kernel | dispatches/step | waves | VALU insts | LDS insts | LDS bank conflicts "
          "| GRBM_GUI_ACTIVE / 8 | clock GHz | VALU busy | lane-ops/butterfly |",
          "|---|---|---|---|---|---|---|---|---|---|"]
    for name, c in sorted(per.items(), key=lambda x: -x[1]["GRBM_GUI_ACTIVE"]):
        g = c["GRBM_GUI_ACTIVE"] / XCDS
        busy = c["SQ_ACTIVE_INST_VALU"] * 4 / (simds * g) if g else float("nan")
        clock = g / dur[name] / 1e9 if dur[name] else float("nan")
        rl = role(name)
        opb = (c["SQ_INSTS_VALU"] * 64 / steps / bfly[rl]) if rl and bfly.get(rl) else None
        short = name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")
        md.append(f"| `{short}` | {len(disp[name]) / steps:.0f} | {c['SQ_WAVES'] / steps:.0f} | "
                  f"{c['SQ_INSTS_VALU'] / steps:.3g} | {c['SQ_INSTS_LDS'] / steps:.3g} | "
                  f"{c['SQ_LDS_BANK_CONFLICT'] / steps:.3g} | {g / steps:.3g} | {clock:.2f} | "
                  f"{busy:.3f} | {'' if opb is None else f'{opb:.2f}'} |")
    with open(os.path.join(ROOT, "profiles", f"{workload}_counters.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print(f"wrote profiles/{workload}_counters.md")


def summarize_batched(root, batched_calls, single_rounds):
    """profiles/c3_batched_kernels.md from a rocprofv3 --kernel-trace run of
    `bench.py --only-batched` under root/sb/: the batched calls' kernels (the
    phase kernels, the single-product kernels of their largest products and
    the corrections of wrapped products, up to the marker kernel that
    bench_batched launches between its two parts) and the one-call-per-product
    kernels after it, as device time per call or round."""
    import collections
    import csv
    import glob
    files = glob.glob(os.path.join(root, "sb", "*kernel_trace.csv"))
    rows = sorted(csv.DictReader(open(files[0])), key=lambda r: int(r["Start_Timestamp"]))
    # (one-time table fills left out)
    rows = [r for r in rows if "pm::" in r["Kernel_Name"] and "fill_" not in r["Kernel_Name"]]
    # the batched calls' kernels (phase kernels, the single-product kernels of
    # their largest products, corrections) run from the first phase kernel's
    # call to the marker kernel that bench.py launches before the single calls
    batch = [i for i, r in enumerate(rows) if "batch_kernel" in r["Kernel_Name"]]
    marks = [i for i, r in enumerate(rows) if "neg_mod_kernel" in r["Kernel_Name"]]
    first, last = 0, marks[0] - 1
    assert batch and batch[-1] < marks[0]

    def table(sel, per):
        agg = collections.defaultdict(lambda: [0, 0.0])
        for r in sel:
            name = (r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
                    .replace("void ", ""))
            agg[name][0] += 1
            agg[name][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
        out = ["| kernel | calls | ms per call or round |", "|---|---|---|"]
        for name, (c, ms) in sorted(agg.items(), key=lambda x: -x[1][1]):
            out.append(f"| `{name}` | {c} | {ms / per:.3f} |")
        tot = sum(v[1] for v in agg.values()) / per
        return out + [f"| total | | {tot:.3f} |"], tot

    cmd = ("rocprofv3 --kernel-trace --output-format csv -d gpurun_out/sb -o sb -- "
           "python3 bench.py --only-batched --settle-seconds 0")
    tb, b_ms = table(rows[first:last + 1], batched_calls)
    ts, s_ms = table(rows[last + 2:], single_rounds)
    md = ["# Kernel profile: c3 (512 products, one batched call vs one pm_mul per product)", "",
          "Command (from the repository root, on one MI355X):", "", "```", cmd, "```", "",
          f"Device time of the kernels per batched call ({batched_calls} calls: warm-up, "
          "graph capture and replays) and per round of 512 single calls "
          f"({single_rounds} rounds), from the kernel trace; the wall time per call in "
          "bench.py's `batched` object also holds the gaps between launches.", "",
          f"## One batched call: {b_ms:.1f} ms of kernels", ""] + tb + \
         ["", f"## 512 single calls: {s_ms:.1f} ms of kernels", ""] + ts
    with open(os.path.join(ROOT, "profiles", "c3_batched_kernels.md"), "w") as f:
        f.write("\n".join(md) + "\n")
    print("wrote profiles/c3_batched_kernels.md")


def load_traffic(workload):
    """Per-step HBM bytes by kernel kind from profiles/, or None when the
    library sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != source_hash():
        return None
    return t.get("bytes_per_step")


def bench_serving(seconds, seed=5, rate=2000.0, pool_size=64, p=998244353,
                  budget_gb=64.0, streams=4, warmup_s=5.0, sweep="", sweep_seconds=10.0):
    """Config 5: Poisson arrivals (`rate` per second) of products with the
    batched shape rule, operands and their evaluations resident in a pool;
    continuous batching against one product per launch in arrival order
    (same resident evaluations) on the same trace. Latency percentiles leave
    out the requests that arrive in the first `warmup_s` seconds. A sweep
    over further rates (shorter traces) follows."""
    import torch

    from paper_1905_04356_amd import serving as S

    dev = torch.device("cuda:0")
    pool = S.make_pool(p, seed, pool_size, dev, with_evals=True)
    # warm-up: a short trace through both servers (table builds, allocator)
    wa, wi = S.trace(seed + 1000, rate, 0.5, pool_size)
    S.Server(p, pool, int(budget_gb * 2 ** 30), streams=streams).run(wa, wi)
    S.run_fifo(p, pool, wa, wi)
    torch.cuda.synchronize()

    def one(r, secs, skip, tseed):
        arrivals, items = S.trace(tseed, r, secs, pool_size)
        progress(f"serving: {r:g} req/s for {secs:g} s, continuous batching")
        srv = S.Server(p, pool, int(budget_gb * 2 ** 30), streams=streams, warmup_s=skip)
        cb = srv.run(arrivals, items)
        torch.cuda.synchronize()
        progress(f"serving: {r:g} req/s for {secs:g} s, one product per launch")
        fifo, _ = S.run_fifo(p, pool, arrivals, items, warmup_s=skip)
        torch.cuda.synchronize()
        offered = sum(pool[i].m * pool[i].n * pool[i].k * pool[i].d for i in items) / secs
        return {"rate": r, "seconds": secs, "offered_coef_mac_per_s": offered,
                "continuous_batching": cb, "one_product_per_launch": fifo}

    main = one(rate, seconds, warmup_s, seed)
    out = {"workload": f"Poisson {rate:g} req/s for {seconds:g} s, {pool_size} resident operand "
                       f"pairs (batched shape rule, seed {seed}), mod {p}; percentiles over "
                       f"arrivals after {warmup_s:g} s",
           "offered_coef_mac_per_s": main["offered_coef_mac_per_s"],
           "continuous_batching": main["continuous_batching"],
           "one_call_per_request": main["one_product_per_launch"],
           "baseline": "one product per launch on one stream, in arrival order, with the same "
                       "resident evaluations",
           "budget_GB": budget_gb, "streams": streams}
    rates = [float(x) for x in sweep.split(",") if x.strip()] if sweep else []
    if rates:
        out["sweep"] = [one(r, sweep_seconds, min(2.0, sweep_seconds / 5), seed + 17 + i)
                        for i, r in enumerate(rates)]
    return out


def valu_probe(blocks=8192, iters=4096, reps=5):
    """The measured issue rate of 32-bit high multiplies (pm_probe_valu:
    independent chains, blocks x 256 threads x iters x 8 lane-ops per
    launch), against the VALU peak the ALU rooflines use; best of `reps`
    event-timed launches."""
    import torch

    from paper_1905_04356_amd import binding as Bd
    out = torch.empty(blocks * 256, dtype=torch.uint32, device="cuda")
    st = torch.cuda.current_stream()
    sp = int(st.cuda_stream)
    Bd._check(Bd.pm_probe_valu(blocks, iters, out.data_ptr(), sp), "pm_probe_valu")
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        Bd._check(Bd.pm_probe_valu(blocks, iters, out.data_ptr(), sp), "pm_probe_valu")
        e1.record(st)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    rate = blocks * 256.0 * iters * 8 / best
    return {"instruction": "v_mul_hi_u32, 8 independent chains per thread",
            "lane_ops_per_s": rate, "frac_of_peak": rate / (VALU_PEAK_TOPS * 1e12),
            "peak_lane_ops_per_s": VALU_PEAK_TOPS * 1e12, "blocks": blocks, "iters": iters}


def progress(msg):
    """A progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def settle(step, seconds):
    """Untimed steps until the device has run for `seconds` (after the
    warm-up steps): the clocks ramp up over the first few hundred
    milliseconds of load, and a timed region that starts earlier measures
    the ramp rather than the kernels. Returns the steps run."""
    import torch
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            step()
        n += 8
        torch.cuda.synchronize()
    return n


def bench_single(workload, steps, warmup, settle_s=1.0):
    """One product per step (pm_mul on resident operands): throughput, the
    per-step device time distribution, per-kernel device times and their
    rooflines, and the whole path's roofline fraction."""
    import numpy as np
    import torch

    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat

    p, m, n, k, d, dt = workload_params(workload)
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

    for _ in range(warmup):
        polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    settled = settle(lambda: polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream),
                     settle_s)

    # Kernel durations come from the dispatch events of every
    # PROFILE_EVERY-th step of the timed loop (each timed launch costs a few
    # microseconds of dispatch work, so not every step carries them).
    Bd.pm_profile_begin()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(steps):
        Bd.pm_profile_pause(i % PROFILE_EVERY != 0)
        polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstats = Bd.pm_profile_end()
    timed_steps = len(range(0, steps, PROFILE_EVERY))

    # Distribution of single-step device times, from a separate loop of the
    # same length with an event between consecutive steps (so these events
    # stay out of the timed loop above).
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        polymat.mul(p, tA, tB, out=tC, workspace=ws, stream=stream)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    dist = {"median": per_step[len(per_step) // 2] if len(per_step) % 2 else
            0.5 * (per_step[len(per_step) // 2 - 1] + per_step[len(per_step) // 2]),
            "min": per_step[0],
            "p90": per_step[max(0, -(-9 * len(per_step) // 10) - 1)],   # nearest rank
            "steps": steps}

    wall = t1 - t0
    work = float(m) * n * k * d
    value = work * steps / wall
    kernels = {}
    folded = plan.mode == 1 and kstats.get("crt", (0.0, 0))[1] == 0
    for kind, (ms, launches) in kstats.items():
        if launches == 0:
            continue
        byts, ops = kernel_work(kind, plan, p, m, n, k, d, eb, crt_folded=folded)
        sec = ms / 1e3 / timed_steps          # device seconds per product
        kernels[kind] = {"ms_per_step": ms / timed_steps, "launches_per_step":
                         launches / timed_steps, "algorithmic_bytes": byts,
                         "ops": ops}
        kernels[kind]["roofline"] = roofline_for(kind, byts, ops, sec, plan)
    traffic = load_traffic(workload)
    for kind in kernels:
        kernels[kind]["roofline"]["traffic"] = traffic.get(kind) if traffic else None
    dominant = max(kernels, key=lambda kk: kernels[kk]["ms_per_step"])
    roof = dict(kernels[dominant]["roofline"])
    # the path's fraction against the median per-step device time (the
    # measurement's definition), and against the timed loop's mean
    mean_ms = ev0.elapsed_time(ev1) / steps
    roof["path"] = path_roofline(kernels, plan, dist["median"])
    roof["path"]["measured"] = "median per-step device time"
    roof["path"]["mean_us"] = mean_ms * 1e3
    roof["path"]["frac_mean"] = roof["path"]["floor_us"] / (mean_ms * 1e3)

    out = {
        "metric": "polymatrix mul mod p: m*n*k*d coefficient-MACs/s",
        "value": value,
        "unit": "coefficient-MAC/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "settle_s": settle_s,
        "untimed_steps_run": warmup + settled,
        "ms_per_step": wall / steps * 1e3,
        "device_ms_per_step": mean_ms,
        "device_ms_per_step_dist": dist,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic: seeded uniform residues in [0, p) (splitmix64)",
        "config": {"workload": f"{m}x{n}.{n}x{k} polynomial matrices, degree<{d}, mod {p}",
                   "p": p, "m": m, "n": n, "k": k, "d": d,
                   "L": 1 << plan.log2_len, "mode": "direct" if plan.mode == 0 else "crt",
                   "primes": plan.num_primes,
                   "pointwise": "mfma_int8" if plan.pointwise == 1 else "valu",
                   "tune_entry": plan.tune_entry},
        "crt_reconstruction": None if plan.mode == 0 else
        ("in the last inverse pass (ntt_inv)" if folded else "separate kernel (crt)"),
        "roofline": roof,
        "kernels": kernels,
        "kernel_timing": f"dispatch start/stop events on {timed_steps} of the {steps} "
                         f"timed steps (every {PROFILE_EVERY}th)",
    }
    del tA, tB, tC, ws
    return {"_out": out, "p": p, "m": m, "n": n, "k": k, "d": d, "A": A, "B": B}


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2]


def bench_tuned_vs_default(workload, rounds=5, steps=10):
    """The product timed under the tuning table and with no table (the
    defaults), alternately: median device ms per product of each."""
    import torch
    from paper_1905_04356_amd import binding as Bd
    from paper_1905_04356_amd import inputs as I
    from paper_1905_04356_amd import polymat
    p, m, n, k, d, dt = workload_params(workload)
    dev = torch.device("cuda:0")
    tdt = torch.uint32 if dt == "u32" else torch.uint64
    A = I.polymat_torch(2, 0, I.TENSOR_A, p, d, m, n, dev, tdt)
    B = I.polymat_torch(2, 0, I.TENSOR_B, p, d, n, k, dev, tdt)
    C = torch.empty((2 * d - 1, m, k), dtype=tdt, device=dev)
    ws = polymat.Workspace(dev)
    stream = torch.cuda.current_stream()
    info = Bd.tune_info()
    entry = Bd.pm_plan(p, m, n, k, d, 4 if dt == "u32" else 8).tune_entry

    def once():
        for _ in range(3):
            polymat.mul(p, A, B, out=C, workspace=ws, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            polymat.mul(p, A, B, out=C, workspace=ws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    tuned, dflt = [], []
    try:
        for _ in range(rounds):
            Bd.tune_load(None)
            tuned.append(once())
            Bd.tune_load("")
            dflt.append(once())
    finally:
        torch.cuda.synchronize()
        Bd.tune_load(None)
    del A, B, C, ws
    return {"table_entries": info[0], "table_source": info[1], "tune_entry": entry,
            "tuned_ms": _median(tuned), "default_ms": _median(dflt),
            "speedup": _median(dflt) / _median(tuned)}


def bench_batched_tuned_vs_default(seed=3, count=512, p=998244353, rounds=3):
    """The batched workload under the tuning table and with no table
    (defaults), alternately: median wall ms per batched call (graph replays)."""
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
    ws = polymat.Workspace(dev)
    stream = torch.cuda.current_stream()
    used = sum(Bd.pm_plan(p, m, n, k, d, 4).tune_entry >= 0 for (m, n, k, d) in shapes)

    def once():
        for _ in range(2):          # eager, then graph capture
            polymat.mul_batched(p, As, Bs, outs, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            polymat.mul_batched(p, As, Bs, outs, workspace=ws, stream=stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / 3 * 1e3

    tuned, dflt = [], []
    try:
        for _ in range(rounds):
            Bd.tune_load(None)
            tuned.append(once())
            Bd.tune_load("")
            dflt.append(once())
    finally:
        torch.cuda.synchronize()
        Bd.tune_load(None)
    del As, Bs, outs, ws
    return {"products_with_table_entries": int(used), "tuned_ms": _median(tuned),
            "default_ms": _median(dflt), "speedup": _median(dflt) / _median(tuned)}


def calibration_copy():
    """A plain device copy of known size (1 GiB, three times), the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 256 << 20
    a = torch.ones(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copied_bytes_per_launch": n * 4, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-middle", action="store_true")
    ap.add_argument("--no-pmbasis", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the tuned-vs-default comparisons and the c1/c4 products")
    ap.add_argument("--batched-steps", type=int, default=5)
    ap.add_argument("--settle-seconds", type=float, default=1.0,
                    help="untimed steps after the warm-up steps until the device has run "
                         "this long (clock ramp-up), before each timed region")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the serving trace (0: skip)")
    ap.add_argument("--serving-warmup", type=float, default=5.0,
                    help="seconds at the start of each trace left out of the percentiles")
    ap.add_argument("--serving-sweep", default="4000,8000",
                    help="further arrival rates (req/s), 10 s each ('' : none)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run only the 1 GiB copy used to calibrate HBM byte counters")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched comparison (configuration 3) and print it")
    ap.add_argument("--summarize-batched", metavar="DIR",
                    help="write profiles/c3_batched_kernels.md from DIR/sb (rocprofv3 trace)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="write profiles/<workload>_counters.md from DIR/vc (rocprofv3 --pmc)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 CSV output in DIR")
    args = ap.parse_args()
    if args.calibration_copy:
        calibration_copy()
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload)
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, 20, 100, 3, args.workload)
        return
    if args.summarize_batched:
        summarize_batched(args.summarize_batched, 2 + args.batched_steps, 2 + args.batched_steps)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs every product on a single "
              "MI355X and has no multi-GPU path (the sharding design is documented).",
              file=sys.stderr)
        sys.exit(2)
    if args.only_batched:
        print(json.dumps(bench_batched(args.batched_steps, 2, settle_s=args.settle_seconds)),
              flush=True)
        return

    import torch

    progress(f"single product {args.workload}: {args.warmup} warm-up, {args.steps} timed steps")
    res = bench_single(args.workload, args.steps, args.warmup, args.settle_seconds)
    out = res.pop("_out")
    p, m, n, k, d = res["p"], res["m"], res["n"], res["k"], res["d"]
    A, B = res["A"], res["B"]
    out["tuning"] = {}
    if not args.no_extra:
        progress("tuning table against the defaults")
        out["tuning"]["single"] = bench_tuned_vs_default(args.workload)
    for w in () if args.no_extra else ("c1", "c4"):
        if w != args.workload:
            progress(f"single product {w}")
            r = bench_single(w, 20, 20, args.settle_seconds)
            o = r.pop("_out")
            keep = {kk: o[kk] for kk in ("value", "unit", "ms_per_step", "device_ms_per_step",
                                         "device_ms_per_step_dist", "dtype", "config",
                                         "roofline", "kernels", "steps", "warmup",
                                         "crt_reconstruction")}
            if not args.no_cpu_baseline:
                keep["cpu_baseline"] = cpu_baseline(r["p"], r["A"], r["B"], r["m"], r["n"],
                                                    r["k"], r["d"], 5.0)
            out[w] = keep
            torch.cuda.empty_cache()
    torch.cuda.empty_cache()
    if not args.no_batched:
        progress("batched: 512 products")
        out["batched"] = bench_batched(args.batched_steps, 2, settle_s=args.settle_seconds)
        if not args.no_extra:
            out["tuning"]["batched"] = bench_batched_tuned_vs_default()
        torch.cuda.empty_cache()
    if not args.no_middle:
        progress("middle product, PM-Basis, Newton, Vandermonde, wrapped lengths")
        out["middle"] = bench_middle()
        torch.cuda.empty_cache()
    if not args.no_pmbasis:
        out["pmbasis"] = bench_pmbasis()
        torch.cuda.empty_cache()
        out["newton"] = bench_newton()
        torch.cuda.empty_cache()
        out["vandermonde"] = bench_vdm()
        torch.cuda.empty_cache()
        out["wrapped_lengths"] = bench_wrap()
        torch.cuda.empty_cache()
    if args.serving_seconds > 0:
        out["serving"] = bench_serving(args.serving_seconds, warmup_s=args.serving_warmup,
                                       sweep=args.serving_sweep, sweep_seconds=10.0)
        torch.cuda.empty_cache()
    out["valu_probe"] = valu_probe()
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(p, A, B, m, n, k, d, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
