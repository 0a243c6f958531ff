"""Tuning driver: measure launch shapes on the device and write the tuning
table that libpm reads on first use (tune_table.json beside libpm.so).

    python -m paper_1905_04356_amd.tune [--out PATH] [--quick]

The paper determines the thresholds between its multiplication variants by
experiment, with separate values for small and large primes (Section 2,
"Polynomial matrix multiplication"). Here every launch shape computes the
same residues, so tuning is a search for the fastest one per (prime class,
log2 L, shape bucket). For each bucket a representative product is timed
(median of device-event times over repeated pm_mul calls on resident
operands) under its current knobs, then one knob at a time is changed
(coordinate descent over the admissible values), keeping a change when it
is faster by more than `--margin`. A bucket gets an entry only when its best
knobs beat the defaults by that margin. Knob values that most buckets of
one length chose become a whole-length entry for that length's other
shapes, if they speed up shapes outside the grid. Global knobs of the batched path
(pointwise work per tile, block-tile size) are tuned on the batched workload
(512 products of the batched shape rule), timed as whole batched calls.

The search is bounded: a fixed list of buckets (the benchmark's single
products and a grid over the batched workload's shapes and lengths), a few
values per knob, and a few passes; about a minute or two of device time.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import torch

from . import binding as B
from . import inputs as I
from . import polymat

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_table.json")

P_LT30 = 998244353        # 119 2^23 + 1
P_GE30 = 2013265921       # 15 2^27 + 1

# Moves of the search: each sets one knob, or a pair that only makes sense
# together (threads and tile size of a block step); the defaults are among
# the values.
MOVES = [
    [{"split": 4}, {"split": 3}, {"split": 5}],
    [{"maxr": 4}, {"maxr": 3}],
    [{"blk_nt": 256, "blk_tile_log": 13}, {"blk_nt": 512, "blk_tile_log": 14},
     {"blk_nt": 512, "blk_tile_log": 13}, {"blk_nt": 256, "blk_tile_log": 12},
     {"blk_nt": 256, "blk_tile_log": 14}],
    [{"blk_nt_inv": 0, "blk_tile_log_inv": 0}, {"blk_nt_inv": 512, "blk_tile_log_inv": 14},
     {"blk_nt_inv": 512, "blk_tile_log_inv": 13}, {"blk_nt_inv": 256, "blk_tile_log_inv": 12},
     {"blk_nt_inv": 256, "blk_tile_log_inv": 14}],
    [{"colvec_fwd": 4}, {"colvec_fwd": 2}],
    [{"colvec_inv": 4}, {"colvec_inv": 2}],
    [{"reg_tile": 1}, {"reg_tile": 0}],
    [{"pointwise": 1}, {"pointwise": 0}],
    [{"pw_small_lds": 45056}, {"pw_small_lds": 0}, {"pw_small_lds": 98304}],
    [{"pw_pipe": -1}, {"pw_pipe": 0}, {"pw_pipe": 1}, {"pw_pipe": 2}],
]
DEFAULTS = {"split": 4, "maxr": 4, "blk_nt": 256, "blk_tile_log": 13, "colvec_fwd": 4,
            "colvec_inv": 4, "reg_tile": 1, "pointwise": 1, "pw_small_lds": 45056,
            "pw_pipe": -1, "blk_nt_inv": 0, "blk_tile_log_inv": 0}
CLASS_NAME = {0: "direct_lt30", 1: "direct_ge30", 2: "crt"}


def clog2(x: int) -> int:
    return max(0, (x - 1).bit_length())


def say(*a):
    print(*a, flush=True)


class Product:
    """Resident operands of one product and a timer for pm_mul on them."""

    def __init__(self, p, m, n, k, d, dtype=torch.uint32, seed=77):
        dev = torch.device("cuda")
        self.p, self.m, self.n, self.k, self.d = p, m, n, k, d
        self.A = I.polymat_torch(seed, 0, I.TENSOR_A, p, d, m, n, dev, dtype)
        self.B = I.polymat_torch(seed, 0, I.TENSOR_B, p, d, n, k, dev, dtype)
        self.C = torch.empty((2 * d - 1, m, k), dtype=dtype, device=dev)
        self.ws = polymat.Workspace()
        eb = 4 if dtype == torch.uint32 else 8
        info = B.pm_plan(p, m, n, k, d, eb)
        self.pclass = 2 if info.mode != 0 else (0 if p < (1 << 30) else 1)
        self.logL = info.log2_len

    def key(self):
        return (self.pclass, self.logL, clog2(self.m), clog2(self.n), clog2(self.k))

    def time_us(self, reps=9, warm=3) -> float:
        for _ in range(warm):
            polymat.mul(self.p, self.A, self.B, out=self.C, workspace=self.ws)
        st = torch.cuda.current_stream()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for a, b in evs:
            a.record(st)
            polymat.mul(self.p, self.A, self.B, out=self.C, workspace=self.ws)
            b.record(st)
        torch.cuda.synchronize()
        ts = sorted(a.elapsed_time(b) * 1e3 for a, b in evs)
        return ts[len(ts) // 2]


def entry_json(key, knobs):
    pclass, logL, ml, nl, kl = key
    return {"prime_class": CLASS_NAME[pclass], "log2_len": logL, "m_log2": ml, "n_log2": nl,
            "k_log2": kl, "knobs": knobs}


def table_json(entries, glob=None):
    t = {"format": "pm-tune-1", "entries": entries}
    if glob:
        t["global"] = glob
    return json.dumps(t)


def time_with(prod: Product, knobs: dict, reps: int) -> float:
    """Time prod with a one-entry table holding `knobs` for its bucket."""
    B.tune_load(table_json([entry_json(prod.key(), knobs)]))
    return prod.time_us(reps)


def tune_bucket(prod: Product, margin: float, passes: int, reps: int):
    knobs = dict(DEFAULTS)
    base = time_with(prod, {}, reps)
    best = base
    tried = 1
    for _ in range(passes):
        improved = False
        for values in MOVES:
            for move in values:
                if all(knobs[k] == v for k, v in move.items()):
                    continue
                cand = dict(knobs, **move)
                t = time_with(prod, {k: x for k, x in cand.items() if x != DEFAULTS[k]}, reps)
                tried += 1
                if t < best * (1 - margin):
                    best, knobs, improved = t, cand, True
        if not improved:
            break
    # confirm: the winner against the defaults, alternately
    if best < base * (1 - margin):
        diff = {k: x for k, x in knobs.items() if x != DEFAULTS[k]}
        w, dflt = [], []
        for _ in range(3):
            w.append(time_with(prod, diff, reps))
            dflt.append(time_with(prod, {}, reps))
        w, dflt = sorted(w)[1], sorted(dflt)[1]
        if w < dflt * (1 - margin):
            return diff, w, dflt, tried
        return None, w, dflt, tried
    return None, best, base, tried


def buckets(quick: bool):
    """Representative products: the benchmark's single products, then a grid
    over the batched workload's shapes (m, k in {16, 64, 128}, n in {8, 32,
    128}) at three lengths, mod 998244353."""
    out = [
        (P_GE30, 64, 64, 32, 4096, torch.uint32),     # single-product benchmark
        (P_LT30, 8, 8, 8, 256, torch.uint32),         # small product
        (I.seeded_prime_60(4), 32, 32, 32, 2048, torch.uint64),   # 60-bit, CRT
    ]
    ds = [500, 2000] if quick else [100, 300, 700, 1500, 3000, 6000, 12000]
    for d in ds:
        for (m, k) in ((16, 16), (64, 64), (128, 64), (128, 128)):
            for n in (8, 32, 128):
                out.append((P_LT30, m, n, k, d, torch.uint32))
    return out


def tune_min_wg(entries, margin, rounds=5):
    """The globals min_wg_unsplit and min_wg (fewest workgroups per transform
    launch before a single product takes fewer entries per workgroup, for
    lengths below and from the split on), each on small products whose
    transforms it governs: the sum of their median times per candidate
    value."""
    u32, u64 = torch.uint32, torch.uint64
    sets = [
        ("min_wg_unsplit", (0, 512, 1024, 2048),
         [(P_LT30, 8, 8, 8, 256, u32), (P_LT30, 16, 16, 16, 300, u32),
          (P_LT30, 32, 32, 32, 500, u32), (P_LT30, 4, 8, 4, 100, u32),
          (P_LT30, 128, 8, 64, 200, u32)]),
        ("min_wg", (0, 256, 1024, 2048),
         [(P_GE30, 16, 8, 16, 900, u32), (P_LT30, 8, 8, 8, 1500, u32),
          (P_LT30, 16, 16, 16, 3000, u32), (I.seeded_prime_60(4), 32, 32, 32, 2048, u64)]),
    ]
    glob, report = {}, {}
    for knob, cands, shapes in sets:
        prods = [Product(p, m, n, k, d, dt) for (p, m, n, k, d, dt) in shapes]

        def total(g):
            B.tune_load(table_json(entries, g))
            return sum(pr.time_us() for pr in prods)

        # small launches are sensitive to the clocks' state: the candidates
        # are timed in interleaved rounds, and each keeps its median
        vals = [None] + list(cands)
        times = {v: [] for v in vals}
        for _ in range(rounds):
            for v in vals:
                times[v].append(total(glob if v is None else dict(glob, **{knob: v})))
        med = {v: sorted(t)[len(t) // 2] for v, t in times.items()}
        base = med[None]
        best, choice = base, None
        for v in cands:
            if med[v] < best * (1 - margin):
                best, choice = med[v], v
        if choice is not None:
            glob[knob] = choice
        report[knob] = (base, best)
        del prods
    return glob, report


def tune_batch_globals(entries, margin, quick, glob0=None):
    """batch_pw_work and batch_tile_log on the batched workload (512
    products, batched shape rule, seed 3), with the entries found."""
    p, seed = P_LT30, 3
    shapes = I.batched_shapes(seed, 128 if quick else 512)
    dev = torch.device("cuda")
    As = [I.polymat_torch(seed, i, I.TENSOR_A, p, d, m, n, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    Bs = [I.polymat_torch(seed, i, I.TENSOR_B, p, d, n, k, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    outs = [torch.empty((2 * d - 1, m, k), dtype=torch.uint32, device=dev)
            for (m, n, k, d) in shapes]
    ws = polymat.Workspace()

    def run(glob):
        B.tune_load(table_json(entries, dict(glob0 or {}, **glob)))
        for _ in range(2):    # first call eager, second captures the graph
            polymat.mul_batched(p, As, Bs, outs, workspace=ws)
        torch.cuda.synchronize()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            polymat.mul_batched(p, As, Bs, outs, workspace=ws)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return sorted(ts)[1]

    base = run({})
    best, glob = base, {}
    for name, values in (("batch_pw_work", [8192, 4096, 16384]),
                         ("batch_tile_log", [14, 13])):
        for v in values:
            g = dict(glob, **{name: v})
            t = run(g)
            if t < best * (1 - margin):
                best, glob = t, g
    del As, Bs, outs, ws
    torch.cuda.empty_cache()
    return glob, best, base


def common_knobs(chosen: list[dict]) -> dict:
    """Knob values that at least 3/4 of the buckets chose ({} for a bucket
    that kept the defaults)."""
    counts = {}
    for c in chosen:
        for kv in c.items():
            counts[kv] = counts.get(kv, 0) + 1
    return {k: v for (k, v), n in counts.items() if 4 * n >= 3 * len(chosen)}


def length_fallbacks(entries, report, margin, rounds=3):
    """Entries for whole lengths (direct primes below 2^30): where at least
    3/4 of the buckets tuned at one log2 L chose the same values of some
    knobs, those values become an entry for that length's other buckets
    (placed after the bucket entries, since the first match wins), kept only
    if they speed up three shapes outside the grid at that length (timed in
    interleaved rounds, median)."""
    groups = {}
    for rec in report:
        if rec["_key"][0] == 0:
            groups.setdefault(rec["_key"][1], []).append(rec)
    out = []
    for logL, recs in sorted(groups.items()):
        if len(recs) < 4:
            continue
        common = common_knobs([rec["_knobs"] for rec in recs])
        if not common:
            continue
        d = recs[0]["shape"][3]
        prods = [Product(P_LT30, m, n, k, d)
                 for (m, n, k) in ((32, 32, 32), (8, 64, 8), (128, 32, 32))]
        fb = {"prime_class": CLASS_NAME[0], "log2_len": logL, "knobs": common}
        times = {0: [], 1: []}
        for _ in range(rounds):
            for with_fb in (0, 1):
                B.tune_load(table_json(entries + out + ([fb] if with_fb else [])))
                times[with_fb].append(sum(pr.time_us() for pr in prods))
        t0, t1 = sorted(times[0])[rounds // 2], sorted(times[1])[rounds // 2]
        kept = t1 < t0 * (1 - margin)
        say(f"[tune] L=2^{logL} fallback {json.dumps(common)}: other shapes {t0:.1f} -> "
            f"{t1:.1f} us{'' if kept else ' (not kept)'}")
        if kept:
            out.append(dict(fb, us=round(t1, 2), default_us=round(t0, 2)))
        del prods
        torch.cuda.empty_cache()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="fewer buckets (a smoke run)")
    ap.add_argument("--margin", type=float, default=0.03,
                    help="relative gain a change must show to be kept")
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--reps", type=int, default=9)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("the tuning driver needs a GPU")
    t_start = time.perf_counter()
    entries, report = [], []
    for (p, m, n, k, d, dt) in buckets(args.quick):
        prod = Product(p, m, n, k, d, dt)
        key = prod.key()
        if any(e["_key"] == key for e in report):
            continue
        knobs, t_best, t_default, tried = tune_bucket(prod, args.margin, args.passes, args.reps)
        rec = {"_key": key, "_knobs": knobs or {}, "shape": [m, n, k, d], "p": p,
               "candidates": tried,
               "us": round(t_best, 2), "default_us": round(t_default, 2)}
        say(f"[tune] {CLASS_NAME[key[0]]} L=2^{key[1]} {m}x{n}x{k} d={d}: "
            f"default {t_default:.1f} us, best {t_best:.1f} us "
            f"{'-> ' + json.dumps(knobs) if knobs else '(defaults kept)'} [{tried} timed]")
        report.append(rec)
        if knobs:
            e = entry_json(key, knobs)
            e.update({k: v for k, v in rec.items() if not k.startswith("_")})
            entries.append(e)
        del prod
        torch.cuda.empty_cache()
    entries += length_fallbacks(entries, report, args.margin)
    gmin, rep = tune_min_wg(entries, args.margin)
    for knob, (t0, t1) in rep.items():
        say(f"[tune] {knob} {gmin.get(knob, 'default')}: small products {t0:.1f} -> {t1:.1f} us")
    glob, t_b, t_b0 = tune_batch_globals(entries, args.margin, args.quick, gmin)
    glob = dict(gmin, **glob)
    say(f"[tune] batched globals {json.dumps(glob)}: {t_b0:.2f} -> {t_b:.2f} ms")
    table = {"format": "pm-tune-1",
             "device": torch.cuda.get_device_name(0),
             "generated_by": "python -m paper_1905_04356_amd.tune",
             "seconds": round(time.perf_counter() - t_start, 1),
             "batched_ms": {"default": round(t_b0, 3), "tuned": round(t_b, 3)},
             "global": glob,
             "entries": entries}
    text = json.dumps(table, indent=1)
    B.tune_load(text)   # validates before writing
    with open(args.out, "w") as f:
        f.write(text + "\n")
    say(f"[tune] wrote {args.out}: {len(entries)} entries, "
        f"{time.perf_counter() - t_start:.0f} s")


if __name__ == "__main__":
    sys.exit(main())
