"""Serving loop: products arriving over time, admitted by HBM footprint and
run with continuous batching on several HIP streams.

Requests name an operand pair from a device-resident pool. The pool keeps
each operand's evaluations at the transform points (the precomputation of
the paper's multiplier classes, Section 2, "Polynomial matrix
multiplication"), so a request costs only its pointwise products, inverse
transform and (for CRT moduli) reconstruction; products that pm_mul
computes in the wrapped form on half the points run as pm_mul calls
instead. The host loop:

* moves requests whose arrival time has passed into a FIFO ready queue;
* polls the events of in-flight batches; a finished batch frees its streams'
  slot and its footprint and stamps its requests' completion times;
* while a stream is free, takes ready requests in arrival order as long as
  their footprint (workspace + output bytes) fits the free HBM budget, and
  launches them as one pm_mul_batched call on that stream. A request of at
  least `solo_work` transform work runs in a launch of its own, so that the
  small requests around it do not wait for it (all of a batch's outputs
  complete together); it overlaps them on another stream instead.

Requests that arrive while others run therefore join the next launch and
overlap them on the device. Latency = completion (observed by the host) -
scheduled arrival; percentiles skip the requests that arrive during a
warm-up interval. The baseline server on the same trace launches one product
per request, in arrival order, on one stream, with the same resident
evaluations.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import torch

from . import binding as _b
from . import inputs as I
from . import polymat


@dataclasses.dataclass
class PoolItem:
    m: int
    n: int
    k: int
    d: int
    A: torch.Tensor
    B: torch.Tensor
    A_eval: torch.Tensor | None
    B_eval: torch.Tensor | None
    footprint: int          # workspace + output bytes of one product
    wraps: bool = False     # pm_mul takes the wrapped form (no evaluations kept)

    @property
    def work(self) -> int:
        """Transform work (m n + n k + m k) L, L = 2^ceil(log2(2d - 1))."""
        L = 1 << max(0, (2 * self.d - 2).bit_length())
        return (self.m * self.n + self.n * self.k + self.m * self.k) * L


def make_pool(p: int, seed: int, count: int, device, with_evals: bool = True,
              dims_cap: int | None = None) -> list[PoolItem]:
    """`count` operand pairs with the batched shape rule, generated on the
    device; evaluations precomputed when `with_evals`, except for products
    that pm_mul computes in the wrapped form (2d - 1 a little above a power
    of two 2^j, large shapes): on 2^j points they cost less than the
    2^(j+1)-point evaluations would save."""
    pool = []
    for i, (m, n, k, d) in enumerate(I.batched_shapes(seed, count)):
        if dims_cap:
            m, n, k = min(m, dims_cap), min(n, dims_cap), min(k, dims_cap)
        A = I.polymat_torch(seed, i, I.TENSOR_A, p, d, m, n, device)
        B = I.polymat_torch(seed, i, I.TENSOR_B, p, d, n, k, device)
        wraps = _b.pm_plan(p, m, n, k, d, 4).wrap_log2_len > 0
        Ae = polymat.evaluate(p, A, 0) if with_evals and not wraps else None
        Be = polymat.evaluate(p, B, 1) if with_evals and not wraps else None
        fp = _b.pm_workspace_bytes(p, m, n, k, d, 4) + 4 * (2 * d - 1) * m * k
        pool.append(PoolItem(m, n, k, d, A, B, Ae, Be, fp, wraps))
    torch.cuda.synchronize()
    return pool


def trace(seed: int, rate: float, duration: float, pool_size: int):
    """Arrival times (Poisson, `rate` per second) and the pool item of each."""
    t = I.poisson_arrivals(seed, rate, duration)
    s = I._Stream(seed, I.SAMPLE_STREAM + 7)
    return t, [s.uniform_int(pool_size) for _ in t]


def _percentiles(lat):
    if not lat:
        return None, None
    xs = sorted(lat)
    return xs[int(0.50 * (len(xs) - 1))], xs[int(0.99 * (len(xs) - 1))]


class Server:
    """Continuous-batching server over `streams` HIP streams.

    `launcher(slot, items) -> (event, outputs)` enqueues one batch; the
    default runs pm_mul_batched on the slot's stream. Tests of the admission
    logic pass a host-side double instead."""

    def __init__(self, p: int, pool: list[PoolItem], budget_bytes: int, streams: int = 4,
                 max_batch: int = 256, keep=(), launcher=None, warmup_s: float = 0.0,
                 solo_work: int = 1 << 25):
        self.p, self.pool, self.budget = p, pool, budget_bytes
        self.warmup_s = warmup_s
        self.max_batch = max_batch
        self.solo_work = solo_work
        self.nslots = streams
        self.launch = launcher or self._gpu_launch
        self.streams = None
        self.ws = None
        self.keep = set(keep)          # request ids whose outputs are kept
        self.kept = {}
        self.peak_used = 0
        self.admitted = []             # request ids in launch order

    def _gpu_launch(self, si, its):
        if self.streams is None:
            self.streams = [torch.cuda.Stream() for _ in range(self.nslots)]
            self.ws = [polymat.Workspace() for _ in range(self.nslots)]
        st = self.streams[si]
        with torch.cuda.stream(st):
            outs = [torch.empty((2 * it.d - 1, it.m, it.k), dtype=torch.uint32,
                                device=it.A.device) for it in its]
            # wrapped-form products one pm_mul each, the rest as one batch
            # reusing their evaluations
            rest = [i for i, it in enumerate(its) if not it.wraps]
            for i, it in enumerate(its):
                if it.wraps:
                    polymat.mul(self.p, it.A, it.B, out=outs[i], workspace=self.ws[si],
                                stream=st)
            if rest:
                polymat.mul_batched(self.p, [its[i].A for i in rest], [its[i].B for i in rest],
                                    [outs[i] for i in rest], workspace=self.ws[si], stream=st,
                                    A_evals=[its[i].A_eval for i in rest],
                                    B_evals=[its[i].B_eval for i in rest])
            ev = torch.cuda.Event()
            ev.record(st)
        return ev, outs

    def run(self, arrivals, items, spin_sleep: float = 20e-6):
        n = len(arrivals)
        done_at = [None] * n
        ready = collections.deque()
        inflight = []                  # (stream idx, event, [ids], footprint, outs)
        free = list(range(self.nslots))
        used = 0
        nxt = 0
        batches = 0
        t0 = time.perf_counter()
        completed = 0
        while completed < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                ready.append(nxt)
                nxt += 1
            still = []
            for (si, ev, ids, fp, outs) in inflight:
                if ev.query():
                    tnow = time.perf_counter() - t0
                    for r, C in zip(ids, outs):
                        done_at[r] = tnow
                        if r in self.keep:
                            self.kept[r] = C
                    completed += len(ids)
                    used -= fp
                    free.append(si)
                else:
                    still.append((si, ev, ids, fp, outs))
            inflight = still
            launched = False
            while free and ready:
                ids, fp, solo = [], 0, False
                while ready and len(ids) < self.max_batch:
                    it = self.pool[items[ready[0]]]
                    big = it.work >= self.solo_work
                    if ids and (big or solo):
                        break          # large requests run alone
                    solo = big
                    if used + fp + it.footprint > self.budget and ids:
                        break
                    if used + fp + it.footprint > self.budget and inflight:
                        break          # wait for memory
                    ids.append(ready.popleft())
                    fp += it.footprint
                if not ids:
                    break
                si = free.pop()
                ev, outs = self.launch(si, [self.pool[items[r]] for r in ids])
                inflight.append((si, ev, ids, fp, outs))
                self.admitted.extend(ids)
                used += fp
                self.peak_used = max(self.peak_used, used)
                batches += 1
                launched = True
            if not launched:
                # sleep until the next arrival only when no batch is running;
                # otherwise poll the running batches at a short interval
                wait = arrivals[nxt] - (time.perf_counter() - t0) if nxt < n else 0.0
                if not inflight and not ready and wait > 2 * spin_sleep:
                    time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(spin_sleep)
        wall = time.perf_counter() - t0
        return self._stats(arrivals, items, done_at, wall, batches)

    def _stats(self, arrivals, items, done_at, wall, batches):
        st = _stats(self.pool, arrivals, items, done_at, wall, self.warmup_s)
        st["batches"] = batches
        st["mean_batch"] = len(arrivals) / max(batches, 1)
        return st


def _stats(pool, arrivals, items, done_at, wall, warmup_s):
    """Latency percentiles over the requests that arrive after `warmup_s`;
    throughput over the whole run (all requests' work / wall time)."""
    n = len(arrivals)
    lat = [done_at[r] - arrivals[r] for r in range(n) if arrivals[r] >= warmup_s]
    p50, p99 = _percentiles(lat)
    work = sum(pool[i].m * pool[i].n * pool[i].k * pool[i].d for i in items)
    return {"requests": n, "measured_requests": len(lat), "warmup_s": warmup_s,
            "wall_s": wall, "throughput": work / wall,
            "p50_ms": p50 * 1e3 if p50 is not None else None,
            "p99_ms": p99 * 1e3 if p99 is not None else None}


def run_fifo(p: int, pool: list[PoolItem], arrivals, items, keep=(), warmup_s: float = 0.0):
    """Baseline: one product per launch, issued on one stream as soon as the
    request has arrived, in arrival order; completions observed through
    per-request events. It uses the same resident evaluations as the batching
    server (a one-product pm_mul_batched call), and wrapped-form products run
    as pm_mul calls there too, so the two servers differ only in batching and
    streams."""
    st = torch.cuda.Stream()
    ws = polymat.Workspace()
    n = len(arrivals)
    done_at = [None] * n
    pending = collections.deque()
    kept = {}
    t0 = time.perf_counter()
    nxt = 0
    completed = 0
    while completed < n:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            it = pool[items[nxt]]
            with torch.cuda.stream(st):
                C = torch.empty((2 * it.d - 1, it.m, it.k), dtype=torch.uint32,
                                device=it.A.device)
                if it.wraps or (it.A_eval is None and it.B_eval is None):
                    polymat.mul(p, it.A, it.B, out=C, workspace=ws, stream=st)
                else:
                    polymat.mul_batched(p, [it.A], [it.B], [C], workspace=ws, stream=st,
                                        A_evals=[it.A_eval], B_evals=[it.B_eval])
                ev = torch.cuda.Event()
                ev.record(st)
            pending.append((nxt, ev, C))
            nxt += 1
        while pending and pending[0][1].query():
            r, _, C = pending.popleft()
            done_at[r] = time.perf_counter() - t0
            if r in keep:
                kept[r] = C
            completed += 1
        if not pending and nxt < n:
            wait = arrivals[nxt] - (time.perf_counter() - t0)
            if wait > 40e-6:
                time.sleep(min(wait, 1e-3))
        elif pending:
            time.sleep(20e-6)
    wall = time.perf_counter() - t0
    return _stats(pool, arrivals, items, done_at, wall, warmup_s), kept
