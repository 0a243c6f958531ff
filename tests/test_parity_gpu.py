"""GPU parity: libpm (HIP kernels through the C ABI) against the CPU oracle.

Exact arithmetic, so the bar is bit-exact equality everywhere. Small sizes
compare every coefficient with the oracle's full schoolbook product; the
full-size configurations compare seeded whole output entries one by one plus
random-point and Freivalds checks over all outputs.
"""
from __future__ import annotations

import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1905_04356_amd import binding as Bd  # noqa: E402
from paper_1905_04356_amd import inputs as I  # noqa: E402
from paper_1905_04356_amd import polymat  # noqa: E402

pytestmark = pytest.mark.gpu

P30 = 998244353
P31 = 2013265921
P32 = 4294967291          # largest prime below 2^32: not NTT-friendly


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tensors(p, m, n, k, d, seed, dtype=np.uint32, product=0):
    A = I.polymat(seed, product, I.TENSOR_A, p, d, m, n, dtype)
    B = I.polymat(seed, product, I.TENSOR_B, p, d, n, k, dtype)
    return A, B


def gpu_mul(p, A, B):
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    tC = polymat.mul(p, tA, tB)
    torch.cuda.synchronize()
    return tC.cpu().numpy()


def full_check(p, m, n, k, d, seed=0, dtype=np.uint32):
    say(f"[parity] p={p} m={m} n={n} k={k} d={d} seed={seed} dtype={np.dtype(dtype).name}")
    A, B = tensors(p, m, n, k, d, seed, dtype)
    C = gpu_mul(p, A, B)
    ref = O.polymatmul(p, A, B)
    assert C.shape == ref.shape
    assert C.dtype == dtype
    bad = np.argwhere(C.astype(np.uint64) != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"


def test_config1_full_oracle():
    """8x8 . 8x8, d = 256, p = 998244353: every coefficient."""
    full_check(P30, 8, 8, 8, 256, seed=1)


SMALL = [
    (1, 1, 1, 1), (3, 2, 5, 1), (2, 3, 2, 2), (1, 1, 1, 3), (5, 7, 3, 17),
    (4, 4, 4, 33), (2, 3, 1, 100), (16, 16, 16, 64), (7, 5, 9, 129),
    (8, 12, 4, 257), (3, 3, 3, 1000), (1, 2, 1, 4097), (2, 1, 3, 2049),
    (1, 1, 1, 8193), (1, 1, 2, 16384),
]


@pytest.mark.parametrize("m,n,k,d", SMALL)
@pytest.mark.parametrize("p", [P30, P31])
def test_direct_mode_small(p, m, n, k, d):
    full_check(p, m, n, k, d, seed=2)


@pytest.mark.parametrize("m,n,k,d", [(1, 1, 1, 1), (3, 2, 5, 7), (4, 4, 4, 33),
                                     (2, 5, 3, 300), (1, 1, 1, 4097)])
@pytest.mark.parametrize("p,dtype", [(P32, np.uint32), (97, np.uint32), (2, np.uint32),
                                     (1 << 31, np.uint32),
                                     (1152921504606846883, np.uint64),
                                     ((1 << 62) - 57, np.uint64), (P31, np.uint64)])
def test_crt_and_u64_small(p, dtype, m, n, k, d):
    full_check(p, m, n, k, d, seed=3, dtype=dtype)


@pytest.mark.parametrize("p,dtype", [(P30, np.uint32), (P31, np.uint32), (P32, np.uint32),
                                     ((1 << 62) - 57, np.uint64)])
def test_all_p_minus_one_hits_the_bound(p, dtype):
    """(p-1)^2 = 1 mod p, and over Z each coefficient is exactly the bound
    n*min(c+1, 2d-1-c)*(p-1)^2 used to size the prime set."""
    m, n, k, d = 3, 8, 2, 64
    say(f"[parity] all p-1 p={p}")
    A = np.full((d, m, n), p - 1, dtype=dtype)
    B = np.full((d, n, k), p - 1, dtype=dtype)
    C = gpu_mul(p, A, B)
    want = np.array([n * min(c + 1, 2 * d - 1 - c) % p for c in range(2 * d - 1)],
                    dtype=np.uint64)
    assert np.array_equal(C.astype(np.uint64), np.broadcast_to(want[:, None, None], C.shape))


def test_identity_and_shift():
    p, n, d = P31, 6, 40
    A = np.zeros((d, n, n), dtype=np.uint32)
    A[5] = np.eye(n, dtype=np.uint32)
    _, B = tensors(p, n, n, n, d, 4)
    C = gpu_mul(p, A, B)
    assert not C[:5].any() and np.array_equal(C[5:5 + d], B) and not C[5 + d:].any()


def sampled_check(p, A, B, C, seed, entries, points=4, rounds=2):
    """Seeded whole output entries against the oracle's schoolbook, then
    `points` random-point and `rounds` Freivalds checks over every output."""
    d, m, n = A.shape
    k = B.shape[2]
    pairs = I.sample_pairs(seed, m, k, entries)
    say(f"[parity]   {len(pairs)} whole entries")
    ref = O.polymatmul_entries(p, A, B, pairs)
    for s, (i, j) in enumerate(pairs):
        assert np.array_equal(C[:, i, j].astype(np.uint64), ref[s]), (i, j)
    say(f"[parity]   {points} points, {rounds} Freivalds rounds")
    assert O.point_check(p, A, B, C, seed=seed, points=points)
    assert O.freivalds_check(p, A, B, C, seed=seed, rounds=rounds)


def test_config2_full_size_sampled():
    """64x64 . 64x32, d = 4096, p = 2013265921 at full size: 256 seeded whole
    entries (of 2048) against the oracle, plus 4 random-point and 2 Freivalds
    checks on all outputs."""
    p, m, n, k, d = P31, 64, 64, 32, 4096
    say("[parity] config 2 full size")
    A, B = tensors(p, m, n, k, d, seed=2)
    C = gpu_mul(p, A, B)
    sampled_check(p, A, B, C, seed=2, entries=256)


def test_config4_full_size_whole_product():
    """60-bit non-NTT prime, 32x32 . 32x32, d = 2048, uint64, five CRT primes:
    every coefficient against the oracle's schoolbook, plus the point and
    Freivalds checks."""
    p = I.seeded_prime_60(4)
    assert O.is_prime(p)
    info = Bd.pm_plan(p, 32, 32, 32, 2048, 8)
    assert info.mode == 1 and info.num_primes == 5
    say(f"[parity] config 4 full size p={p}")
    A, B = tensors(p, 32, 32, 32, 2048, seed=4, dtype=np.uint64)
    C = gpu_mul(p, A, B)
    say("[parity]   whole product (schoolbook)")
    ref = O.polymatmul(p, A, B)
    bad = np.argwhere(C != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"
    assert O.point_check(p, A, B, C, seed=4, points=4)
    assert O.freivalds_check(p, A, B, C, seed=4, rounds=2)


def test_batched_equals_single_calls():
    p = P30
    shapes = I.batched_shapes(7, 12, log2_dmin=1.0, log2_dmax=10.0)
    say(f"[parity] batched {len(shapes)} products")
    As, Bs, refs = [], [], []
    for idx, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=7, product=idx)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        refs.append(polymat.mul(p, As[-1], Bs[-1]).clone())
    outs = polymat.mul_batched(p, As, Bs)
    torch.cuda.synchronize()
    for (m, n, k, d), C, R, A, B in zip(shapes, outs, refs, As, Bs):
        assert torch.equal(C, R)
    # and against the oracle for the small ones
    for (m, n, k, d), C, A, B in zip(shapes, outs, As, Bs):
        if m * n * k * d * d <= 1 << 26:
            ref = O.polymatmul(p, A.cpu().numpy(), B.cpu().numpy())
            assert np.array_equal(C.cpu().numpy().astype(np.uint64), ref)


def test_repeat_runs_are_identical():
    p, m, n, k, d = P31, 16, 16, 16, 1000
    A, B = tensors(p, m, n, k, d, seed=9)
    first = gpu_mul(p, A, B)
    for _ in range(3):
        assert np.array_equal(gpu_mul(p, A, B), first)


def test_check_residues():
    x = torch.from_numpy(np.array([0, 5, 96, 97, 98, 1 << 31, 3], dtype=np.uint32)).cuda()
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    n = Bd.pm_check_residues(97, x.data_ptr(), x.numel(), 4, ws.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    assert n == 3


@pytest.mark.parametrize("m,n,k,d", [(8, 8, 8, 256), (16, 64, 16, 100), (5, 12, 7, 33),
                                     (17, 4, 33, 65), (64, 64, 32, 64), (3, 128, 2, 20),
                                     (32, 68, 48, 9), (128, 128, 128, 6), (128, 64, 96, 5),
                                     (20, 252, 3, 2)])
@pytest.mark.parametrize("p", [P30, P31, P32])
def test_pointwise_variants_match_oracle(p, m, n, k, d):
    """Both pointwise kernels (int8-MFMA limbs and VALU) against the oracle."""
    Bd.tune_load("")
    try:
        info = Bd.pm_plan(p, m, n, k, d, 4)
        assert info.pointwise == 1, "shape expected on the MFMA path"
        full_check(p, m, n, k, d, seed=11)
        Bd.tune_load('{"format": "pm-tune-1", "entries": [{"knobs": {"pointwise": 0}}]}')
        assert Bd.pm_plan(p, m, n, k, d, 4).pointwise == 0
        full_check(p, m, n, k, d, seed=11)
    finally:
        torch.cuda.synchronize()
        Bd.tune_load(None)


@pytest.mark.parametrize("p,m,n,k,d", [
    (P30, 128, 8, 128, 2048),    # 4 A groups + 1 B block per thread; ng = 16, 32 block columns
    (P31, 128, 128, 128, 2048),  # 8 A groups + 2 B blocks per thread
    (P30, 96, 36, 112, 1500),    # contraction padded 36 -> 64
    (P31, 121, 20, 4, 1100),     # rows padded 121 -> 128, 4 columns
    (P30, 40, 200, 24, 700),     # ng = 64: four 16-group bands per block column
    (P32, 128, 32, 64, 600),     # three CRT primes (one grid row each)
])
def test_pipelined_pointwise_long_sequences(p, m, n, k, d):
    """Limb planes above 44 KiB take the pipelined MFMA kernel, whose
    workgroups each run a sequence of points (here 3-16 per workgroup)
    while the next point loads; outputs against the oracle."""
    info = Bd.pm_plan(p, m, n, k, d, 4)
    assert info.pointwise == 1
    say(f"[parity] pipelined pointwise p={p} m={m} n={n} k={k} d={d}")
    A, B = tensors(p, m, n, k, d, seed=13)
    C = gpu_mul(p, A, B)
    sampled_check(p, A, B, C, seed=13, entries=3)


@pytest.mark.parametrize("m,n,k", [(16, 64, 16), (24, 16, 40), (16, 4, 16)])
def test_mfma_limb_extremes(m, n, k):
    """Residues at the centring boundary ((q-1)/2, (q+1)/2), 0, 1, q-1 in every
    position exercise the largest limb magnitudes, with the contraction padded
    to 64 and packed (n <= 16)."""
    p, d = P31, 8
    vals = np.array([0, 1, (p - 1) // 2, (p + 1) // 2, p - 1, p - 2], dtype=np.uint32)
    rng = np.random.default_rng(12)
    A = vals[rng.integers(0, len(vals), size=(d, m, n))]
    B = vals[rng.integers(0, len(vals), size=(d, n, k))]
    assert Bd.pm_plan(p, m, n, k, d, 4).pointwise == 1
    C = gpu_mul(p, A, B)
    assert np.array_equal(C.astype(np.uint64), O.polymatmul(p, A, B))


def _batch_vs_single(p, shapes, seed, dtype=np.uint32, oracle_limit=1 << 26):
    As, Bs, refs = [], [], []
    for idx, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=seed, product=idx, dtype=dtype)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        refs.append(polymat.mul(p, As[-1], Bs[-1]).clone())
    torch.cuda.synchronize()
    outs = polymat.mul_batched(p, As, Bs)
    torch.cuda.synchronize()
    for i, (C, R) in enumerate(zip(outs, refs)):
        assert torch.equal(C, R), f"product {i} {shapes[i]} differs from its single call"
    checked = 0
    for (m, n, k, d), C, A, B in zip(shapes, outs, As, Bs):
        if m * n * k * d * d <= oracle_limit:
            ref = O.polymatmul(p, A.cpu().numpy(), B.cpu().numpy())
            assert np.array_equal(C.cpu().numpy().astype(np.uint64), ref)
            checked += 1
        else:
            Cn, An, Bn = C.cpu().numpy(), A.cpu().numpy(), B.cpu().numpy()
            assert O.point_check(p, An, Bn, Cn, seed=seed, points=1)
    return checked


def test_batched_config3_distribution_subset():
    """24 products drawn by the batched shape rule (degrees up to 8192, so
    split and unsplit transforms and both pointwise kernels mix in one batch):
    byte-identical to one call per product; oracle on the small ones, a
    random-point check on the rest."""
    shapes = [(min(m, 32), min(n, 32), min(k, 32), d) for (m, n, k, d) in
              I.batched_shapes(3, 24)]
    say(f"[parity] batched subset {shapes}")
    _batch_vs_single(P30, shapes, seed=13)


def test_batched_crt_u64_and_u32():
    p = I.seeded_prime_60(5)
    shapes = [(3, 4, 2, 40), (8, 8, 8, 300), (1, 1, 1, 1), (16, 32, 16, 1500), (5, 3, 7, 3000)]
    say("[parity] batched CRT u64")
    _batch_vs_single(p, shapes, seed=14, dtype=np.uint64)
    say("[parity] batched CRT u32")
    _batch_vs_single(P32, shapes, seed=15)


def test_batched_pipelined_pointwise_crt():
    """Large limb planes in batched calls take the pipelined pointwise tiles
    (phase 2 with 4 register slots, phase 6 with 8) and small contractions
    the packed form; CRT moduli with 64-bit and 32-bit elements."""
    shapes = [(128, 128, 128, 300), (128, 64, 96, 200), (96, 36, 112, 260),
              (128, 8, 128, 150), (40, 200, 24, 90), (64, 64, 32, 120)]
    for sh in shapes:
        assert Bd.pm_plan(P30, *sh, 4).pointwise == 1
    say("[parity] batched pipelined pointwise, CRT u64")
    _batch_vs_single(I.seeded_prime_60(6), shapes, seed=21, dtype=np.uint64)
    say("[parity] batched pipelined pointwise, CRT u32")
    _batch_vs_single(P32, shapes, seed=22)


def test_batched_single_product_and_repeats():
    shapes = [(64, 64, 32, 4096)]
    A, B = tensors(P31, 64, 64, 32, 4096, seed=16)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = polymat.mul(P31, tA, tB).clone()
    for _ in range(2):
        (C,) = polymat.mul_batched(P31, [tA], [tB])
        torch.cuda.synchronize()
        assert torch.equal(C, ref)


def test_config3_full_batch_sampled():
    """Config 3 at full size and in the launch configuration the benchmark
    times: 512 products (batched shape rule, seed 3) in one batched call.
    Checks: the device generator reproduces the host generator; every one of
    the 512 products passes 2 random-point checks and 1 Freivalds round
    against the oracle; 16 seeded products with m n k d^2 <= 2^33 are compared
    whole with the oracle's schoolbook; 16 seeded products are byte-identical
    to their single calls."""
    p, seed = P30, 3
    shapes = I.batched_shapes(seed, 512)
    dev = torch.device("cuda")
    say("[parity] config 3 full batch: generating")
    As = [I.polymat_torch(seed, i, I.TENSOR_A, p, d, m, n, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    Bs = [I.polymat_torch(seed, i, I.TENSOR_B, p, d, n, k, dev) for i, (m, n, k, d) in
          enumerate(shapes)]
    m0, n0, k0, d0 = shapes[5]
    assert np.array_equal(Bs[5].cpu().numpy(), I.polymat(seed, 5, I.TENSOR_B, p, d0, n0, k0))
    say("[parity] config 3 full batch: batched call")
    outs = polymat.mul_batched(p, As, Bs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    for i in rng.choice(512, size=16, replace=False):
        R = polymat.mul(p, As[i], Bs[i])
        torch.cuda.synchronize()
        assert torch.equal(R, outs[i]), f"product {i} {shapes[i]}"
    small = [i for i, (m, n, k, d) in enumerate(shapes) if m * n * k * d * d <= 1 << 33]
    whole = set(int(i) for i in rng.choice(small, size=min(16, len(small)), replace=False))
    say(f"[parity] config 3: points and Freivalds on all 512, {len(whole)} whole products")
    for i, (m, n, k, d) in enumerate(shapes):
        A, B, C = As[i].cpu().numpy(), Bs[i].cpu().numpy(), outs[i].cpu().numpy()
        assert O.point_check(p, A, B, C, seed=1000 + i, points=2), f"product {i} {shapes[i]}"
        assert O.freivalds_check(p, A, B, C, seed=1000 + i, rounds=1), f"product {i} {shapes[i]}"
        if i in whole:
            assert np.array_equal(C.astype(np.uint64), O.polymatmul(p, A, B)), \
                f"product {i} {shapes[i]}"
        if i % 64 == 63:
            say(f"[parity] config 3: {i + 1} products checked")


def test_serving_results_same_alone_and_in_mix():
    """Continuous batching over 4 streams with resident evaluations, on
    configuration-3 shapes (uncapped, up to 128x128.128x128): sampled requests
    are byte-identical to the same product computed alone (one pm_mul call,
    no cached evaluations) and to the FIFO baseline, and each passes a
    random-point check against the oracle (the small ones whole)."""
    from paper_1905_04356_amd import serving as S
    p = P30
    dev = torch.device("cuda")
    pool = S.make_pool(p, 21, 12, dev, with_evals=True)
    arrivals, items = S.trace(21, 600.0, 0.5, len(pool))
    keep = list(range(0, len(arrivals), max(1, len(arrivals) // 24)))
    srv = S.Server(p, pool, 8 << 30, streams=4, keep=keep)
    stats = srv.run(arrivals, items)
    torch.cuda.synchronize()
    say(f"[serving] {stats}")
    assert stats["requests"] == len(arrivals) and stats["batches"] >= 1
    fifo, kept_fifo = S.run_fifo(p, pool, arrivals, items, keep=keep)
    torch.cuda.synchronize()
    for r in keep:
        it = pool[items[r]]
        alone = polymat.mul(p, it.A, it.B)
        torch.cuda.synchronize()
        assert torch.equal(srv.kept[r], alone), r
        assert torch.equal(kept_fifo[r], alone), r
        A, B, C = it.A.cpu().numpy(), it.B.cpu().numpy(), alone.cpu().numpy()
        if it.m * it.n * it.k * it.d * it.d <= 1 << 28:
            assert np.array_equal(C.astype(np.uint64), O.polymatmul(p, A, B)), r
        else:
            assert O.point_check(p, A, B, C, seed=r, points=1), r


def test_eval_entry_points_match_plain_products():
    """pm_eval_* evaluations fed to a batch give the same bytes as products
    that transform their own operands (direct and CRT moduli)."""
    for p, dt in ((P31, np.uint32), (I.seeded_prime_60(6), np.uint64)):
        shapes = [(5, 8, 3, 100), (16, 32, 16, 2500), (1, 4, 2, 1)]
        As, Bs, Ae, Be = [], [], [], []
        for i, (m, n, k, d) in enumerate(shapes):
            A, B = tensors(p, m, n, k, d, seed=22, product=i, dtype=dt)
            As.append(torch.from_numpy(A).cuda())
            Bs.append(torch.from_numpy(B).cuda())
            Ae.append(polymat.evaluate(p, As[-1], 0))
            Be.append(polymat.evaluate(p, Bs[-1], 1))
        ref = polymat.mul_batched(p, As, Bs)
        got = polymat.mul_batched(p, As, Bs, A_evals=Ae, B_evals=Be)
        half = polymat.mul_batched(p, As, Bs, A_evals=Ae, B_evals=[None] * 3)
        # two products: the direct (per-product launch) path of small batches
        two = polymat.mul_batched(p, As[:2], Bs[:2], A_evals=[None, Ae[1]], B_evals=Be[:2])
        torch.cuda.synchronize()
        for r, g, h in zip(ref, got, half):
            assert torch.equal(r, g) and torch.equal(r, h)
        for r, t in zip(ref, two):
            assert torch.equal(r, t)


def test_batched_graph_replays_match_eager():
    """A batch that repeats is run eagerly, then captured into a HIP graph,
    then replayed: with eager work and synchronisations between calls and the
    outputs cleared each time, every call must reproduce the single-call
    results."""
    p = P30
    shapes = [(4, 8, 4, 100), (16, 16, 8, 3000), (8, 4, 8, 40), (32, 32, 32, 700),
              (4, 4, 4, 1), (64, 32, 16, 2100)]
    As, Bs, refs = [], [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=23, product=i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        refs.append(polymat.mul(p, As[-1], Bs[-1]).clone())
    outs = [torch.empty_like(r) for r in refs]
    ws = polymat.Workspace()
    for call in range(5):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        polymat.mul_batched(p, As, Bs, outs, workspace=ws)
        # unrelated eager work between calls
        polymat.mul(p, As[0], Bs[0])
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), f"call {call} product {i}"


@pytest.mark.parametrize("fill", ["max", "random"])
@pytest.mark.parametrize("n", [64, 12])
def test_mfma_centred_limbs_for_primes_above_0x7f7f7f7f(fill, n):
    """A direct-mode prime above 0x7F7F7F7F (2^31 - 1 at d = 1, one point)
    takes the MFMA kernel's centred digit path; all-(p-1) and random inputs,
    padded and packed contractions."""
    p, m, k, d = (1 << 31) - 1, 8, 8, 1
    info = Bd.pm_plan(p, m, n, k, d, 4)
    assert info.mode == 0 and info.pointwise == 1
    if fill == "max":
        A = np.full((d, m, n), p - 1, dtype=np.uint32)
        B = np.full((d, n, k), p - 1, dtype=np.uint32)
    else:
        A, B = tensors(p, m, n, k, d, seed=13)
    C = gpu_mul(p, A, B)
    assert np.array_equal(C.astype(np.uint64), O.polymatmul(p, A, B))


def _wrapped(p, A, B):
    """The product on the GPU and whether it took the wrapped path (in direct
    mode only the wrap's correction kernel is timed as Chinese remaindering)."""
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Bd.pm_profile_begin()
    tC = polymat.mul(p, tA, tB)
    stats = Bd.pm_profile_end()
    torch.cuda.synchronize()
    return tC.cpu().numpy(), stats["crt"][1] > 0


@pytest.mark.parametrize("p,m,n,k,d,wraps", [
    (P30, 3, 4, 2, 600, False),      # small products: plain transforms
    (P30, 64, 64, 64, 1100, False),  # (mn + nk + mk) 2^11 below 2^25
    (P30, 128, 128, 64, 560, True),  # 2^10 points + a 95-coefficient top
    (P30, 128, 128, 64, 600, False), # top 175 > 2^10 / 8: three-quarter transform
    (P31, 64, 64, 64, 2100, True),   # 2^12 + 103
    (P30, 64, 64, 64, 2304, True),   # top 511 <= 2^12 / 8: wrapped
    (P30, 64, 64, 64, 2306, False),  # top 515: the 6144-point three-quarter transform
    (P30, 64, 64, 32, 4600, True),   # L = 2^14: tops up to 2^13 / 4 (here 1007) wrap
])
def test_wrapped_lengths(p, m, n, k, d, wraps):
    """Products with 2^j < 2d-1 <= 1.25 2^j and enough work: a cyclic product
    on 2^j points, the top coefficients from a short window product, and the
    correction; sampled entries against the oracle, points and Freivalds on
    all, and the path taken as the rule says."""
    say(f"[parity] wrapped p={p} m={m} n={n} k={k} d={d}")
    A, B = tensors(p, m, n, k, d, seed=14)
    C, took = _wrapped(p, A, B)
    assert took == wraps
    sampled_check(p, A, B, C, seed=14, entries=4)


def test_wrapped_crt_u64():
    """The wrapped path in CRT mode with 64-bit residues."""
    p, m, n, k, d = (1 << 61) - 1, 64, 64, 64, 2100
    say("[parity] wrapped CRT u64")
    A, B = tensors(p, m, n, k, d, seed=18, dtype=np.uint64)
    C = gpu_mul(p, A, B)
    sampled_check(p, A, B, C, seed=18, entries=2)


def test_wrapped_equals_plain_transforms():
    p, m, n, k = P30, 64, 64, 64
    for d in (2050, 2100, 2304):
        A, B = tensors(p, m, n, k, d, seed=15)
        wrapped, took = _wrapped(p, A, B)
        assert took, d
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        plain = polymat.middle(p, tA, tB, 0, 2 * d - 1)   # whole window: plain transforms
        torch.cuda.synchronize()
        assert np.array_equal(wrapped, plain.cpu().numpy()), d


def test_batched_wraps_like_single_calls():
    """A batch takes the wrapped form for the products pm_mul wraps (two
    entries and a correction each) and plain transforms for the others."""
    p = P30
    shapes = [(128, 128, 64, 1100), (8, 8, 8, 100), (64, 64, 64, 2100), (64, 64, 64, 1100)]
    As, Bs = [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=19, product=i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    Bd.pm_profile_begin()
    outs = polymat.mul_batched(p, As, Bs)
    stats = Bd.pm_profile_end()
    torch.cuda.synchronize()
    assert stats["crt"][1] == 2                       # two corrections: two wrapped products
    for (m, n, k, d), tA, tB, C in zip(shapes, As, Bs, outs):
        plain = polymat.middle(p, tA, tB, 0, 2 * d - 1)
        torch.cuda.synchronize()
        assert torch.equal(C, plain), (m, n, k, d)


def test_kernel_timing_counts_only_unpaused_launches():
    """Timed launches carry dispatch events; paused ones are not counted, and
    timing changes no result."""
    p, m, n, k, d = P31, 16, 16, 8, 4096
    A, B = tensors(p, m, n, k, d, seed=16)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = polymat.mul(p, tA, tB)
    Bd.pm_profile_begin()
    C1 = polymat.mul(p, tA, tB)
    one = Bd.pm_profile_end()
    Bd.pm_profile_begin()
    C2 = polymat.mul(p, tA, tB)
    Bd.pm_profile_pause(True)
    C3 = polymat.mul(p, tA, tB)
    Bd.pm_profile_pause(False)
    C4 = polymat.mul(p, tA, tB)
    two = Bd.pm_profile_end()
    torch.cuda.synchronize()
    for C in (C1, C2, C3, C4):
        assert torch.equal(C, ref)
    for kind in ("ntt_fwd", "pointwise", "ntt_inv"):
        assert one[kind][1] >= 1 and one[kind][0] > 0.0, kind
        assert two[kind][1] == 2 * one[kind][1], kind
    assert one["crt"][1] == 0 and one["batched"][1] == 0


def test_operand_transforms_share_launches():
    """Where both operands' split transforms have the same pass structure, the
    forward transforms of A and B run as one first-pass and one block-step
    launch (two launches instead of four), with register tiles or with
    LDS-resident ones; the result equals the one from each operand's
    evaluations made alone. Short unsplit transforms run as one launch for
    both operands."""
    p, m, n, k, d = P31, 64, 64, 32, 3000
    A, B = tensors(p, m, n, k, d, seed=21)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Bd.pm_profile_begin()
    C = polymat.mul(p, tA, tB)
    st = Bd.pm_profile_end()
    assert st["ntt_fwd"][1] == 2, st["ntt_fwd"]
    Bd.tune_load(json.dumps({"format": "pm-tune-1", "entries": [{"knobs": {"reg_tile": 0}}]}))
    try:
        Bd.pm_profile_begin()
        C2 = polymat.mul(p, tA, tB)
        st2 = Bd.pm_profile_end()
        torch.cuda.synchronize()
    finally:
        Bd.tune_load(None)
    assert st2["ntt_fwd"][1] == 2, st2["ntt_fwd"]        # LDS-resident tiles, paired too
    assert torch.equal(C, C2)
    # each operand transformed alone (evaluations), then the product from them
    Ae, Be = polymat.evaluate(p, tA, 0), polymat.evaluate(p, tB, 1)
    (C3,) = polymat.mul_batched(p, [tA], [tB], A_evals=[Ae], B_evals=[Be])
    torch.cuda.synchronize()
    assert torch.equal(C, C3)
    sampled_check(p, A, B, C.cpu().numpy(), seed=21, entries=4)
    # short lengths (one LDS kernel per operand): one launch for both, with
    # 16-byte vectors, and with 1-word vectors where an entry count is odd;
    # split transforms with LDS-resident block tiles (few entries): two
    for (p, m, n, k, d, launches) in ((P30, 8, 8, 8, 256, 1), (P31, 3, 5, 7, 300, 1),
                                      (P30, 4, 6, 4, 500, 1), (P30, 4, 6, 4, 1000, 2),
                                      (P31, 3, 5, 7, 2500, 2)):
        A, B = tensors(p, m, n, k, d, seed=22)
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        Bd.pm_profile_begin()
        C = polymat.mul(p, tA, tB)
        st = Bd.pm_profile_end()
        torch.cuda.synchronize()
        assert st["ntt_fwd"][1] == launches, (m, n, k, d, st["ntt_fwd"])
        assert np.array_equal(C.cpu().numpy().astype(np.uint64), O.polymatmul(p, A, B))


@pytest.mark.parametrize("p,m,n,k,d", [
    (P30, 8, 8, 8, 1024),     # L = 2^11: block passes {4, 3}, 64-entry tiles
    (P31, 8, 8, 6, 2048),     # 2^12: {4, 4}, 32-entry tiles, 48 entries (ragged)
    (P30, 8, 4, 6, 4096),     # 2^13: {3, 3, 3}, 16-entry tiles, 24 and 48 entries
    (P31, 4, 4, 2, 8192),     # 2^14: {4, 3, 3}, 8-entry tiles
    (P30, 3, 3, 1, 6000),     # 2^14, odd entry counts: LDS-tile path
    (P30, 2, 2, 3, 16384),    # 2^15: {4, 4, 3}, 4-entry tiles, 6 entries
    (P31, 3, 3, 1, 16384),    # 2^15, odd entry counts: 1-word vectors, LDS-tile path
])
def test_block_step_pass_structures(p, m, n, k, d):
    """Split transforms at every length from 2^11 to 2^15, so the block step
    runs each of its pass structures (forward and inverse), with tiles whose
    last entries lie beyond the matrix."""
    say(f"[parity] block step p={p} m={m} n={n} k={k} d={d}")
    A, B = tensors(p, m, n, k, d, seed=17)
    C = gpu_mul(p, A, B)
    sampled_check(p, A, B, C, seed=17, entries=2 if d >= 16384 else 4)


def test_batched_wraps_crt_u64():
    """Wrapped products inside a batch in CRT mode with 64-bit residues equal
    single pm_mul calls (whose wrapped path is checked against the oracle)."""
    p = (1 << 61) - 1
    shapes = [(64, 64, 64, 2100), (4, 4, 4, 300), (64, 64, 64, 2100)]
    As, Bs = [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=21, dtype=np.uint64, product=i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    outs = polymat.mul_batched(p, As, Bs)
    for tA, tB, C in zip(As, Bs, outs):
        ref = polymat.mul(p, tA, tB)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
