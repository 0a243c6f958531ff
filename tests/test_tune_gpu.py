"""Launch shapes from the tuning table never change a result: products under
tables that force other pass structures, block-step threads and tiles,
column item widths, LDS instead of register tiles, VALU pointwise and
pipelined pointwise slots equal the oracle coefficient by coefficient, single
and batched, direct and CRT moduli; evaluations made under one table feed
products planned under another. Wrapped lengths with the size bound lowered
(a global knob) are compared with the oracle on small products, including
the extreme tops t = 1 and t = 2^j / 4."""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(autouse=True)
def _restore_table():
    yield
    torch.cuda.synchronize()
    Bd.tune_load(None)


def table(knobs, glob=None):
    t = {"format": "pm-tune-1", "entries": [{"knobs": knobs}]}
    if glob:
        t["global"] = glob
    return json.dumps(t)


TABLES = [
    {"split": 3, "maxr": 3, "blk_nt": 512, "colvec_fwd": 2, "colvec_inv": 1},
    {"split": 2, "maxr": 2, "reg_tile": 0, "pointwise": 0},
    {"blk_tile_log": 12, "colvec_fwd": 1, "pw_pipe": 2, "pw_small_lds": 0},
    {"blk_tile_log": 14, "blk_nt": 512, "maxr": 3, "pw_pipe": 0, "pw_small_lds": 0},
    {"split": 0, "maxr": 4, "pw_pipe": 1, "pw_small_lds": 0},
    {"split": 5, "colvec_fwd": 4, "colvec_inv": 4},
    {"split": 5, "maxr": 3, "blk_nt": 512, "blk_tile_log": 14, "colvec_fwd": 1},
]
GLOBAL = {"batch_tile_log": 13, "batch_pw_work": 2048, "batch_direct_max": 0,
          "batch_graph": 0}

SHAPES = [  # (p, m, n, k, d, dtype): lengths 2^11 .. 2^13, odd entry counts
    (P31, 16, 16, 16, 1500, np.uint32),
    (P30, 8, 12, 4, 3000, np.uint32),
    (P31, 5, 7, 3, 600, np.uint32),
    (P30, 3, 5, 7, 2000, np.uint32),
    (1152921504606846883, 4, 8, 4, 700, np.uint64),
]


def operands(p, m, n, k, d, dtype, seed):
    A = I.polymat(seed, 0, I.TENSOR_A, p, d, m, n, dtype)
    B = I.polymat(seed, 0, I.TENSOR_B, p, d, n, k, dtype)
    return A, B


@pytest.mark.parametrize("ti", range(len(TABLES)))
def test_products_under_forced_knobs_equal_the_oracle(ti):
    knobs = TABLES[ti]
    if knobs.get("split") == 0:
        shapes = [s for s in SHAPES if 2 * s[4] - 1 <= 4096]   # unsplit: L <= 2^12
    else:
        shapes = SHAPES
    say(f"[tune] table {ti}: {knobs}")
    Bd.tune_load(table(knobs, GLOBAL))
    refs, As, Bs = [], [], []
    for idx, (p, m, n, k, d, dt) in enumerate(shapes):
        A, B = operands(p, m, n, k, d, dt, seed=40 + idx)
        assert Bd.pm_plan(p, m, n, k, d, 4 if dt == np.uint32 else 8).tune_entry == 0
        ref = O.polymatmul(p, A, B)
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        C = polymat.mul(p, tA, tB)
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy().astype(np.uint64), ref), (ti, idx)
        refs.append(ref)
        As.append(tA)
        Bs.append(tB)
    # the same products in one batched call per modulus and element size
    groups = {}
    for idx, s in enumerate(shapes):
        groups.setdefault((s[0], s[5]), []).append(idx)
    for (p, dt), ids in groups.items():
        outs = polymat.mul_batched(p, [As[i] for i in ids], [Bs[i] for i in ids])
        torch.cuda.synchronize()
        for i, C in zip(ids, outs):
            assert np.array_equal(C.cpu().numpy().astype(np.uint64), refs[i]), (ti, i)


@pytest.mark.parametrize("ta,tb,tc", [
    ({"split": 3, "maxr": 2}, {"split": 4, "maxr": 4, "reg_tile": 0}, {"split": 2, "maxr": 3}),
    ({"split": 5}, {"split": 4}, {"split": 5, "maxr": 3}),
])
def test_evaluations_under_one_table_feed_products_under_another(ta, tb, tc):
    """The point order of evaluations does not depend on the pass structure."""
    p, m, n, k, d = P31, 8, 16, 4, 1800
    A, B = operands(p, m, n, k, d, np.uint32, seed=50)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = O.polymatmul(p, A, B)
    Bd.tune_load(table(ta))
    Ae = polymat.evaluate(p, tA, 0)
    torch.cuda.synchronize()
    Bd.tune_load(table(tb))
    Be = polymat.evaluate(p, tB, 1)
    torch.cuda.synchronize()
    Bd.tune_load(table(tc))
    (C,) = polymat.mul_batched(p, [tA], [tB], A_evals=[Ae], B_evals=[Be])
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.uint64), ref)


@pytest.mark.parametrize("p,m,n,k,d,j", [
    (P30, 3, 4, 2, 513, 10),       # 2d - 1 = 1025 = 2^10 + 1: top t = 1
    (P30, 2, 3, 2, 640, 10),       # 1279 = 2^10 + 255: t = 2^10 / 4 - 1
    (P30, 4, 4, 4, 641, 10),       # 1281 = 2^10 + 257 > 2^10 + 2^10 / 4: plain
    (P31, 5, 2, 3, 1025, 11),      # 2049 = 2^11 + 1
    (P31, 3, 3, 3, 1280, 11),      # 2559 = 2^11 + 511 = 2^11 + 2^11 / 4 - 1
    (P30, 2, 2, 2, 4097, 13),      # 8193 = 2^13 + 1
])
def test_small_wrapped_products_equal_the_oracle(p, m, n, k, d, j):
    """The wrapped form (cyclic product on 2^j points, short top product,
    correction) on small products, every coefficient against the oracle."""
    # (three-quarter transforms off: with them the wrapped form keeps only
    # tops up to 2^j / 8 at these lengths)
    Bd.tune_load(json.dumps({"format": "pm-tune-1",
                             "global": {"wrap_min_work_log": 0, "trunc34": 0}}))
    t = 2 * d - 1 - (1 << j)
    want_j = j if t <= (1 << j) // 4 else 0
    assert Bd.pm_plan(p, m, n, k, d, 4).wrap_log2_len == want_j
    A, B = operands(p, m, n, k, d, np.uint32, seed=60 + d)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = polymat.mul(p, tA, tB)
    torch.cuda.synchronize()
    ref = O.polymatmul(p, A, B)
    bad = np.argwhere(C.cpu().numpy().astype(np.uint64) != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"


def test_large_products_of_a_batch_run_as_single_products():
    """With batch_single_min_log, the products of a batched call with at
    least that much transform work run on the single-product kernels and the
    rest in the phase launches; results equal the all-phase batch and the
    oracle (sampled), for thresholds that take none, some and all of them."""
    p = P30
    shapes = [(64, 32, 64, 2000), (8, 8, 8, 300), (32, 64, 16, 1500), (4, 4, 4, 50),
              (16, 16, 16, 3000), (64, 64, 64, 700)]
    As, Bs, refs = [], [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = operands(p, m, n, k, d, np.uint32, seed=70 + i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        refs.append(O.polymatmul_entries(p, A, B, [(0, 0), (m - 1, k - 1)]))
    results = {}
    for v in (0, 24, 23, 1):
        Bd.tune_load(table({}, {"batch_single_min_log": v}))
        say(f"[tune] batch_single_min_log={v}")
        Bd.pm_profile_begin()
        for _ in range(3):      # eager, graph capture, replay
            outs = polymat.mul_batched(p, As, Bs)
        st = Bd.pm_profile_end()
        torch.cuda.synchronize()
        # the phase launches run while some products remain for them
        assert (st["batched"][1] > 0) == (v != 1), (v, st["batched"])
        results[v] = [C.cpu().numpy() for C in outs]
    for v in (24, 23, 1):
        for a, b in zip(results[0], results[v]):
            assert np.array_equal(a, b), v
    for (m, n, k, d), C, ref in zip(shapes, results[0], refs):
        got = np.stack([C[:, 0, 0], C[:, m - 1, k - 1]]).astype(np.uint64)
        assert np.array_equal(got, np.asarray(ref).reshape(got.shape)), (m, n, k, d)


def test_lazy_butterflies_change_no_result():
    """Register-tile block steps with Harvey's lazy range ([0, 2q), moduli
    with 2q - 1 <= 0x7F7F7F7F) and with canonical residues give the same
    products, single and batched, with evaluations, at full and
    three-quarter lengths, with LDS-resident tiles on one side (global knob
    lazy)."""
    p = P30
    shapes = [(16, 16, 16, 1500), (8, 12, 4, 3000), (5, 7, 3, 2100), (16, 16, 8, 4096)]
    As, Bs, refs = [], [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = operands(p, m, n, k, d, np.uint32, seed=90 + i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        refs.append(O.polymatmul(p, A, B))
    got = {}
    for lazy in (1, 0):
        Bd.tune_load(table({}, {"lazy": lazy}))
        say(f"[tune] lazy={lazy}")
        singles = [polymat.mul(p, a, b) for a, b in zip(As, Bs)]
        batched = polymat.mul_batched(p, As, Bs)
        ev = [polymat.mul_batched(p, [a], [b], A_evals=[polymat.evaluate(p, a, 0)])[0]
              for a, b in zip(As, Bs)]
        torch.cuda.synchronize()
        got[lazy] = [c.cpu().numpy().astype(np.uint64) for c in singles + batched + ev]
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)
    for i, ref in enumerate(refs):
        assert np.array_equal(got[1][i], ref), shapes[i]


@pytest.mark.parametrize("crt_fused", [1, 0])
def test_lazy_butterflies_in_crt_mode(crt_fused):
    """CRT products take primes below 2^30 where as many suffice, so their
    register-tile block steps keep lazy residues too: lazy and canonical
    butterflies give the same products (single and batched, 60-bit u64 and
    32-bit u32 moduli, with the reconstruction folded into the last inverse
    pass or separate, full and three-quarter lengths), equal to the oracle."""
    p60, p32 = I.seeded_prime_60(4), 4294967291
    cases = [(p60, 8, 8, 8, 1500, np.uint64), (p60, 5, 7, 3, 2100, np.uint64),
             (p32, 8, 16, 4, 3000, np.uint32), (p32, 3, 5, 7, 1100, np.uint32)]
    As, Bs, refs = {}, {}, {}
    for i, (p, m, n, k, d, dt) in enumerate(cases):
        info = Bd.pm_plan(p, m, n, k, d, 8 if dt == np.uint64 else 4)
        qs = [info.primes[j] for j in range(info.num_primes)]
        assert info.mode == 1 and all(2 * q - 1 <= 0x7F7F7F7F for q in qs), qs
        A, B = operands(p, m, n, k, d, dt, seed=120 + i)
        As[i], Bs[i] = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        refs[i] = O.polymatmul(p, A, B)
    got = {}
    for lazy in (1, 0):
        Bd.tune_load(table({}, {"lazy": lazy, "crt_fused": crt_fused}))
        say(f"[tune] crt lazy={lazy} crt_fused={crt_fused}")
        outs = []
        for p in (p60, p32):
            idx = [i for i, c in enumerate(cases) if c[0] == p]
            outs += [polymat.mul(p, As[i], Bs[i]) for i in idx]
            outs += polymat.mul_batched(p, [As[i] for i in idx], [Bs[i] for i in idx])
        torch.cuda.synchronize()
        got[lazy] = [c.cpu().numpy().astype(np.uint64) for c in outs]
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)
    order = [0, 1, 0, 1, 2, 3, 2, 3]
    for c, i in zip(got[1], order):
        assert np.array_equal(c, refs[i]), cases[i]


@pytest.mark.parametrize("knobs", [{"split": 5}, {"split": 5, "blk_nt": 512, "blk_tile_log": 14}])
def test_five_stage_column_passes_at_long_lengths(knobs):
    """Column passes of 5 stages at L = 2^14 and 2^15 (full and three-quarter
    lengths), the block steps after them on 9 and 10 stages; single calls and
    a batched call (which runs such products on the single-product kernels),
    equal to the oracle."""
    shapes = [(P30, 2, 3, 2, 5000), (P31, 3, 2, 2, 7000), (P30, 2, 2, 3, 9000)]
    Bd.tune_load(table(knobs, {"batch_direct_max": 0}))
    As, Bs, refs = [], [], []
    for idx, (p, m, n, k, d) in enumerate(shapes):
        info = Bd.pm_plan(p, m, n, k, d, 4)
        assert info.tune_entry == 0 and info.log2_len in (14, 15)
        say(f"[tune] split 5: {m}x{n}x{k} d={d} L=2^{info.log2_len} pts={info.num_points}")
        A, B = operands(p, m, n, k, d, np.uint32, seed=130 + idx)
        refs.append(O.polymatmul(p, A, B))
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
        C = polymat.mul(p, As[-1], Bs[-1])
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy().astype(np.uint64), refs[-1]), idx
    for p in (P30, P31):
        ids = [i for i, s in enumerate(shapes) if s[0] == p]
        outs = polymat.mul_batched(p, [As[i] for i in ids], [Bs[i] for i in ids])
        torch.cuda.synchronize()
        for i, C in zip(ids, outs):
            assert np.array_equal(C.cpu().numpy().astype(np.uint64), refs[i]), i
