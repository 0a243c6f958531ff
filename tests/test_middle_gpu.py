"""GPU parity of the middle product / coefficient window (pm_middle_*)
against the oracle's whole-product-then-slice, bit-exact.

Cases cover the paper's MiddleProduct shape (F in K[x]_c, G in K[x]_{c+d}),
the residual shape of Algorithm PM-Basis (a basis of degree <= c times the
series truncated at order c + d), prefixes (truncated products), single
coefficients, the top coefficient, inputs longer than half the transform
length in both the unsplit (L < 2^11) and split (L >= 2^11) transforms, CRT
moduli in 32 and 64 bits, full-size sampled entries, and windows under
5-stage first passes.
"""
from __future__ import annotations

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
P32 = 4294967291


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def operands(p, m, n, k, da, db, seed, dtype=np.uint32):
    A = I.polymat(seed, 0, I.TENSOR_A, p, da, m, n, dtype)
    B = I.polymat(seed, 0, I.TENSOR_B, p, db, n, k, dtype)
    return A, B


def gpu_middle(p, A, B, lo, length):
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    tC = polymat.middle(p, tA, tB, lo, length)
    torch.cuda.synchronize()
    return tC.cpu().numpy()


def check(p, m, n, k, da, db, lo, length, seed=0, dtype=np.uint32):
    say(f"[middle] p={p} m={m} n={n} k={k} da={da} db={db} lo={lo} len={length} "
        f"dtype={np.dtype(dtype).name}")
    A, B = operands(p, m, n, k, da, db, seed, dtype)
    C = gpu_middle(p, A, B, lo, length)
    ref = O.middle_product(p, A, B, lo, length)
    assert C.shape == ref.shape and C.dtype == dtype
    bad = np.argwhere(C.astype(np.uint64) != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"


def shapes_for(c, d, m, n, k):
    # (m, n, k, da, db, lo, len) cases around one (c, d)
    return [
        (m, n, k, c, c + d, c, d),          # MiddleProduct(F, G, c, d)
        (m, n, k, c + 1, c + d, c, d),      # PM-Basis residual (basis degree <= c)
        (m, n, k, c, c + d, 0, d),          # prefix: (F G) mod x^d
        (m, n, k, c, c + d, 2 * c + d - 2, 1),  # top coefficient
        (m, n, k, c, c + d, c + d // 2, 1),     # one coefficient
    ]


SMALL = []
for (c, d) in [(1, 1), (3, 2), (4, 5), (16, 16), (33, 31), (100, 60), (256, 256)]:
    SMALL += shapes_for(c, d, 3, 4, 2)


@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("p", [P30, P31])
def test_middle_small_direct(p, case):
    check(p, *case, seed=1)


@pytest.mark.parametrize("case", [
    (2, 3, 2, 1024, 2048, 1024, 1024),   # L = 2^11: split, input longer than L/2
    (2, 3, 2, 1025, 2048, 1024, 1024),
    (1, 2, 3, 2048, 4096, 2048, 2048),   # L = 2^12
    (4, 4, 4, 700, 3000, 650, 2300),     # ragged window, L = 2^12
    (1, 1, 1, 4096, 4096, 4095, 4096),   # upper half of a whole product
    (3, 5, 2, 1, 3000, 0, 3000),         # constant left factor
    (2, 2, 2, 4097, 8192, 4096, 4096),   # PM-Basis residual at order 8192, L = 2^13
])
def test_middle_split_transforms(case):
    check(P30, *case, seed=2)


@pytest.mark.parametrize("p,dtype", [(P32, np.uint32), (97, np.uint32),
                                     ((1 << 61) - 1, np.uint64),
                                     (1152921504606847009, np.uint64)])
@pytest.mark.parametrize("case", [(3, 4, 2, 5, 9, 5, 4), (2, 3, 2, 33, 64, 33, 31),
                                  (2, 2, 3, 1025, 2048, 1024, 1024)])
def test_middle_crt(p, dtype, case):
    check(p, *case, seed=3, dtype=dtype)


def test_middle_equals_window_of_product():
    # da = db = d: the window of the whole product computed by pm_mul
    p, m, n, k, d = P31, 8, 8, 4, 777
    A, B = operands(p, m, n, k, d, d, seed=4)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    full = polymat.mul(p, tA, tB)
    for lo, length in [(0, 2 * d - 1), (d - 1, d), (100, 900), (2 * d - 2, 1)]:
        win = polymat.middle(p, tA, tB, lo, length)
        torch.cuda.synchronize()
        assert torch.equal(win, full[lo:lo + length]), (lo, length)


def test_middle_rejects_bad_windows():
    t = torch.zeros((4, 2, 2), dtype=torch.uint32, device="cuda")
    for lo, length in [(-1, 2), (0, 0), (7, 1), (5, 3)]:
        with pytest.raises(Bd.PmError) as e:
            polymat.middle(P30, t, t, lo, length)
        assert e.value.status == Bd.PM_EINVAL


def test_middle_pm_basis_size_sampled():
    """32x32 basis (degree <= 2048) times a 32x16 series of order 4096:
    the residual of PM-Basis at order 4096; 16 whole entries vs the oracle."""
    p, m, n, k, c, d = P30, 32, 32, 16, 2048, 2048
    A, B = operands(p, m, n, k, c + 1, c + d, seed=5)
    say("[middle] pm-basis size")
    C = gpu_middle(p, A, B, c, d)
    pairs = I.sample_pairs(5, m, k, 16)
    rows = O.middle_entries(p, A, B, c, d, pairs)
    for s, (i, j) in enumerate(pairs):
        assert np.array_equal(C[:, i, j].astype(np.uint64), rows[s]), (i, j)


@pytest.mark.parametrize("case", [
    (2, 3, 2, 1024, 2048, 1024, 1024),   # L = 2^11, input longer than L/2
    (2, 2, 2, 4097, 8192, 4096, 4096),   # L = 2^13
    (1, 2, 2, 6000, 9000, 5000, 4000),   # L = 2^14, ragged window
])
@pytest.mark.parametrize("p,dtype", [(P30, np.uint32), ((1 << 61) - 1, np.uint64)])
def test_middle_under_five_stage_first_passes(p, dtype, case):
    """Coefficient windows with a 5-stage first pass (tuning knob split 5):
    inputs longer than half the transform take the one-entry full-load
    column pass; direct and CRT moduli."""
    import json
    Bd.tune_load(json.dumps({"format": "pm-tune-1", "entries": [{"knobs": {"split": 5}}]}))
    try:
        check(p, *case, seed=4, dtype=dtype)
    finally:
        torch.cuda.synchronize()
        Bd.tune_load(None)
