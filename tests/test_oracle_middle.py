"""Pins of the oracle's middle product (coefficients lo .. lo+len-1 of A B),
independent of the whole-product-then-slice code it uses: brute-force
convolution over Python integers, the product by x^s times the identity, and
the paper's MiddleProduct(F, G, c, d) written as the sums it denotes (Section
2, "Polynomial multiplication"). CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O


def brute_window(p, A, B, lo, length):
    da, m, n = A.shape
    db, _, k = B.shape
    out = np.zeros((length, m, k), dtype=np.uint64)
    for t in range(lo, lo + length):
        for i in range(m):
            for j in range(k):
                acc = 0
                for a in range(da):
                    b = t - a
                    if 0 <= b < db:
                        for l in range(n):
                            acc += int(A[a, i, l]) * int(B[b, l, j])
                out[t - lo, i, j] = acc % p
    return out


@pytest.mark.parametrize("p,shape,lo,length", [
    (97, (3, 2, 2, 5, 1), 0, 7),          # whole product
    (97, (3, 2, 2, 5, 1), 3, 4),          # the paper's c = 3, d = 2 case, shifted
    (998244353, (4, 3, 2, 9, 2), 4, 5),   # MiddleProduct(F, G, 4, 5)
    (998244353, (5, 1, 3, 4, 2), 2, 1),   # a single coefficient
    (2, (6, 2, 2, 6, 2), 10, 1),          # the top coefficient, p = 2
    ((1 << 61) - 1, (3, 2, 3, 7, 2), 2, 6),
])
def test_middle_matches_brute_force(p, shape, lo, length):
    da, m, n, db, k = shape
    rng = np.random.default_rng(da * 1000 + db * 10 + lo)
    A = rng.integers(0, p, size=(da, m, n), dtype=np.uint64)
    B = rng.integers(0, p, size=(db, n, k), dtype=np.uint64)
    got = O.middle_product(p, A, B, lo, length, threads=2)
    assert np.array_equal(got, brute_window(p, A, B, lo, length))


def test_middle_of_shift_is_a_window_of_the_other_factor():
    p, m, k, s = 1000003, 3, 2, 4
    db = 9
    A = np.zeros((s + 1, m, m), dtype=np.uint64)
    A[s] = np.eye(m, dtype=np.uint64)            # x^s I
    rng = np.random.default_rng(7)
    B = rng.integers(0, p, size=(db, m, k), dtype=np.uint64)
    for lo, length in [(0, s + db), (s, db), (s + 2, 3), (1, 5)]:
        got = O.middle_product(p, A, B, lo, length, threads=2)
        want = np.zeros((length, m, k), dtype=np.uint64)
        for c in range(length):
            b = lo + c - s
            if 0 <= b < db:
                want[c] = B[b]
        assert np.array_equal(got, want), (lo, length)


def test_paper_middle_product_sums():
    # F in K[x]_c, G in K[x]_{c+d}: coefficient c+i of F G is
    # sum_{j<c} F_j G_{c+i-j}, every index in range.
    p, c, d, m, n, k = 65537, 5, 4, 2, 3, 2
    rng = np.random.default_rng(11)
    F = rng.integers(0, p, size=(c, m, n), dtype=np.uint64)
    G = rng.integers(0, p, size=(c + d, n, k), dtype=np.uint64)
    got = O.middle_product(p, F, G, c, d, threads=1)
    for i in range(d):
        want = np.zeros((m, k), dtype=object)
        for j in range(c):
            want = want + F[j].astype(object).dot(G[c + i - j].astype(object))
        assert np.array_equal(got[i].astype(object), want % p)


def test_middle_entries_match_full_window():
    p = 998244353
    rng = np.random.default_rng(3)
    A = rng.integers(0, p, size=(6, 3, 4), dtype=np.uint64)
    B = rng.integers(0, p, size=(11, 4, 2), dtype=np.uint64)
    full = O.middle_product(p, A, B, 5, 11, threads=2)
    pairs = [(0, 1), (2, 0), (1, 1)]
    rows = O.middle_entries(p, A, B, 5, 11, pairs, threads=2)
    for s, (i, j) in enumerate(pairs):
        assert np.array_equal(rows[s], full[:, i, j])


def test_middle_rejects_windows_outside_the_product():
    A = np.zeros((3, 1, 1), dtype=np.uint64)
    B = np.zeros((4, 1, 1), dtype=np.uint64)
    for lo, length in [(-1, 2), (0, 0), (5, 2), (6, 1)]:
        with pytest.raises(ValueError):
            O.middle_product(97, A, B, lo, length)
