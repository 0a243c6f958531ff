"""Pins for the CPU oracle, each independent of the oracle's own code.

The oracle computes the product of polynomial matrices over F_p from its
definition (Section 2, "Polynomial matrix multiplication"; entries in K[x]_d,
Section 2, "Polynomial multiplication"). These tests tie it to things other
than itself:

* hand-worked examples (tests/golden/hand_examples.json);
* d = 1, where the product is a plain matrix product over F_p (numpy object
  arithmetic on Python integers);
* Kronecker substitution with Python big integers, an independent route to
  the same polynomial product;
* closed forms (identity, shift by x^s, zeros, all-ones, all-(p-1));
* first and last coefficients (C_0 = A_0 B_0, C_{2d-2} = A_{d-1} B_{d-1});
* the evaluation homomorphism, computed with Python-int Horner;
* exhaustive brute force on tiny inputs against sympy's polynomial product;
* Miller-Rabin against sympy.isprime and known pseudoprimes.

A final test builds oracle mutants with planted mistakes and checks that these
pins reject every one of them.
"""
from __future__ import annotations

import itertools
import json
import os
import tempfile

import numpy as np
import pytest

from oracle import oracle as O
from oracle import build as OB

HERE = os.path.dirname(os.path.abspath(__file__))
P30 = 998244353
P31 = 2013265921
P62 = (1 << 62) - 57  # largest prime below 2^62
P61 = (1 << 61) - 1   # Mersenne prime


def rand_pm(rng, p, d, r, c):
    return rng.integers(0, p, size=(d, r, c), dtype=np.uint64)


# ---- independent references (no oracle code) ------------------------------

def ref_matmul_obj(p, X, Y):
    """Matrix product mod p on Python ints (numpy object arrays)."""
    Z = np.asarray(X, dtype=object).dot(np.asarray(Y, dtype=object))
    return np.vectorize(lambda v: int(v) % p, otypes=[object])(Z)


def kronecker_entry(p, A, B, i, j):
    """C_ij by Kronecker substitution: pack each polynomial into one big
    integer in base 2^b, multiply integers, unpack, reduce mod p."""
    d, m, n = A.shape
    bound = n * d * (p - 1) ** 2 + 1
    b = bound.bit_length() + 1

    def pack(coeffs):
        v = 0
        for c in reversed([int(x) for x in coeffs]):
            v = (v << b) | c
        return v

    total = 0
    for l in range(n):
        total += pack(A[:, i, l]) * pack(B[:, l, j])
    mask = (1 << b) - 1
    out = []
    for _ in range(2 * d - 1):
        out.append((total & mask) % p)
        total >>= b
    return out


def horner_py(p, coeffs, r):
    v = 0
    for c in reversed([int(x) for x in coeffs]):
        v = (v * r + c) % p
    return v


# ---- pins ------------------------------------------------------------------

def check_golden(L=None):
    data = json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))
    for case in data["cases"]:
        C = O.polymatmul(case["p"], case["A"], case["B"], L=L)
        if C.tolist() != case["C"]:
            return False
    return True


def test_golden_hand_examples():
    assert check_golden()


def check_d1(L=None):
    rng = np.random.default_rng(1)
    for p, (m, n, k) in [(7, (3, 4, 5)), (P31, (5, 3, 2)), (P62, (4, 4, 4))]:
        A = rand_pm(rng, p, 1, m, n)
        B = rand_pm(rng, p, 1, n, k)
        C = O.polymatmul(p, A, B, L=L)
        ref = ref_matmul_obj(p, [[int(x) for x in r] for r in A[0]],
                             [[int(x) for x in r] for r in B[0]])
        if C.shape != (1, m, k) or [[int(x) for x in r] for r in C[0]] != ref.tolist():
            return False
    return True


def test_d1_is_matrix_product():
    assert check_d1()


def check_kronecker(L=None, cases=None):
    rng = np.random.default_rng(2)
    cases = cases or [(97, 2, 3, 2, 5), (P30, 3, 2, 4, 17), (P31, 2, 5, 3, 33),
                      (P62, 2, 3, 2, 40), (P61, 1, 2, 1, 64), (2, 3, 3, 3, 9),
                      (1 << 40, 2, 2, 2, 7)]  # composite modulus too
    for p, m, n, k, d in cases:
        A = rand_pm(rng, p, d, m, n)
        B = rand_pm(rng, p, d, n, k)
        C = O.polymatmul(p, A, B, L=L)
        for i in range(m):
            for j in range(k):
                if [int(x) for x in C[:, i, j]] != kronecker_entry(p, A, B, i, j):
                    return False
    return True


def test_kronecker_substitution():
    assert check_kronecker()


def check_closed_forms(L=None):
    rng = np.random.default_rng(3)
    for p, n, d in [(P30, 3, 7), (P31, 4, 16), (P62, 8, 64), (5, 2, 3)]:
        m = k = n
        B = rand_pm(rng, p, d, n, k)
        # A = I (constant): C = B followed by d-1 zero coefficients
        A = np.zeros((d, m, n), dtype=np.uint64)
        A[0] = np.eye(n, dtype=np.uint64)
        C = O.polymatmul(p, A, B, L=L)
        if not (np.array_equal(C[:d], B) and not C[d:].any()):
            return False
        # A = x^s I: C = x^s B
        s = d // 2
        A = np.zeros((d, m, n), dtype=np.uint64)
        A[s] = np.eye(n, dtype=np.uint64)
        C = O.polymatmul(p, A, B, L=L)
        if not (not C[:s].any() and np.array_equal(C[s:s + d], B)
                and not C[s + d:].any()):
            return False
        # zeros
        if O.polymatmul(p, np.zeros((d, m, n), np.uint64), B, L=L).any():
            return False
        # all (p-1): (p-1)^2 = 1, coefficient c collects n*min(c+1, 2d-1-c) terms
        A = np.full((d, m, n), p - 1, dtype=np.uint64)
        Bf = np.full((d, n, k), p - 1, dtype=np.uint64)
        C = O.polymatmul(p, A, Bf, L=L)
        want = [n * min(c + 1, 2 * d - 1 - c) % p for c in range(2 * d - 1)]
        if [int(C[c, i, j]) for c in range(2 * d - 1)
                for i in range(m) for j in range(k)] != \
                [w for w in want for _ in range(m * k)]:
            return False
        # all ones
        C = O.polymatmul(p, np.ones((d, m, n), np.uint64),
                         np.ones((d, n, k), np.uint64), L=L)
        if not all(int(C[c, 0, 0]) == n * min(c + 1, 2 * d - 1 - c) % p
                   for c in range(2 * d - 1)):
            return False
    return True


def test_closed_forms():
    assert check_closed_forms()


def check_end_coefficients_and_points(L=None):
    rng = np.random.default_rng(4)
    for p, m, n, k, d in [(P30, 3, 4, 2, 10), (P62, 2, 3, 3, 20), (P31, 4, 4, 4, 31)]:
        A = rand_pm(rng, p, d, m, n)
        B = rand_pm(rng, p, d, n, k)
        C = O.polymatmul(p, A, B, L=L)
        lo = ref_matmul_obj(p, A[0].tolist(), B[0].tolist())
        hi = ref_matmul_obj(p, A[d - 1].tolist(), B[d - 1].tolist())
        if C[0].tolist() != lo.tolist() or C[2 * d - 2].tolist() != hi.tolist():
            return False
        for r in (0, 1, p - 1, 123456789 % p):
            Ar = [[horner_py(p, A[:, i, l], r) for l in range(n)] for i in range(m)]
            Br = [[horner_py(p, B[:, l, j], r) for j in range(k)] for l in range(n)]
            Cr = [[horner_py(p, C[:, i, j], r) for j in range(k)] for i in range(m)]
            if ref_matmul_obj(p, Ar, Br).tolist() != Cr:
                return False
    return True


def test_end_coefficients_and_evaluation_homomorphism():
    assert check_end_coefficients_and_points()


def test_bilinearity():
    rng = np.random.default_rng(5)
    p, m, n, k, d = P31, 3, 4, 2, 12
    A1, A2 = rand_pm(rng, p, d, m, n), rand_pm(rng, p, d, m, n)
    B = rand_pm(rng, p, d, n, k)
    lhs = O.polymatmul(p, (A1 + A2) % np.uint64(p), B)
    rhs = (O.polymatmul(p, A1, B) + O.polymatmul(p, A2, B)) % np.uint64(p)
    assert np.array_equal(lhs, rhs)


def check_bruteforce_tiny(L=None):
    sympy = pytest.importorskip("sympy")
    x = sympy.Symbol("x")
    # all pairs for p = 3, 1x1, d = 2 (81 cases) and p = 2, d = 3 (64 cases)
    for p, d in [(3, 2), (2, 3)]:
        for a in itertools.product(range(p), repeat=d):
            for b in itertools.product(range(p), repeat=d):
                A = np.array(a, dtype=np.uint64).reshape(d, 1, 1)
                B = np.array(b, dtype=np.uint64).reshape(d, 1, 1)
                C = O.polymatmul(p, A, B, L=L)[:, 0, 0]
                pa = sympy.Poly(list(reversed(a)), x, modulus=p)
                pb = sympy.Poly(list(reversed(b)), x, modulus=p)
                prod = (pa * pb).all_coeffs()[::-1]
                want = [int(c) % p for c in prod] + [0] * (2 * d - 1 - len(prod))
                if [int(c) for c in C] != want[:2 * d - 1]:
                    return False
    # all 2x2 . 2x2 constant matrices over F_2 (256 cases) vs sympy matrices
    for bits in range(256):
        a = [(bits >> t) & 1 for t in range(4)]
        b = [(bits >> (t + 4)) & 1 for t in range(4)]
        A = np.array(a, dtype=np.uint64).reshape(1, 2, 2)
        B = np.array(b, dtype=np.uint64).reshape(1, 2, 2)
        want = (sympy.Matrix(2, 2, a) * sympy.Matrix(2, 2, b)).applyfunc(lambda v: v % 2)
        if O.polymatmul(2, A, B, L=L)[0].tolist() != [[int(want[i, j]) for j in range(2)]
                                                      for i in range(2)]:
            return False
    return True


def test_bruteforce_tiny_vs_sympy():
    assert check_bruteforce_tiny()


def test_entries_match_full_product():
    rng = np.random.default_rng(6)
    p, m, n, k, d = P31, 5, 3, 4, 9
    A, B = rand_pm(rng, p, d, m, n), rand_pm(rng, p, d, n, k)
    C = O.polymatmul(p, A, B)
    pairs = [(0, 0), (4, 3), (2, 1), (4, 0)]
    E = O.polymatmul_entries(p, A, B, pairs)
    for s, (i, j) in enumerate(pairs):
        assert np.array_equal(E[s], C[:, i, j])


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        O.polymatmul(1, np.zeros((1, 1, 1)), np.zeros((1, 1, 1)))
    with pytest.raises(ValueError):
        O.polymatmul(7, np.zeros((2, 1, 2)), np.zeros((2, 3, 1)))


# ---- checkers --------------------------------------------------------------

def test_checkers_accept_true_product_and_catch_one_wrong_coefficient():
    rng = np.random.default_rng(7)
    for p, m, n, k, d in [(P31, 4, 3, 5, 16), (P62, 3, 2, 2, 8)]:
        A, B = rand_pm(rng, p, d, m, n), rand_pm(rng, p, d, n, k)
        C = O.polymatmul(p, A, B)
        assert O.point_check(p, A, B, C)
        assert O.freivalds_check(p, A, B, C)
        for (c, i, j) in [(0, 0, 0), (2 * d - 2, m - 1, k - 1), (d, 1, k - 1)]:
            bad = C.copy()
            bad[c, i, j] = (int(bad[c, i, j]) + 1) % p
            assert not O.point_check(p, A, B, bad)
            assert not O.freivalds_check(p, A, B, bad)


def test_checker_pieces_against_python_integers():
    """The threaded checker pieces against plain Python-integer sums on small
    inputs: Horner values at several points (both the 64-bit path, p < 2^32,
    and the 128-bit one), the two Freivalds projections, and the sum of
    univariate products, with several threads splitting the work."""
    rng = np.random.default_rng(8)
    for p in (P31, 4294967291, P62):
        D, R, S = 7, 5, 3
        X = rand_pm(rng, p, D, R, S)
        pts = [0, 1, p - 1, 12345 % p]
        got = O.eval_points(p, X, pts, threads=3)
        for t, r in enumerate(pts):
            for i in range(R):
                for j in range(S):
                    want = sum(int(X[c, i, j]) * pow(r, c, p) for c in range(D)) % p
                    assert int(got[t, i, j]) == want
        u = rng.integers(0, p, size=R, dtype=np.uint64)
        v = rng.integers(0, p, size=S, dtype=np.uint64)
        L = O.lib()
        uX = np.zeros((D, S), dtype=np.uint64)
        Xv = np.zeros((D, R), dtype=np.uint64)
        L.orc_project_left_mt(p, R, S, D, O._ptr(X), O._ptr(u), O._ptr(uX), 2)
        L.orc_project_right_mt(p, R, S, D, O._ptr(X), O._ptr(v), O._ptr(Xv), 2)
        for c in range(D):
            for j in range(S):
                assert int(uX[c, j]) == sum(int(u[i]) * int(X[c, i, j]) for i in range(R)) % p
            for i in range(R):
                assert int(Xv[c, i]) == sum(int(X[c, i, j]) * int(v[j]) for j in range(S)) % p
        n, d = 4, 9
        U = rng.integers(0, p, size=(n, d), dtype=np.uint64)
        V = rng.integers(0, p, size=(n, d), dtype=np.uint64)
        out = np.zeros(2 * d - 1, dtype=np.uint64)
        L.orc_polymul_sum(p, n, d, O._ptr(U), O._ptr(V), O._ptr(out), 3)
        for c in range(2 * d - 1):
            want = sum(int(U[l, a]) * int(V[l, c - a]) for l in range(n)
                       for a in range(max(0, c - d + 1), min(c, d - 1) + 1)) % p
            assert int(out[c]) == want


# ---- number theory ---------------------------------------------------------

def test_miller_rabin_against_sympy_and_pseudoprimes():
    sympy = pytest.importorskip("sympy")
    known_primes = [2, 3, 998244353, 2013265921, 2113929217, 1811939329,
                    1711276033, 469762049, 167772161, 754974721, P61, P62,
                    18446744073709551557]  # largest 64-bit prime
    for q in known_primes:
        assert O.is_prime(q), q
    # Carmichael numbers and strong pseudoprimes to small bases
    composites = [1, 4, 561, 1105, 41041, 2047, 1373653, 25326001, 3215031751,
                  2152302898747, 3474749660383, 341550071728321,
                  3825123056546413051, P30 * 3, (1 << 61) + 1]
    for c in composites:
        assert not O.is_prime(c), c
    rng = np.random.default_rng(8)
    for x in rng.integers(1 << 20, 1 << 62, size=300, dtype=np.uint64):
        assert O.is_prime(int(x)) == sympy.isprime(int(x))
    assert O.powmod(3, 998244352, 998244353) == 1
    assert O.powmod(3, 998244352 // 2, 998244353) == 998244352


# ---- mutants with planted mistakes ------------------------------------------

PIN_SUITE = [check_golden, check_d1, check_kronecker, check_closed_forms,
             check_end_coefficients_and_points, check_bruteforce_tiny]


@pytest.mark.parametrize("plant", [1, 2, 3, 4, 5])
def test_pins_reject_planted_mistakes(plant):
    """Each mutant (dropped term, transposed B, off-by-one index, missing
    overflow reduction, wrong modulus) must fail at least one pin."""
    with tempfile.TemporaryDirectory() as tmp:
        path = OB.build(os.path.join(tmp, f"liborc_plant{plant}.so"), plant=plant)
        L = O.lib(path)
        failed = []
        for pin in PIN_SUITE:
            try:
                ok = pin(L=L)
            except Exception:
                ok = False
            if not ok:
                failed.append(pin.__name__)
        assert failed, f"planted mistake {plant} passed every pin"
