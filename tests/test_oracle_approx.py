"""Pins of the approximant-basis oracle (Section 3, "Approximant bases"):
certificates that do not use the algorithms (P F = 0 mod x^sigma, s-pivots on
the diagonal, pivot degrees summing to the codimension of the module computed
by linear algebra), brute-force uniqueness of M-Basis-1 over small fields,
and agreement of PM-Basis with M-Basis (the predictable-degree property makes
them the same matrix). CPU only."""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import approx as X


def certify(P, F, sigma, s, p):
    assert X.is_approximant(P, F, sigma, p)
    assert X.is_ordered_weak_popov(P, s)
    assert X.pivot_degree_sum(P) == X.module_degree(F, sigma, p)


def rand_F(p, sigma, m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, p, size=(sigma, m, n)).astype(object)


@pytest.mark.parametrize("p,m,n,seed", [(5, 3, 1, 0), (7, 4, 2, 1), (5, 3, 2, 2), (2, 4, 2, 3)])
def test_mbasis1_kernel_rows_are_unique(p, m, n, seed):
    """Each constant row of M-Basis-1 is the only vector with 1 at i, support on
    i and the earlier independent rows, in the left kernel of R (brute force)."""
    rng = np.random.default_rng(seed)
    R = rng.integers(0, p, size=(m, n)).astype(object)
    R[m - 1] = (R[0] + R[1]) % p            # force a dependency
    s = [int(x) for x in rng.integers(-2, 3, size=m)]
    Q = X.mbasis1(R, s, p)
    order = sorted(range(m), key=lambda i: (s[i], i))
    indep = [i for i in range(m) if Q[1, i, i] == 1]
    for pos, i in enumerate(order):
        if i in indep:
            assert not np.any(Q[0, i])
            continue
        allowed = [j for j in order[:pos] if j in indep]
        sols = []
        for vals in itertools.product(range(p), repeat=len(allowed)):
            v = [0] * m
            v[i] = 1
            for j, c in zip(allowed, vals):
                v[j] = c
            if not any(sum(v[r] * int(R[r, c]) for r in range(m)) % p for c in range(n)):
                sols.append(v)
        assert len(sols) == 1
        assert [int(x) for x in Q[0, i]] == sols[0]
    certify(X.trim(Q), R[None], 1, s, p)


@pytest.mark.parametrize("p,sigma,m,n,shift,seed", [
    (97, 6, 3, 1, [0, 0, 0], 1),
    (97, 8, 4, 2, [0, 0, 0, 0], 2),
    (101, 7, 4, 2, [3, -1, 0, 2], 3),
    (998244353, 9, 3, 2, [0, 5, 1], 4),
    (5, 10, 4, 1, [1, 1, 0, 0], 5),
    (2, 12, 3, 1, [0, 0, 0], 6),
])
def test_mbasis_and_pmbasis_are_certified_and_equal(p, sigma, m, n, shift, seed):
    F = rand_F(p, sigma, m, n, seed)
    Pm = X.mbasis(F, sigma, shift, p)
    certify(Pm, F, sigma, shift, p)
    for T in (1, 2, 3, sigma):
        Pp = X.pmbasis(F, sigma, shift, p, T)
        certify(Pp, F, sigma, shift, p)
        assert Pp.shape == Pm.shape and np.array_equal(Pp, Pm), T


def test_degenerate_inputs():
    p, sigma, m, n = 11, 6, 3, 2
    F = X._z((sigma, m, n))                  # F = 0: the identity is a basis
    P = X.pmbasis(F, sigma, [0, 0, 0], p, 2)
    assert P.shape[0] == 1 and np.array_equal(P[0], np.identity(m, dtype=object))
    F = rand_F(p, sigma, m, n, 9)
    F[:, :, 1] = 0                           # a zero column
    F[0] = 0                                 # F(0) = 0: rank-deficient at 0
    P = X.pmbasis(F, sigma, [2, 0, 1], p, 1)
    certify(P, F, sigma, [2, 0, 1], p)


def test_certificates_reject_wrong_bases():
    p, sigma, m, n = 97, 6, 3, 1
    F = rand_F(p, sigma, m, n, 11)
    s = [0, 0, 0]
    P = X.pmbasis(F, sigma, s, p, 1)
    bad = P.copy()
    bad[0, 0, 0] = (bad[0, 0, 0] + 1) % p      # a perturbed coefficient
    assert not X.is_approximant(bad, F, sigma, p)
    x2 = X._z((P.shape[0] + 1,) + P.shape[1:])  # x times row 0: still in the module,
    x2[1:] = P                                  # but no longer generates it
    x2[1:, 1:] = 0
    x2[:-1, 1:] = P[:, 1:]
    assert X.is_approximant(x2, F, sigma, p)
    assert X.pivot_degree_sum(x2) != X.module_degree(F, sigma, p)
