"""Pins of the truncated-inverse oracle: the certificate A S = I mod x^N
(schoolbook, independent of the recurrence), the geometric series of
I - x M, scalar 1/(1 - a x), and matrix inverses mod p checked by product.
CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import series as S


@pytest.mark.parametrize("p,n,da,N,seed", [(97, 3, 4, 10, 1), (998244353, 4, 7, 20, 2),
                                           (2, 3, 3, 9, 3), ((1 << 61) - 1, 2, 5, 12, 4)])
def test_truncated_inverse_certificate(p, n, da, N, seed):
    rng = np.random.default_rng(seed)
    while True:
        A = np.array([[[int(rng.integers(0, 1 << 62)) % p for _ in range(n)] for _ in range(n)]
                      for _ in range(da)], dtype=object)
        try:
            S.matinv(A[0], p)
            break
        except ValueError:
            continue
    X = S.truncated_inverse(A, N, p)
    assert X.shape == (N, n, n)
    assert S.is_truncated_inverse(A, X, N, p)
    bad = X.copy()
    bad[N - 1, 0, 0] = (bad[N - 1, 0, 0] + 1) % p
    assert not S.is_truncated_inverse(A, bad, N, p)


def test_geometric_series():
    p, n, N = 1000003, 3, 8
    rng = np.random.default_rng(5)
    M = rng.integers(0, p, size=(n, n)).astype(object)
    A = np.zeros((2, n, n), dtype=object)
    A[0] = np.identity(n, dtype=object)
    A[1] = (-M) % p
    X = S.truncated_inverse(A, N, p)
    Mk = np.identity(n, dtype=object)
    for k in range(N):
        assert np.array_equal(X[k], Mk % p)
        Mk = Mk.dot(M) % p


def test_scalar_series():
    p, a, N = 97, 5, 12
    A = np.array([[[1]], [[p - a]]], dtype=object)      # 1 - a x
    X = S.truncated_inverse(A, N, p)
    assert [int(X[k, 0, 0]) for k in range(N)] == [pow(a, k, p) for k in range(N)]


def test_matinv():
    p = 998244353
    rng = np.random.default_rng(6)
    M = rng.integers(0, p, size=(5, 5)).astype(object)
    inv = S.matinv(M, p)
    assert np.array_equal(M.dot(inv) % p, np.identity(5, dtype=object))
    with pytest.raises(ValueError):
        S.matinv(np.zeros((2, 2), dtype=object), p)
