"""Truncated inverses of polynomial matrices over F_p, plain and slow (test
infrastructure only).

For A in K[x]^{n x n} with A(0) invertible, the truncated inverse
S = A^{-1} mod x^N (used before Dixon's lifting, Section 4 of Hyun, Neiger,
Schost, ISSAC 2019, "Lifting techniques") is the unique S of degree < N with
A S = I mod x^N.  Comparing coefficients of A S = I gives its definition as
a recurrence: S_0 = A_0^{-1}, and for k >= 1
    S_k = -A_0^{-1} (A_1 S_{k-1} + A_2 S_{k-2} + ... + A_k S_0).
Everything is on Python integers; matrices are numpy object arrays,
polynomial matrices have shape (coefficients, n, n).
"""
from __future__ import annotations

import numpy as np


def matinv(M, p: int) -> np.ndarray:
    """Inverse of a square matrix mod p by Gauss-Jordan elimination; raises
    ValueError if it is singular."""
    n = len(M)
    a = [[int(M[i][j]) % p for j in range(n)] + [1 if i == j else 0 for j in range(n)]
         for i in range(n)]
    for col in range(n):
        piv = next((r for r in range(col, n) if a[r][col]), None)
        if piv is None:
            raise ValueError("singular matrix")
        a[col], a[piv] = a[piv], a[col]
        inv = pow(a[col][col], p - 2, p)
        a[col] = [x * inv % p for x in a[col]]
        for r in range(n):
            if r != col and a[r][col]:
                f = a[r][col]
                a[r] = [(x - f * y) % p for x, y in zip(a[r], a[col])]
    return np.array([row[n:] for row in a], dtype=object)


def truncated_inverse(A, N: int, p: int) -> np.ndarray:
    """S = A^{-1} mod x^N by the coefficient recurrence, shape (N, n, n)."""
    A = np.asarray(A).astype(object)
    n = A.shape[1]
    inv0 = matinv(A[0], p)
    S = np.zeros((N, n, n), dtype=object)
    S[0] = inv0
    for k in range(1, N):
        acc = np.zeros((n, n), dtype=object)
        for j in range(1, min(k, A.shape[0] - 1) + 1):
            acc = acc + A[j].dot(S[k - j])
        S[k] = (-inv0.dot(acc % p)) % p
    return S


def is_truncated_inverse(A, S, N: int, p: int) -> bool:
    """A S = I mod x^N, by the schoolbook product of the first N coefficients."""
    A = np.asarray(A).astype(object)
    S = np.asarray(S).astype(object)
    n = A.shape[1]
    for c in range(N):
        acc = np.zeros((n, n), dtype=object)
        for a in range(min(c, A.shape[0] - 1) + 1):
            if c - a < S.shape[0]:
                acc = acc + A[a].dot(S[c - a])
        want = np.identity(n, dtype=object) if c == 0 else np.zeros((n, n), dtype=object)
        if np.any((acc - want) % p):
            return False
    return True
