"""Approximant bases over F_p, plain and slow (test infrastructure only).

Section 3 of Hyun, Neiger, Schost (ISSAC 2019), "Approximant bases": for F in
K[x]^{m x n} and an order sigma, an approximant basis is a nonsingular
m x m polynomial matrix whose rows generate the module of all row vectors p
with p F = 0 mod x^sigma; the algorithms return it in s-ordered weak Popov
form (the s-pivot of row i, the rightmost entry reaching the row's s-degree,
is on the diagonal).  Here, on Python integers, in the paper's order:

* `mbasis1(R, s, p)`: the s-Popov approximant basis of a constant matrix R at
  order 1 (the signature of M-Basis-1): rows taken by increasing shift (ties
  by index) are either combinations of earlier independent rows (a constant
  row with 1 on the diagonal) or independent (the row x e_i).
* `mbasis(F, sigma, s, p)`: Algorithm M-Basis: sigma rounds of residual
  (coefficient k of P F), M-Basis-1 on it, P := Q P, s' := rdeg_s(P).
* `pmbasis(F, sigma, s, p, T)`: Algorithm PM-Basis with threshold T: two
  half-order calls joined by the middle product of the first basis and F.
* Certificates, independent of the algorithms: `is_approximant` (P F = 0 mod
  x^sigma), `is_ordered_weak_popov`, and `module_degree` (the rank of the
  linear map p -> p F mod x^sigma on vectors of degree < sigma, which is the
  degree of the determinant of any basis of the module); for a basis in
  weak Popov form that degree is the sum of its pivot degrees.

Polynomial matrices are numpy object arrays of shape (coefficients, rows,
cols), coefficient c at index c, trailing zero coefficients trimmed.
"""
from __future__ import annotations

import numpy as np

NEG = -(1 << 60)  # degree of the zero polynomial in shift arithmetic


def _z(shape) -> np.ndarray:
    return np.zeros(shape, dtype=object)


def trim(P: np.ndarray) -> np.ndarray:
    """Drop trailing zero coefficient matrices (keep at least one)."""
    D = P.shape[0]
    while D > 1 and not np.any(P[D - 1]):
        D -= 1
    return P[:D]


def as_obj(X) -> np.ndarray:
    return np.asarray(X).astype(object)


def polymul(p: int, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A B mod p, schoolbook over coefficient matrices."""
    da, db = A.shape[0], B.shape[0]
    C = _z((da + db - 1, A.shape[1], B.shape[2]))
    for a in range(da):
        if not np.any(A[a]):
            continue
        for b in range(db):
            C[a + b] = (C[a + b] + A[a].dot(B[b])) % p
    return C


def entry_degree(P: np.ndarray, i: int, j: int) -> int:
    for c in range(P.shape[0] - 1, -1, -1):
        if P[c, i, j] != 0:
            return c
    return NEG


def rdeg(P: np.ndarray, s) -> list[int]:
    """s-row degrees: max_j deg(P_ij) + s_j."""
    m, k = P.shape[1], P.shape[2]
    return [max(entry_degree(P, i, j) + s[j] for j in range(k)) for i in range(m)]


def s_pivot(P: np.ndarray, s, i: int) -> int:
    """Index of the rightmost entry of row i reaching its s-degree."""
    best, at = NEG, -1
    for j in range(P.shape[2]):
        v = entry_degree(P, i, j) + s[j]
        if v >= best and entry_degree(P, i, j) != NEG:
            best, at = v, j
    return at


def mbasis1(R: np.ndarray, s, p: int) -> np.ndarray:
    """M-Basis-1: the s-Popov approximant basis of the constant m x n matrix R
    at order 1, as a (2, m, m) polynomial matrix."""
    m, n = R.shape
    order = sorted(range(m), key=lambda i: (s[i], i))
    pivots = []          # (pivot column, reduced row, combination of rows)
    Q = _z((2, m, m))
    for i in order:
        v = [int(x) % p for x in R[i]]
        comb = [0] * m
        comb[i] = 1
        for col, w, cw in pivots:
            if v[col]:
                f = v[col] * pow(w[col], p - 2, p) % p
                v = [(a - f * b) % p for a, b in zip(v, w)]
                comb = [(a - f * b) % p for a, b in zip(comb, cw)]
        if any(v):
            col = next(c for c in range(n) if v[c])
            pivots.append((col, v, comb))
            Q[1, i, i] = 1
        else:
            for j in range(m):
                Q[0, i, j] = comb[j]
    return Q


def mbasis(F: np.ndarray, sigma: int, s, p: int) -> np.ndarray:
    """Algorithm M-Basis on F (at least sigma coefficients used)."""
    F = as_obj(F)
    m = F.shape[1]
    P = _z((1, m, m))
    P[0] = np.identity(m, dtype=object)
    sc = list(s)
    for k in range(sigma):
        PF = polymul(p, P, F[:k + 1])
        R = PF[k] if PF.shape[0] > k else _z(PF.shape[1:])
        Q = mbasis1(R, sc, p)
        P = trim(polymul(p, Q, P))
        sc = rdeg(P, s)
    return P


def pmbasis(F: np.ndarray, sigma: int, s, p: int, T: int = 1) -> np.ndarray:
    """Algorithm PM-Basis with threshold T (M-Basis at orders <= T)."""
    F = as_obj(F)
    if sigma <= T:
        return mbasis(F, sigma, s, p)
    c = (sigma + 1) // 2
    d = sigma - c
    P1 = pmbasis(F[:c], c, s, p, T)
    PF = polymul(p, P1, F[:sigma])                 # MiddleProduct: the whole product,
    R = _z((d,) + PF.shape[1:])                    # then coefficients c .. sigma-1
    top = min(PF.shape[0], sigma)
    if top > c:
        R[:top - c] = PF[c:top]
    s2 = rdeg(P1, s)
    P2 = pmbasis(R, d, s2, p, T)
    return trim(polymul(p, P2, P1))


# ---- certificates ----------------------------------------------------------

def is_approximant(P: np.ndarray, F: np.ndarray, sigma: int, p: int) -> bool:
    PF = polymul(p, as_obj(P), as_obj(F)[:sigma])
    return not np.any(PF[:sigma] % p)


def is_ordered_weak_popov(P: np.ndarray, s) -> bool:
    m = P.shape[1]
    return all(s_pivot(P, s, i) == i for i in range(m))


def pivot_degree_sum(P: np.ndarray) -> int:
    return sum(entry_degree(P, i, i) for i in range(P.shape[1]))


def _rank_mod(M: list[list[int]], p: int) -> int:
    M = [row[:] for row in M]
    rank, cols = 0, len(M[0]) if M else 0
    for col in range(cols):
        piv = next((r for r in range(rank, len(M)) if M[r][col] % p), None)
        if piv is None:
            continue
        M[rank], M[piv] = M[piv], M[rank]
        inv = pow(M[rank][col], p - 2, p)
        M[rank] = [x * inv % p for x in M[rank]]
        for r in range(len(M)):
            if r != rank and M[r][col] % p:
                f = M[r][col]
                M[r] = [(a - f * b) % p for a, b in zip(M[r], M[rank])]
        rank += 1
    return rank


def module_degree(F: np.ndarray, sigma: int, p: int) -> int:
    """Rank over F_p of p -> p F mod x^sigma on row vectors of degree < sigma
    (the codimension of the approximant module, i.e. deg det of its bases)."""
    F = as_obj(F)
    m, n = F.shape[1], F.shape[2]
    rows = []
    for a in range(sigma):          # p = x^a e_i
        for i in range(m):
            r = [0] * (n * sigma)
            for c in range(a, sigma):
                if c - a < F.shape[0]:
                    for j in range(n):
                        r[c * n + j] = int(F[c - a, i, j]) % p
            rows.append(r)
    return _rank_mod(rows, p)
