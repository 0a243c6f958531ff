"""Python face of the CPU oracle (test infrastructure only).

Every function here either calls the plain C schoolbook in pm_oracle.c or is a
checker built from the definitions in Section 2 of Hyun, Neiger, Schost
(ISSAC 2019), "Polynomial matrix multiplication":

* `polymatmul`       -- the full product C = A B over F_p, coefficient-major.
* `polymatmul_entries` -- selected whole output entries C_ij (all 2d-1
                        coefficients), for sizes where the full product is slow.
* `middle_product`, `middle_entries` -- coefficients lo .. lo+len-1 of A B
                        for operands of different lengths: the whole product,
                        then the slice (Section 2, "Polynomial
                        multiplication": the direct approach to the middle
                        product).
* `point_check`      -- C(r) == A(r) B(r) at seeded points r of F_p: the
                        evaluation map at r is a ring homomorphism, which is
                        what evaluation/interpolation schemes rest on.
* `freivalds_check`  -- u^T C(x) v == sum_l (u^T A)_l(x) (B v)_l(x), compared
                        coefficient by coefficient.
* `is_prime`, `powmod` -- the oracle's own number theory.

Layout: a polynomial matrix with R x S entries of D coefficients is a numpy
array of shape (D, R, S), element (c, i, j) at offset (c*R + i)*S + j.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["lib", "is_prime", "powmod", "polymatmul", "polymatmul_entries",
           "middle_product", "middle_entries", "eval_at", "eval_points", "matmul", "polymul",
           "point_check", "freivalds_check", "host_threads"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load(path: str | None = None):
    path = path or os.path.join(_HERE, "liborc.so")
    if not os.path.exists(path):
        from . import build as _b  # builds from pm_oracle.c with gcc
        _b.build(path)
    L = ctypes.CDLL(path)
    L.orc_is_prime.argtypes = [ctypes.c_uint64]
    L.orc_is_prime.restype = ctypes.c_int
    L.orc_powmod.argtypes = [ctypes.c_uint64] * 3
    L.orc_powmod.restype = ctypes.c_uint64
    L.orc_polymatmul.argtypes = [ctypes.c_uint64] + [ctypes.c_int] * 4 + [
        _u64p, _u64p, _u64p, ctypes.c_int]
    L.orc_polymatmul.restype = ctypes.c_int
    L.orc_polymatmul_entries.argtypes = [ctypes.c_uint64] + [ctypes.c_int] * 4 + [
        _u64p, _u64p, ctypes.c_int, _i32p, _i32p, _u64p, ctypes.c_int]
    L.orc_polymatmul_entries.restype = ctypes.c_int
    L.orc_eval_at.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, _u64p, ctypes.c_uint64, _u64p]
    L.orc_eval_at.restype = None
    L.orc_matmul.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, _u64p, _u64p, _u64p]
    L.orc_matmul.restype = None
    L.orc_polymul.argtypes = [ctypes.c_uint64, ctypes.c_int, _u64p,
                              ctypes.c_int, _u64p, _u64p]
    L.orc_polymul.restype = None
    for f in (L.orc_project_left, L.orc_project_right):
        f.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      _u64p, _u64p, _u64p]
        f.restype = None
    for f in (L.orc_project_left_mt, L.orc_project_right_mt):
        f.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      _u64p, _u64p, _u64p, ctypes.c_int]
        f.restype = None
    L.orc_eval_points.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  _u64p, ctypes.c_int, _u64p, _u64p, ctypes.c_int]
    L.orc_eval_points.restype = None
    L.orc_polymul_sum.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, _u64p, _u64p,
                                  _u64p, ctypes.c_int]
    L.orc_polymul_sum.restype = None
    return L


def lib(path: str | None = None):
    """The loaded oracle library (the default build, or a given mutant)."""
    global _LIB
    if path is not None:
        return _load(path)
    if _LIB is None:
        _LIB = _load()
    return _LIB


def host_threads() -> int:
    """Threads the oracle uses: the CPUs this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def _ptr(a: np.ndarray, t=_u64p):
    return a.ctypes.data_as(t)


def is_prime(n: int, L=None) -> bool:
    return bool((L or lib()).orc_is_prime(int(n)))


def powmod(b: int, e: int, p: int, L=None) -> int:
    return int((L or lib()).orc_powmod(int(b), int(e), int(p)))


def polymatmul(p: int, A, B, threads: int | None = None, L=None) -> np.ndarray:
    """Full product C = A B mod p. A: (d, m, n), B: (d, n, k) -> C: (2d-1, m, k)."""
    A, B = _u64(A), _u64(B)
    d, m, n = A.shape
    d2, n2, k = B.shape
    if d2 != d or n2 != n:
        raise ValueError("shape mismatch")
    C = np.zeros((2 * d - 1, m, k), dtype=np.uint64)
    rc = (L or lib()).orc_polymatmul(int(p), m, n, k, d, _ptr(A), _ptr(B),
                                    _ptr(C), threads or host_threads())
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return C


def polymatmul_entries(p: int, A, B, pairs, threads: int | None = None,
                       L=None) -> np.ndarray:
    """Rows out[s, c] = C[c, i_s, j_s] for the (i, j) pairs given."""
    A, B = _u64(A), _u64(B)
    d, m, n = A.shape
    _, _, k = B.shape
    ii = np.ascontiguousarray([q[0] for q in pairs], dtype=np.int32)
    jj = np.ascontiguousarray([q[1] for q in pairs], dtype=np.int32)
    out = np.zeros((len(pairs), 2 * d - 1), dtype=np.uint64)
    rc = (L or lib()).orc_polymatmul_entries(
        int(p), m, n, k, d, _ptr(A), _ptr(B), len(pairs), _ptr(ii, _i32p),
        _ptr(jj, _i32p), _ptr(out), threads or host_threads())
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    return out


def _pad_to(X: np.ndarray, d: int) -> np.ndarray:
    """X with zero coefficients appended up to d (the polynomial is unchanged)."""
    if X.shape[0] == d:
        return X
    out = np.zeros((d,) + X.shape[1:], dtype=np.uint64)
    out[:X.shape[0]] = X
    return out


def _check_window(da: int, db: int, lo: int, length: int) -> None:
    if lo < 0 or length < 1 or lo + length > da + db - 1:
        raise ValueError("window outside the product's coefficients")


def middle_product(p: int, A, B, lo: int, length: int, threads: int | None = None,
                   L=None) -> np.ndarray:
    """Coefficients lo .. lo+length-1 of A B mod p, A: (da, m, n),
    B: (db, n, k) -> (length, m, k).  The paper's MiddleProduct(F, G, c, d)
    is middle_product(p, F, G, c, d) with F of c and G of c+d coefficients."""
    A, B = _u64(A), _u64(B)
    da, db = A.shape[0], B.shape[0]
    _check_window(da, db, lo, length)
    d = max(da, db)
    C = polymatmul(p, _pad_to(A, d), _pad_to(B, d), threads=threads, L=L)
    return np.ascontiguousarray(C[lo:lo + length])


def middle_entries(p: int, A, B, lo: int, length: int, pairs,
                   threads: int | None = None, L=None) -> np.ndarray:
    """Rows out[s, c] = (A B)[lo + c, i_s, j_s] for the (i, j) pairs given."""
    A, B = _u64(A), _u64(B)
    da, db = A.shape[0], B.shape[0]
    _check_window(da, db, lo, length)
    d = max(da, db)
    rows = polymatmul_entries(p, _pad_to(A, d), _pad_to(B, d), pairs, threads=threads, L=L)
    return np.ascontiguousarray(rows[:, lo:lo + length])


def eval_at(p: int, X, r: int, L=None) -> np.ndarray:
    """X(r) for every entry of a (D, R, S) polynomial matrix, by Horner."""
    X = _u64(X)
    D, R, S = X.shape
    out = np.zeros((R, S), dtype=np.uint64)
    (L or lib()).orc_eval_at(int(p), R, S, D, _ptr(X), int(r) % int(p), _ptr(out))
    return out


def matmul(p: int, X, Y, L=None) -> np.ndarray:
    X, Y = _u64(X), _u64(Y)
    m, n = X.shape
    n2, k = Y.shape
    Z = np.zeros((m, k), dtype=np.uint64)
    (L or lib()).orc_matmul(int(p), m, n, k, _ptr(X), _ptr(Y), _ptr(Z))
    return Z


def polymul(p: int, a, b, L=None) -> np.ndarray:
    a, b = _u64(a), _u64(b)
    out = np.zeros(len(a) + len(b) - 1, dtype=np.uint64)
    (L or lib()).orc_polymul(int(p), len(a), _ptr(a), len(b), _ptr(b), _ptr(out))
    return out


def _seeded_vectors(seed: int, p: int, count: int, length: int) -> list[np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.integers(0, p, size=length, dtype=np.uint64) if p > 1 else
            np.zeros(length, dtype=np.uint64) for _ in range(count)]


def eval_points(p: int, X, pts, threads: int | None = None, L=None) -> np.ndarray:
    """X(r) for every entry of a (D, R, S) polynomial matrix and every r in
    pts, by Horner: shape (len(pts), R, S)."""
    X = _u64(X)
    D, R, S = X.shape
    pts = _u64([int(r) % int(p) for r in pts])
    out = np.zeros((len(pts), R, S), dtype=np.uint64)
    (L or lib()).orc_eval_points(int(p), R, S, D, _ptr(X), len(pts), _ptr(pts), _ptr(out),
                                 threads or host_threads())
    return out


def _seeded_points(seed: int, p: int, count: int) -> list[int]:
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(rng.integers(0, p, dtype=np.uint64)) if p > 1 else 0 for _ in range(count)]


def point_check(p: int, A, B, C, seed: int = 0, points: int = 4, L=None,
                threads: int | None = None) -> bool:
    """C(r) == A(r) B(r) for `points` seeded r in F_p, on every entry.

    A wrong coefficient anywhere in C survives one point with probability at
    most (2d-2)/p (a nonzero polynomial of degree <= 2d-2 has at most 2d-2
    roots)."""
    L = L or lib()
    pts = _seeded_points(seed, p, points)
    eA = eval_points(p, A, pts, threads, L)
    eB = eval_points(p, B, pts, threads, L)
    eC = eval_points(p, C, pts, threads, L)
    for t in range(len(pts)):
        if not np.array_equal(eC[t], matmul(p, eA[t], eB[t], L)):
            return False
    return True


def freivalds_check(p: int, A, B, C, seed: int = 1, rounds: int = 2, L=None,
                    threads: int | None = None) -> bool:
    """u^T C(x) v == sum_l (u^T A)_l(x) * (B v)_l(x) coefficient by coefficient,
    for `rounds` seeded pairs (u, v). A wrong coefficient c of one entry C_ij
    changes coefficient c of the projection unless u_i v_j == 0 (probability
    about 2/p)."""
    L = L or lib()
    th = threads or host_threads()
    A, B, C = _u64(A), _u64(B), _u64(C)
    d, m, n = A.shape
    k = B.shape[2]
    for t in range(rounds):
        u, v = _seeded_vectors(seed * 1000 + t, p, 2, max(m, k))
        u, v = np.ascontiguousarray(u[:m]), np.ascontiguousarray(v[:k])
        uA = np.zeros((d, n), dtype=np.uint64)
        Bv = np.zeros((d, n), dtype=np.uint64)
        L.orc_project_left_mt(int(p), m, n, d, _ptr(A), _ptr(u), _ptr(uA), th)
        L.orc_project_right_mt(int(p), n, k, d, _ptr(B), _ptr(v), _ptr(Bv), th)
        uC = np.zeros((2 * d - 1, k), dtype=np.uint64)
        L.orc_project_left_mt(int(p), m, k, 2 * d - 1, _ptr(C), _ptr(u), _ptr(uC), th)
        uCv = np.zeros((2 * d - 1, 1), dtype=np.uint64)
        L.orc_project_right_mt(int(p), 1, k, 2 * d - 1,
                               _ptr(np.ascontiguousarray(uC.reshape(2 * d - 1, 1, k))),
                               _ptr(v), _ptr(uCv), th)
        # sum over l of the univariate products (u^T A)_l (B v)_l
        rhs = np.zeros(2 * d - 1, dtype=np.uint64)
        L.orc_polymul_sum(int(p), n, d, _ptr(np.ascontiguousarray(uA.T)),
                          _ptr(np.ascontiguousarray(Bv.T)), _ptr(rhs), th)
        if not np.array_equal(uCv[:, 0], rhs):
            return False
    return True
