"""pm_mbasis_host (host code of libpm, the leaves of PM-Basis) against the
oracle's M-Basis: the same matrix and row degrees (M-Basis is deterministic and
its order-1 bases are unique), and argument checks. CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import approx as X
from paper_1905_04356_amd import binding as B


@pytest.mark.parametrize("p,sigma,m,n,shift,seed", [
    (97, 6, 3, 1, [0, 0, 0], 1),
    (101, 7, 4, 2, [3, -1, 0, 2], 3),
    (998244353, 9, 3, 2, [0, 5, 1], 4),
    (2, 12, 3, 1, [0, 0, 0], 6),
    ((1 << 61) - 1, 8, 4, 3, [0, 1, 2, 3], 7),
    (2013265921, 20, 5, 2, [0, 0, 0, 0, 0], 8),
])
def test_host_mbasis_equals_oracle(p, sigma, m, n, shift, seed):
    rng = np.random.default_rng(seed)
    F = np.array([[[int(rng.integers(0, 1 << 62)) % p for _ in range(n)] for _ in range(m)]
                  for _ in range(sigma)], dtype=object)
    ref = X.mbasis(F, sigma, shift, p)
    P, rd = B.pm_mbasis_host(p, F.astype(np.uint64), sigma, shift)
    got = X.trim(P.astype(object))
    assert got.shape == ref.shape and np.array_equal(got, ref)
    assert rd == X.rdeg(ref, shift)


def test_host_mbasis_wide_combinations_62bit():
    """A 62-bit prime with m = 48 > n = 40: the dependent rows of the first
    round combine 41 rows, and a 128-bit sum of 41 products of residues near
    2^62 wraps without the intermediate reductions."""
    p = (1 << 62) - 57
    sigma, m, n = 2, 48, 40
    rng = np.random.default_rng(62)
    F = np.array([[[int(rng.integers(p - (1 << 40), p)) for _ in range(n)] for _ in range(m)]
                  for _ in range(sigma)], dtype=object)
    shift = [0] * m
    ref = X.mbasis(F, sigma, shift, p)
    P, rd = B.pm_mbasis_host(p, F.astype(np.uint64), sigma, shift)
    got = X.trim(P.astype(object))
    assert got.shape == ref.shape and np.array_equal(got, ref)
    assert rd == X.rdeg(ref, shift)


def test_host_mbasis_rejects_bad_arguments():
    F = np.zeros((2, 2, 1), dtype=np.uint64)
    for p in (1, 91, 1 << 40):               # not prime
        with pytest.raises(B.PmError) as e:
            B.pm_mbasis_host(p, F, 2, [0, 0])
        assert e.value.status == B.PM_EINVAL
    with pytest.raises(B.PmError) as e:
        B.pm_mbasis_host((1 << 62) + 135, F, 2, [0, 0])
    assert e.value.status == B.PM_ERANGE
    L = B.lib()
    assert L.pm_mbasis_host(97, 2, 1, 0, F.ctypes.data, None, None, None) == B.PM_EINVAL


@pytest.mark.parametrize("p,n,seed", [(97, 4, 1), (998244353, 9, 2), ((1 << 61) - 1, 5, 3),
                                      (2, 6, 4)])
def test_host_matinv_equals_oracle(p, n, seed):
    from oracle import series as S
    rng = np.random.default_rng(seed)
    while True:
        M = np.array([[int(rng.integers(0, 1 << 62)) % p for _ in range(n)] for _ in range(n)],
                     dtype=object)
        try:
            ref = S.matinv(M, p)
            break
        except ValueError:
            continue
    got = B.pm_matinv_host(p, M.astype(np.uint64)).astype(object)
    assert np.array_equal(got, ref)


def test_host_matinv_rejects_singular():
    with pytest.raises(B.PmError) as e:
        B.pm_matinv_host(97, np.array([[1, 2], [2, 4]], dtype=np.uint64))
    assert e.value.status == B.PM_EINVAL
