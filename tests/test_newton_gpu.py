"""Newton iteration for truncated inverses with GPU middle products: equal to
the oracle's coefficient recurrence (the truncated inverse is unique) on small
cases, certified by sampled entries of A S mod x^N at larger sizes, and the
truncated inverse reused as a multiplier class (evaluations computed once)
giving the same products as plain calls."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import series as S  # noqa: E402
from paper_1905_04356_amd import inputs as I  # noqa: E402
from paper_1905_04356_amd import newton  # noqa: E402
from paper_1905_04356_amd import polymat  # noqa: E402

pytestmark = pytest.mark.gpu

P30 = 998244353
P31 = 2013265921


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def invertible(p, da, n, seed, dtype=np.uint32):
    for t in range(20):
        A = I.polymat(seed + 1000 * t, 0, I.TENSOR_A, p, da, n, n, dtype)
        try:
            S.matinv(A[0].astype(object), p)
            return A
        except ValueError:
            continue
    raise RuntimeError("no invertible A(0)")


@pytest.mark.parametrize("p,n,da,N", [(P30, 3, 4, 1), (P30, 3, 4, 2), (P30, 4, 5, 17),
                                      (P31, 2, 3, 64), (97, 3, 2, 40), (P30, 5, 40, 33),
                                      ((1 << 61) - 1, 2, 4, 20)])
def test_newton_equals_recurrence(p, n, da, N):
    say(f"[newton] p={p} n={n} da={da} N={N}")
    dt = np.uint64 if p >= (1 << 32) else np.uint32
    A = invertible(p, da, n, seed=N + n, dtype=dt)
    X = newton.truncated_inverse(p, torch.from_numpy(A).cuda(), N)
    torch.cuda.synchronize()
    got = X.cpu().numpy().astype(object)
    ref = S.truncated_inverse(A.astype(object), N, p)
    assert got.shape == ref.shape and np.array_equal(got, ref)


@pytest.mark.parametrize("p,n,da,N", [(P31, 16, 1025, 2048), (P30, 32, 64, 4096)])
def test_newton_certified_sampled(p, n, da, N):
    say(f"[newton] certify p={p} n={n} da={da} N={N}")
    A = invertible(p, da, n, seed=7)
    X = newton.truncated_inverse(p, torch.from_numpy(A).cuda(), N)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy().astype(np.uint64)
    pairs = I.sample_pairs(8, n, n, 6)
    rows = O.middle_entries(p, A.astype(np.uint64), Xh, 0, N, pairs)
    for s, (i, j) in enumerate(pairs):
        want = np.zeros(N, dtype=np.uint64)
        want[0] = 1 if i == j else 0
        assert np.array_equal(rows[s], want), (i, j)


def test_inverse_as_multiplier_class():
    p, n, N, K = P31, 8, 512, 6
    A = invertible(p, 300, n, seed=11)
    Sx = newton.truncated_inverse(p, torch.from_numpy(A).cuda(), N)
    Se = newton.evaluations(p, Sx)
    Bs = [torch.from_numpy(I.polymat(12, i, I.TENSOR_B, p, N, n, 2)).cuda() for i in range(K)]
    got = polymat.mul_batched(p, [Sx] * K, Bs, A_evals=[Se] * K)
    for b, g in zip(Bs, got):
        assert torch.equal(g, polymat.mul(p, Sx, b))
    torch.cuda.synchronize()
