"""pm_mbasis_u32 (M-Basis on the device, the leaves of PM-Basis) against the
oracle's M-Basis on small cases and against pm_mbasis_host, residue for
residue, on larger ones: several instances per call, rank-deficient and zero
residuals, equal and negative shifts, eliminations that need more than
64 KiB of LDS, odd row counts."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import approx as X  # noqa: E402
from paper_1905_04356_amd import binding as Bd  # noqa: E402
from paper_1905_04356_amd import polymat  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def device_mbasis(p, Fs, sigma, shifts):
    F = torch.from_numpy(np.stack(Fs).astype(np.uint32)).cuda()
    sh = torch.tensor(shifts, dtype=torch.int64)
    P, rd = polymat.mbasis(p, F, sigma, sh)
    torch.cuda.synchronize()
    return P.cpu().numpy(), rd.cpu().tolist()


def random_series(rng, p, sigma, m, n):
    return rng.integers(0, p, size=(sigma, m, n), dtype=np.int64)


@pytest.mark.parametrize("p,sigma,m,n,shift,seed", [
    (97, 6, 3, 1, [0, 0, 0], 1),
    (101, 7, 4, 2, [3, -1, 0, 2], 3),
    (998244353, 9, 3, 2, [0, 5, 1], 4),
    (2, 12, 3, 1, [0, 0, 0], 6),
    (2013265921, 20, 5, 2, [0, 0, 0, 0, 0], 8),
])
def test_device_mbasis_equals_oracle(p, sigma, m, n, shift, seed):
    say(f"[mbasis] oracle p={p} sigma={sigma} m={m} n={n}")
    rng = np.random.default_rng(seed)
    F = random_series(rng, p, sigma, m, n)
    P, rd = device_mbasis(p, [F], sigma, [shift])
    ref = X.mbasis(F.astype(object), sigma, shift, p)
    got = X.trim(P[0].astype(object))
    assert got.shape == ref.shape and np.array_equal(got, ref)
    assert rd[0] == X.rdeg(ref, shift)


def _cases(rng, p, sigma, m, n, count):
    Fs, shifts = [], []
    for c in range(count):
        F = random_series(rng, p, sigma, m, n)
        if c % 4 == 1:
            F[:, : m // 2] = F[:, m // 2: 2 * (m // 2)]     # repeated rows: rank deficient
        elif c % 4 == 2:
            F[0] = 0                                         # zero residual in round 0
        elif c % 4 == 3:
            F[:, :, 0] = 0                                   # a zero column
        sh = [int(x) for x in rng.integers(-3, 4, size=m)]
        if c % 2:
            sh = [0] * m                                     # ties broken by index
        Fs.append(F)
        shifts.append(sh)
    return Fs, shifts


@pytest.mark.parametrize("p,sigma,m,n,count", [
    (998244353, 1, 128, 64, 2),     # 96 KiB of elimination matrix
    (998244353, 3, 128, 128, 1),    # 128 KiB
    (786433, 8, 32, 16, 4),
    (2013265921, 5, 7, 4, 4),       # odd m, even n
    (97, 10, 9, 3, 4),              # small field: many zero multipliers
    (998244353, 4, 16, 16, 4),      # n = m
])
def test_device_mbasis_equals_host(p, sigma, m, n, count):
    say(f"[mbasis] host p={p} sigma={sigma} m={m} n={n} count={count}")
    rng = np.random.default_rng(1000 * m + sigma)
    Fs, shifts = _cases(rng, p, sigma, m, n, count)
    P, rd = device_mbasis(p, Fs, sigma, shifts)
    for c in range(count):
        Ph, rdh = Bd.pm_mbasis_host(p, Fs[c].astype(np.uint64), sigma, shifts[c])
        assert np.array_equal(P[c].astype(np.uint64), Ph), c
        assert rd[c] == rdh, c


def test_device_mbasis_zero_series():
    p, sigma, m, n = 998244353, 4, 6, 3
    F = np.zeros((sigma, m, n), dtype=np.int64)
    P, rd = device_mbasis(p, [F], sigma, [[0, 1, 2, 0, 1, 2]])
    assert np.array_equal(P[0][0], np.eye(m, dtype=np.uint32)) and not P[0][1:].any()
    assert rd[0] == [0, 1, 2, 0, 1, 2]
