"""PM-Basis driven through the GPU middle products (Section 3, Algorithm
PM-Basis): equal, coefficient by coefficient, to the oracle's PM-Basis with the
same threshold on small cases (the algorithm is deterministic and M-Basis-1
outputs are unique), and certified at larger sizes (P F = 0 mod x^sigma
computed by the oracle, s-pivots on the diagonal, pivot degrees summing to
n sigma for F(0) of full column rank)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import approx as X  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_1905_04356_amd import binding as Bd  # noqa: E402
from paper_1905_04356_amd import inputs as I  # noqa: E402
from paper_1905_04356_amd import pmbasis as PB  # noqa: E402

pytestmark = pytest.mark.gpu

P30 = 998244353
P31 = 2013265921


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def series(p, sigma, m, n, seed, dtype=np.uint32):
    return I.polymat(seed, 0, I.TENSOR_A, p, sigma, m, n, dtype)


def run_gpu(p, F, sigma, s, T):
    tF = torch.from_numpy(F).cuda()
    P, rd = PB.pmbasis(p, tF, sigma, s, threshold=T)
    torch.cuda.synchronize()
    return P.cpu().numpy().astype(object), rd


@pytest.mark.parametrize("p,sigma,m,n,shift,T", [
    (P30, 8, 3, 1, [0, 0, 0], 1),
    (P30, 13, 4, 2, [0, 0, 0, 0], 2),
    (P31, 21, 4, 2, [3, -1, 0, 2], 4),
    (97, 17, 3, 2, [0, 5, 1], 3),
    (P30, 40, 5, 2, [0, 0, 0, 0, 0], 8),
    (P30, 64, 2, 1, [0, 0], 16),
    ((1 << 61) - 1, 12, 3, 1, [1, 0, 2], 2),
])
def test_pmbasis_equals_oracle(p, sigma, m, n, shift, T):
    say(f"[pmbasis] p={p} sigma={sigma} m={m} n={n} shift={shift} T={T}")
    dt = np.uint64 if p >= (1 << 32) else np.uint32
    F = series(p, sigma, m, n, seed=sigma + m, dtype=dt)
    P, rd = run_gpu(p, F, sigma, shift, T)
    ref = X.pmbasis(F.astype(object), sigma, shift, p, T)
    assert P.shape == ref.shape and np.array_equal(P, ref)
    assert rd == X.rdeg(ref, shift)


def test_pmbasis_threshold_does_not_change_the_basis():
    p, sigma, m, n, s = P30, 96, 4, 2, [0, 1, 0, 2]
    F = series(p, sigma, m, n, seed=9)
    bases = [run_gpu(p, F, sigma, s, T)[0] for T in (1, 5, 16, 96)]
    for B in bases[1:]:
        assert B.shape == bases[0].shape and np.array_equal(B, bases[0])


@pytest.mark.parametrize("p,sigma,m,n,T", [(P30, 512, 8, 4, 16), (P31, 1000, 6, 2, 32),
                                           (P30, 2048, 4, 1, 16)])
def test_pmbasis_certified(p, sigma, m, n, T):
    say(f"[pmbasis] certify p={p} sigma={sigma} m={m} n={n} T={T}")
    F = series(p, sigma, m, n, seed=sigma)
    s = [0] * m
    P, rd = run_gpu(p, F, sigma, s, T)
    Pu = P.astype(np.uint64)
    # P F = 0 mod x^sigma (the oracle's schoolbook window)
    PF = O.middle_product(p, Pu, F.astype(np.uint64), 0, sigma)
    assert not PF.any()
    # s-pivots on the diagonal, and pivot degrees summing to the module degree
    assert X.is_ordered_weak_popov(P, s)
    F0 = [[int(F[0, i, j]) for j in range(n)] for i in range(m)]
    assert X._rank_mod(F0, p) == n          # F(0) of full column rank
    assert X.pivot_degree_sum(P) == n * sigma
    assert rd == X.rdeg(P, s)


def test_pmbasis_many_equals_single_runs():
    """Instances in lockstep (batched residuals and products) give the same
    bases as one run each; the small instance also equals the oracle."""
    p, sigma, T = P30, 300, 8
    cases = [(4, 2, [0, 0, 0, 0]), (6, 3, [1, 0, 2, 0, 0, 1]), (5, 1, [0, 0, 0, 0, 0]),
             (3, 2, [0, 2, 1])]
    Fs = [torch.from_numpy(series(p, sigma, m, n, seed=20 + i)).cuda()
          for i, (m, n, _) in enumerate(cases)]
    many = PB.PMBasisMany(p, T)(Fs, sigma, [s for _, _, s in cases])
    for F, (m, n, s), (P, rd) in zip(Fs, cases, many):
        P1, rd1 = PB.pmbasis(p, F, sigma, s, threshold=T)
        assert P.shape == P1.shape and torch.equal(P, P1) and rd == rd1
    torch.cuda.synchronize()
    small = series(p, 40, 3, 2, seed=31)
    (P, rd), = PB.PMBasisMany(p, 4)([torch.from_numpy(small).cuda()], 40, [[0, 1, 0]])
    ref = X.pmbasis(small.astype(object), 40, [0, 1, 0], p, 4)
    assert np.array_equal(P.cpu().numpy().astype(object), ref)


def test_middle_batched_equals_single_windows():
    from paper_1905_04356_amd import polymat
    p = P31
    specs = [(3, 4, 2, 10, 25, 10, 15), (8, 8, 4, 1025, 2048, 1024, 1024),
             (2, 2, 2, 700, 3000, 650, 2300), (4, 4, 4, 33, 64, 0, 96), (1, 1, 1, 1, 1, 0, 1),
             (16, 8, 8, 513, 1024, 512, 512)]
    As, Bs, wins = [], [], []
    for i, (m, n, k, da, db, lo, ln) in enumerate(specs):
        As.append(torch.from_numpy(I.polymat(40, i, I.TENSOR_A, p, da, m, n)).cuda())
        Bs.append(torch.from_numpy(I.polymat(40, i, I.TENSOR_B, p, db, n, k)).cuda())
        wins.append((lo, ln))
    for rep in range(3):        # repeats: the third replays a captured graph
        got = polymat.middle_batched(p, As, Bs, wins)
        for A, B, (lo, ln), g in zip(As, Bs, wins, got):
            assert torch.equal(g, polymat.middle(p, A, B, lo, ln)), (rep, lo, ln)
        torch.cuda.synchronize()


@pytest.mark.parametrize("p,sigma,m,n,shift,T", [
    (P30, 13, 4, 2, [0, 0, 0, 0], 2),
    (P31, 21, 4, 2, [3, -1, 0, 2], 4),
    (97, 17, 3, 2, [0, 5, 1], 3),
    (786433, 64, 32, 16, [0] * 32, 8),
])
def test_pmbasis_device_leaves_equal_host_leaves(p, sigma, m, n, shift, T):
    """Leaves on the device (pm_mbasis_u32) give the same basis as leaves on
    the host, for one instance and for a lockstep family of two shapes."""
    say(f"[pmbasis] device leaves p={p} sigma={sigma} m={m} n={n} T={T}")
    F = torch.from_numpy(series(p, sigma, m, n, seed=sigma + 3 * m)).cuda()
    dev = PB.PMBasis(p, T, device_leaf_min=1)
    Pd, rdd = dev(F, sigma, shift)
    Ph, rdh = PB.PMBasis(p, T, device_leaf_min=1 << 30)(F, sigma, shift)
    assert dev.leaves > 0 and Pd.shape == Ph.shape and torch.equal(Pd, Ph) and rdd == rdh
    if m <= 5:
        ref = X.pmbasis(F.cpu().numpy().astype(object), sigma, shift, p, T)
        assert np.array_equal(Pd.cpu().numpy().astype(object), ref)
    G = torch.from_numpy(series(p, sigma, m + 1, n, seed=7)).cuda()
    fam = [F, G, F.flip(1).contiguous(), G]
    shifts = [shift, [0] * (m + 1), shift[::-1], [1] * (m + 1)]
    many = PB.PMBasisMany(p, T, device_leaf_min=2)(fam, sigma, shifts)
    for Fi, si, (P, rd) in zip(fam, shifts, many):
        P1, rd1 = PB.PMBasis(p, T, device_leaf_min=1 << 30)(Fi, sigma, si)
        assert P.shape == P1.shape and torch.equal(P, P1) and rd == rd1
