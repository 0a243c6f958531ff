"""Products by evaluation and interpolation at a geometric progression
(pm_mul_geo_u32): every coefficient against the oracle's schoolbook, for
moduli without roots of unity of 2-power order (10^9 + 7, 2^31 - 1), a small
prime with 2d - 1 = p - 1 (every point of F_p^* used), and an FFT prime;
equal to the transform path; rejected arguments."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1905_04356_amd import binding as Bd  # noqa: E402
from paper_1905_04356_amd import inputs as I  # noqa: E402
from paper_1905_04356_amd import polymat  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    (1000000007, 1, 1, 1, 1), (1000000007, 3, 2, 5, 7), (1000000007, 8, 8, 8, 64),
    (1000000007, 16, 32, 8, 100), (1000000007, 5, 7, 3, 256), (1000000007, 4, 4, 4, 1024),
    (1000000007, 2, 3, 2, 2049), (2147483647, 6, 4, 5, 300), (2147483647, 32, 32, 32, 64),
    (97, 3, 4, 2, 48), (101, 2, 2, 2, 50), (998244353, 9, 5, 7, 500),
]


@pytest.mark.parametrize("p,m,n,k,d", CASES)
def test_geometric_products_equal_the_oracle(p, m, n, k, d):
    say(f"[geo] p={p} {m}x{n}.{n}x{k} d={d}")
    A = I.polymat(70 + d, 0, I.TENSOR_A, p, d, m, n)
    B = I.polymat(70 + d, 0, I.TENSOR_B, p, d, n, k)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = polymat.mul_geo(p, tA, tB)
    torch.cuda.synchronize()
    ref = O.polymatmul(p, A, B)
    bad = np.argwhere(C.cpu().numpy().astype(np.uint64) != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"
    # the same product through the transforms
    assert torch.equal(C, polymat.mul(p, tA, tB))


def test_geometric_rejects():
    assert Bd.pm_geo_workspace_bytes(97, 2, 2, 2, 49) is None        # 2d - 1 = 97 > p - 1
    assert Bd.pm_geo_workspace_bytes(100, 2, 2, 2, 5) is None        # not prime
    assert Bd.pm_geo_workspace_bytes(2, 2, 2, 2, 1) is None          # p < 3
    assert Bd.pm_geo_workspace_bytes(1 << 31, 2, 2, 2, 5) is None    # p >= 2^31
    assert Bd.pm_geo_workspace_bytes(1000000007, 2, 4096, 2, 5) is None
    assert Bd.pm_geo_workspace_bytes(1000000007, 2, 3, 2, 5) > 0
