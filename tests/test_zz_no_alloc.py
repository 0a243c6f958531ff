"""pm_mul_noalloc (no workspace, no allocation: a static scratch array)
against pm_mul_u32 / pm_mul_u64 with a caller workspace, through the C ABI:
byte-identical outputs on consecutive calls, the second one smaller, for a
direct-mode prime and for CRT moduli (u32 and u64), and the size limit."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1905_04356_amd import binding as Bd  # noqa: E402
from paper_1905_04356_amd import inputs as I  # noqa: E402
from paper_1905_04356_amd import polymat  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def operands(p, m, n, k, d, seed, dtype):
    A = I.polymat(seed, 0, I.TENSOR_A, p, d, m, n, dtype)
    B = I.polymat(seed, 0, I.TENSOR_B, p, d, n, k, dtype)
    return torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()


def noalloc(p, A, B):
    d, m, n = A.shape
    k = B.shape[2]
    eb = 4 if A.dtype == torch.uint32 else 8
    C = torch.full((2 * d - 1, m, k), 7, dtype=A.dtype, device=A.device)
    st = Bd.lib().pm_mul_noalloc(p, m, n, k, d, eb, A.data_ptr(), B.data_ptr(), C.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert st == Bd.PM_OK, Bd.status_str(st)
    return C


@pytest.mark.parametrize("p,dtype,first,second", [
    (998244353, np.uint32, (32, 32, 32, 1024), (8, 8, 8, 256)),
    (2013265921, np.uint32, (16, 24, 8, 3000), (3, 5, 2, 17)),
    (4294967291, np.uint32, (16, 16, 16, 700), (4, 4, 4, 33)),
    (1152921504606846883, np.uint64, (8, 16, 8, 900), (2, 3, 4, 100)),
])
def test_noalloc_equals_pm_mul_on_two_calls(p, dtype, first, second):
    outs = []
    for call, (m, n, k, d) in enumerate((first, second)):
        say(f"[noalloc] p={p} call {call}: {m}x{n}.{n}x{k} d={d}")
        A, B = operands(p, m, n, k, d, seed=31 + call, dtype=dtype)
        got = noalloc(p, A, B)
        want = polymat.mul(p, A, B)
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {call}"
        outs.append(got)
    assert outs[0].shape != outs[1].shape


def test_noalloc_refuses_products_beyond_its_scratch():
    p, m, n, k, d = 2013265921, 64, 64, 32, 4096
    A, B = operands(p, m, n, k, 2, seed=1, dtype=np.uint32)  # pointers only
    C = torch.empty(16, dtype=torch.uint32, device="cuda")
    st = Bd.lib().pm_mul_noalloc(p, m, n, k, d, 4, A.data_ptr(), B.data_ptr(), C.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert st == Bd.PM_ESCRATCH
