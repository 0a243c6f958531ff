"""Device tables in caller-owned regions (pm_tables_attach): filled by kernels
on the caller's stream, usable from a first call inside a stream capture,
ordered between streams, and refused (PM_ETABLES, nothing enqueued) when the
regions are full. Every product is compared with the CPU oracle or with the
eager result, bit for bit.
"""
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


def tensors(p, m, n, k, d, seed, product=0, dtype=np.uint32):
    A = I.polymat(seed, product, I.TENSOR_A, p, d, m, n, dtype)
    B = I.polymat(seed, product, I.TENSOR_B, p, d, n, k, dtype)
    return A, B


def test_first_ever_table_inside_torch_graph_capture():
    """A (prime, length) pair used nowhere else (p = 7 2^20 + 1, L = 2^10)
    meets its first call inside torch.cuda.graph capture: the table fill is
    captured with the product, every replay (with eager work and
    synchronisations between replays) equals the oracle, and a later eager
    call refills the table and gives the same result."""
    p, m, n, k, d = 7340033, 6, 5, 4, 300
    say(f"[tables] capture first use p={p} d={d}")
    polymat.attach_tables()               # regions exist before the capture
    A, B = tensors(p, m, n, k, d, seed=41)
    ref = O.polymatmul(p, A, B)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ws = polymat.Workspace()
    ws.get(Bd.pm_workspace_bytes(p, m, n, k, d, 4))
    C = torch.zeros((2 * d - 1, m, k), dtype=torch.uint32, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        polymat.mul(p, tA, tB, out=C, workspace=ws)
    other_A, other_B = tensors(998244353, 8, 8, 8, 64, seed=42)
    oA, oB = torch.from_numpy(other_A).cuda(), torch.from_numpy(other_B).cuda()
    for rep in range(3):
        C.zero_()
        g.replay()
        polymat.mul(998244353, oA, oB)    # unrelated eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(C.cpu().numpy().astype(np.uint64), ref), f"replay {rep}"
    eager = polymat.mul(p, tA, tB)
    torch.cuda.synchronize()
    assert np.array_equal(eager.cpu().numpy().astype(np.uint64), ref)
    del g


def test_batched_inside_caller_capture_replays_match_eager():
    """pm_mul_batched (count >= 3) captured by the caller's torch.cuda.graph:
    the replays equal the eager batched result (the call launches its
    products with kernel arguments only, so the graph holds no pointer to
    host memory of the call)."""
    p = 998244353
    shapes = [(4, 8, 4, 100), (16, 16, 8, 900), (8, 4, 8, 40), (2, 2, 2, 1)]
    As, Bs = [], []
    for i, (m, n, k, d) in enumerate(shapes):
        A, B = tensors(p, m, n, k, d, seed=43, product=i)
        As.append(torch.from_numpy(A).cuda())
        Bs.append(torch.from_numpy(B).cuda())
    say("[tables] batched in caller capture")
    refs = [r.clone() for r in polymat.mul_batched(p, As, Bs)]
    outs = [torch.zeros_like(r) for r in refs]
    ws = polymat.Workspace()
    arr = Bd.products_array([(A.shape[1], A.shape[2], B.shape[2], A.shape[0], A.data_ptr(),
                              B.data_ptr(), C.data_ptr()) for A, B, C in zip(As, Bs, outs)])
    ws.get(Bd.pm_batched_workspace_bytes(p, arr, len(shapes), 4))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        polymat.mul_batched(p, As, Bs, outs, workspace=ws)
    for rep in range(3):
        for o in outs:
            o.zero_()
        g.replay()
        polymat.mul(p, As[0], Bs[0])
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), f"replay {rep} product {i}"
    del g


def test_tables_filled_on_one_stream_used_on_another():
    """After a reset, the first product on stream s1 fills the table and a
    product with the same (prime, length) follows at once on stream s2: s2
    waits for the fill (both results equal the oracle)."""
    p, m, n, k, d = 2013265921, 16, 16, 16, 2000
    say("[tables] two streams after reset")
    torch.cuda.synchronize()
    polymat.reset_tables()
    A, B = tensors(p, m, n, k, d, seed=44)
    ref = O.polymatmul_entries(p, A, B, [(0, 0), (15, 15), (3, 7)])
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    ws1, ws2 = polymat.Workspace(), polymat.Workspace()
    with torch.cuda.stream(s1):
        C1 = polymat.mul(p, tA, tB, workspace=ws1)
    with torch.cuda.stream(s2):
        C2 = polymat.mul(p, tA, tB, workspace=ws2)
    torch.cuda.synchronize()
    for C in (C1, C2):
        h = C.cpu().numpy().astype(np.uint64)
        for s, (i, j) in enumerate([(0, 0), (15, 15), (3, 7)]):
            assert np.array_equal(h[:, i, j], ref[s])
    assert torch.equal(C1, C2)


def test_full_regions_refuse_before_enqueueing():
    """With only a 256-byte region attached, a product whose table does not
    fit returns PM_ETABLES and leaves its output untouched; after attaching
    a real region the same call succeeds."""
    p, m, n, k, d = 998244353, 4, 4, 4, 1000
    say("[tables] full regions")
    torch.cuda.synchronize()
    polymat.reset_tables()
    tiny = torch.empty(256, dtype=torch.uint8, device="cuda")
    assert Bd.pm_tables_attach(tiny.data_ptr(), 256) == Bd.PM_OK
    A, B = tensors(p, m, n, k, d, seed=45)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = torch.full((2 * d - 1, m, k), 7, dtype=torch.uint32, device="cuda")
    need = Bd.pm_workspace_bytes(p, m, n, k, d, 4)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    st = Bd.pm_mul_u32(p, m, n, k, d, tA.data_ptr(), tB.data_ptr(), C.data_ptr(),
                       ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    assert st == Bd.PM_ETABLES
    torch.cuda.synchronize()
    assert bool((C == 7).all())
    attached, used, count = Bd.pm_tables_info()
    assert attached == 256 and used == 0 and count == 0
    region = torch.empty(Bd.pm_tables_bytes(p, m, n, k, d, 4), dtype=torch.uint8,
                         device="cuda")
    assert Bd.pm_tables_attach(region.data_ptr(), region.numel()) == Bd.PM_OK
    st = Bd.pm_mul_u32(p, m, n, k, d, tA.data_ptr(), tB.data_ptr(), C.data_ptr(),
                       ws.data_ptr(), need, torch.cuda.current_stream().cuda_stream)
    assert st == Bd.PM_OK
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy().astype(np.uint64), O.polymatmul(p, A, B))
    # hand the device back to polymat's own regions for the tests that follow
    polymat.reset_tables()
    del tiny, region


@pytest.mark.parametrize("p,dtype", [(998244353, np.uint32), (4294967291, np.uint32),
                                     ((1 << 62) - 57, np.uint64), (2, np.uint32)])
def test_neg_mod(p, dtype):
    rng = np.random.default_rng(46)
    x = (rng.integers(0, 1 << 62, size=10007, dtype=np.uint64) % np.uint64(p)).astype(dtype)
    x[:3] = [0, 1, p - 1]
    t = torch.from_numpy(x).cuda()
    y = polymat.neg(p, t)
    torch.cuda.synchronize()
    want = np.array([(p - int(v)) % p for v in x], dtype=np.uint64)
    assert np.array_equal(y.cpu().numpy().astype(np.uint64), want)
    polymat.neg(p, t, out=t)               # in place
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy().astype(np.uint64), want)


def test_valu_probe_computes_its_chains():
    """pm_probe_valu's output is the xor of its 8 chains x <- floor(x m / 2^32)
    (m = 0x9E3779B1), so the launch is checked exactly against the host."""
    from paper_1905_04356_amd import binding as Bd
    blocks, iters, m = 3, 7, 0x9E3779B1
    out = torch.zeros(blocks * 256, dtype=torch.int64, device="cuda").view(torch.uint32)
    st = torch.cuda.current_stream()
    assert Bd.pm_probe_valu(blocks, iters, out.data_ptr(), int(st.cuda_stream)) == Bd.PM_OK
    torch.cuda.synchronize()
    got = out[:blocks * 256].cpu().numpy().astype(np.uint64)
    for t in range(256):
        acc = 0
        for c in range(8):
            x = (t + 0x9E3779B9 * (c + 1)) & 0xFFFFFFFF
            for _ in range(iters):
                x = (x * m) >> 32
            acc ^= x
        assert all(int(got[b * 256 + t]) == acc for b in range(blocks)), t
    assert Bd.pm_probe_valu(0, 1, out.data_ptr(), 0) == Bd.PM_EINVAL
    assert Bd.pm_probe_valu(1, 0, out.data_ptr(), 0) == Bd.PM_EINVAL
