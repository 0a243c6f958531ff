"""C-ABI library: loads, exports every declared symbol, plans correctly, and
rejects bad arguments before touching a device. CPU only (no GPU needed)."""
from __future__ import annotations

import ctypes
import math
import os
import re

import pytest

from paper_1905_04356_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions() -> list[str]:
    text = open(os.path.join(ROOT, "include", "pm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = header_functions()
    assert names, "no declarations parsed"
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(B.EXPORTS)
    assert L.pm_abi_version() == 8
    assert B.status_str(B.PM_EWORKSPACE).startswith("PM_EWORKSPACE")


def crt_bound(p, n, d):
    return n * d * (p - 1) ** 2


def test_plan_direct_mode():
    info = B.pm_plan(998244353, 8, 8, 8, 256, 4)
    assert (info.mode, info.log2_len, info.num_primes) == (0, 9, 1)
    assert info.primes[0] == 998244353
    info = B.pm_plan(2013265921, 64, 64, 32, 4096, 4)
    assert (info.mode, info.log2_len, info.num_primes) == (0, 13, 1)
    # workspace: three u32 evaluation sets of L points
    L = 8192
    assert info.workspace_bytes >= 4 * L * (64 * 64 + 64 * 32 + 64 * 32)
    # d = 1: a single point
    info = B.pm_plan(998244353, 3, 3, 3, 1, 4)
    assert (info.mode, info.log2_len) == (0, 0)


@pytest.mark.parametrize("p,n,d,eb", [
    (1152921504606847009, 32, 2048, 8),   # 60-bit modulus
    ((1 << 62) - 57, 128, 16384, 8),
    (4294967291, 64, 4096, 4),            # largest 32-bit prime: no 2^13 roots
    (998244353, 8, 1 << 15, 4),           # 2^23 | p-1 but L = 2^16 > LDS limit
    (2, 3, 100, 4),
    (1 << 40, 5, 77, 8),                  # composite modulus
])
def test_plan_crt_uses_the_fewest_primes(p, n, d, eb):
    try:
        info = B.pm_plan(p, 4, n, 4, d, eb)
    except B.PmError as e:
        assert e.status == B.PM_EUNSUPPORTED and 2 * d - 1 > (1 << 15)
        return
    assert info.mode == 1
    qs = [info.primes[i] for i in range(info.num_primes)]
    assert len(set(qs)) == len(qs)
    for q in qs:
        v2 = ((q - 1) & -(q - 1)).bit_length() - 1
        assert v2 >= info.log2_len and q < (1 << 31)
    bound = crt_bound(p, n, d)
    assert math.prod(qs) > bound
    assert math.prod(qs[:-1]) <= bound  # no prime is superfluous


def test_plan_crt_prefers_primes_below_2_30_at_the_same_count():
    """Primes with 2q - 1 <= 0x7F7F7F7F let the transforms keep lazy residues;
    the planner takes them when as many suffice, else the larger primes."""
    lazy = lambda qs: all(2 * q - 1 <= 0x7F7F7F7F for q in qs)  # noqa: E731
    p60 = (1 << 61) - 1
    c4 = B.pm_plan(p60, 32, 32, 32, 2048, 8)
    qs = [c4.primes[i] for i in range(c4.num_primes)]
    assert c4.num_primes == 5 and lazy(qs) and math.prod(qs) > crt_bound(p60, 32, 2048)
    u32 = B.pm_plan(4294967291, 64, 64, 32, 4096, 4)
    qs = [u32.primes[i] for i in range(u32.num_primes)]
    assert u32.num_primes == 3 and lazy(qs)
    # bound 32 (p-1)^2 ~ 2^61: two primes below 2^30 give 2^59.9, two of
    # 31 bits 2^62.0, so the larger primes stay
    p28 = 268435399
    w = B.pm_plan(p28, 4, 4, 4, 8, 4)
    qs = [w.primes[i] for i in range(w.num_primes)]
    assert w.num_primes == 2 and not lazy(qs) and math.prod(qs) > crt_bound(p28, 4, 8)


def test_plan_length_is_next_power_of_two():
    for d in (1, 2, 3, 4, 5, 16, 17, 33, 4096, 4097, 8192):
        info = B.pm_plan(2013265921, 2, 2, 2, d, 4)
        assert info.log2_len == (2 * d - 2).bit_length() if d > 1 else info.log2_len == 0
        assert (1 << info.log2_len) >= 2 * d - 1 > (1 << info.log2_len) // 2 or d == 1


@pytest.mark.parametrize("args,status", [
    ((1, 2, 2, 2, 4, 4), B.PM_EINVAL),             # p < 2
    ((97, 0, 2, 2, 4, 4), B.PM_EINVAL),            # m = 0
    ((97, 2, 2, 2, 0, 4), B.PM_EINVAL),            # d = 0
    ((97, 2, -1, 2, 4, 4), B.PM_EINVAL),
    ((97, 2, 2, 2, 4, 2), B.PM_EINVAL),            # elem_bytes
    ((1 << 32, 2, 2, 2, 4, 4), B.PM_ERANGE),       # p too big for u32
    ((1 << 62, 2, 2, 2, 4, 8), B.PM_ERANGE),       # p too big for u64
    ((97, 65536, 65536, 2, 4, 4), B.PM_ERANGE),    # size overflow
    ((998244353, 2, 2, 2, 1 << 20, 4), B.PM_EUNSUPPORTED),
])
def test_plan_rejects(args, status):
    with pytest.raises(B.PmError) as e:
        B.pm_plan(*args)
    assert e.value.status == status


def test_mul_argument_checks_fail_before_device_work():
    L = B.lib()
    A, Bp, C, WS = 1 << 20, 2 << 20, 3 << 20, 64 << 20  # never dereferenced
    need = B.pm_workspace_bytes(998244353, 4, 4, 4, 16, 4)
    cases = [
        ((998244353, 4, 4, 4, 16, 0, Bp, C, WS, need, None), B.PM_EINVAL),     # NULL A
        ((998244353, 4, 4, 4, 16, A + 4, Bp, C, WS, need, None), B.PM_EINVAL),  # misaligned
        ((998244353, 4, 4, 4, 16, A, Bp, A + 64, WS, need, None), B.PM_EINVAL),  # C overlaps A
        ((998244353, 4, 4, 4, 16, A, Bp, C, 0, need, None), B.PM_EWORKSPACE),
        ((998244353, 4, 4, 4, 16, A, Bp, C, WS + 16, need, None), B.PM_EWORKSPACE),
        ((998244353, 4, 4, 4, 16, A, Bp, C, WS, need - 1, None), B.PM_EWORKSPACE),
        ((998244353, 4, 4, 4, 16, A, Bp, C, A, need, None), B.PM_EINVAL),       # ws overlaps A
        ((998244353, 0, 4, 4, 16, A, Bp, C, WS, need, None), B.PM_EINVAL),
    ]
    for args, status in cases:
        assert L.pm_mul_u32(*args) == status, args
    assert L.pm_mul_u64(1 << 62, 4, 4, 4, 16, A, Bp, C, WS, need, None) == B.PM_ERANGE


def test_batched_argument_checks():
    A, Bp, C = 1 << 20, 2 << 20, 3 << 20
    arr = B.products_array([(4, 4, 4, 16, A, Bp, C), (8, 4, 2, 100, A, Bp, C + (1 << 16))])
    need = B.pm_batched_workspace_bytes(998244353, arr, 2, 4)
    one = B.pm_workspace_bytes(998244353, 4, 4, 4, 16, 4)
    two = B.pm_workspace_bytes(998244353, 8, 4, 2, 100, 4)
    assert need >= one + two
    L = B.lib()
    assert L.pm_mul_batched_u32(998244353, 2, arr, 64 << 20, need - 1, None) == B.PM_EWORKSPACE
    assert L.pm_mul_batched_u32(998244353, -1, arr, 64 << 20, need, None) == B.PM_EINVAL
    assert L.pm_mul_batched_u32(998244353, 0, arr, 64 << 20, need, None) == B.PM_OK
    bad = B.products_array([(4, 4, 4, 0, A, Bp, C)])
    with pytest.raises(B.PmError):
        B.pm_batched_workspace_bytes(998244353, bad, 1, 4)


def test_check_residues_rejects_bad_arguments():
    L = B.lib()
    out = ctypes.c_uint64(0)
    assert L.pm_check_residues(97, 0, 10, 4, ctypes.byref(out), 1 << 20, None) == B.PM_EINVAL
    assert L.pm_check_residues(97, 1 << 20, 10, 3, ctypes.byref(out), 1 << 20, None) == B.PM_EINVAL


@pytest.mark.parametrize("da,db,lo,length", [(1, 1, 0, 1), (5, 9, 5, 4), (4097, 8192, 4096, 4096),
                                             (100, 100, 0, 199), (3, 3000, 0, 3000),
                                             (2048, 4096, 2048, 2048), (7, 7, 12, 1)])
def test_middle_plan_length_is_the_least_that_keeps_the_window_exact(da, db, lo, length):
    info = B.pm_middle_plan(998244353, 2, 3, 2, da, db, lo, length, 4)
    need = max(da + db - 1 - lo, lo + length)
    L = 1 << info.log2_len
    assert L >= need and (L // 2 < need or L == 1)
    # the paper's MiddleProduct with c = d uses half the points of the whole product
    if (da, db, lo, length) == (2048, 4096, 2048, 2048):
        full = B.pm_plan(998244353, 2, 3, 2, 4096, 4)
        assert info.log2_len == full.log2_len - 1


def test_middle_plan_crt_bound_uses_the_shorter_operand():
    p = 4294967291                     # not NTT-friendly: CRT mode
    a = B.pm_middle_plan(p, 4, 64, 4, 10, 4000, 10, 3990, 4)
    b = B.pm_plan(p, 4, 64, 4, 4000, 4)
    assert a.mode == b.mode == 1
    qs = [a.primes[i] for i in range(a.num_primes)]
    assert math.prod(qs) > 64 * 10 * (p - 1) ** 2
    assert a.num_primes <= b.num_primes


@pytest.mark.parametrize("args", [(3, 3, -1, 2), (3, 3, 0, 0), (3, 3, 4, 2), (0, 3, 0, 1),
                                  (3, 0, 0, 1)])
def test_middle_plan_rejects_bad_windows(args):
    da, db, lo, length = args
    with pytest.raises(B.PmError) as e:
        B.pm_middle_plan(97, 2, 2, 2, da, db, lo, length, 4)
    assert e.value.status == B.PM_EINVAL


def test_middle_batched_workspace_and_checks():
    A, Bp, C = 1 << 20, 2 << 20, 3 << 20
    arr = B.windows_array([(4, 4, 4, 16, 32, 16, 16, A, Bp, C),
                           (2, 3, 2, 5, 9, 5, 4, A, Bp, C + (1 << 16))])
    need = B.pm_middle_batched_workspace_bytes(998244353, arr, 2, 4)
    one = B.pm_middle_plan(998244353, 4, 4, 4, 16, 32, 16, 16, 4).workspace_bytes
    assert need >= one
    L = B.lib()
    assert L.pm_middle_batched_u32(998244353, 2, arr, 64 << 20, need - 1, None) == B.PM_EWORKSPACE
    assert L.pm_middle_batched_u32(998244353, -1, arr, 64 << 20, need, None) == B.PM_EINVAL
    assert L.pm_middle_batched_u32(998244353, 0, arr, 64 << 20, need, None) == B.PM_OK
    bad = B.windows_array([(4, 4, 4, 16, 32, 40, 16, A, Bp, C)])   # window past the product
    with pytest.raises(B.PmError):
        B.pm_middle_batched_workspace_bytes(998244353, bad, 1, 4)


def test_profile_session_rules():
    """pm_profile_pause works only inside a begin/end session; an empty
    session reports nothing (no device calls are made)."""
    lib = B.lib()
    assert lib.pm_profile_pause(1) == B.PM_EINVAL
    B.pm_profile_begin()
    B.pm_profile_pause(True)
    B.pm_profile_pause(False)
    stats = B.pm_profile_end()
    assert set(stats) == set(B.KERNEL_KINDS)
    assert all(ms == 0.0 and n == 0 for ms, n in stats.values())
    assert lib.pm_profile_pause(0) == B.PM_EINVAL


@pytest.mark.parametrize("m,n,k,d,j", [
    (128, 8, 128, 4740, 13),   # 2d - 1 = 9479: 8192 points plus a 1287-coefficient top
                               # (L = 2^14: tops up to 2^13 / 4)
    (64, 64, 64, 2304, 12),    # top 511 <= 2^12 / 8 (L = 2^13 also fits 3L/4 points)
    (64, 64, 64, 2306, 0),     # top 515 > 2^12 / 8: the three-quarter transform
    (64, 64, 64, 2562, 0),     # top 1027 > 2^12 / 4
    (64, 64, 64, 1100, 0),     # (mn + nk + mk) 2^11 < 2^25
    (128, 128, 64, 560, 10),   # top 95 <= 2^10 / 8
    (128, 128, 64, 600, 0),    # top 175 > 2^10 / 8
    (3, 4, 2, 600, 0),
    (64, 64, 32, 4096, 0),     # 2d - 1 = 8191 < 2^13: no top
])
def test_plan_reports_the_wrapped_form(m, n, k, d, j):
    """pm_plan's wrap_log2_len follows the rule pm_mul applies: wrap only
    large products whose top t = 2d - 1 - 2^j is at most 2^j / 4, or 2^j / 8
    where a three-quarter transform of at most 2^13 points also fits."""
    assert B.pm_plan(998244353, m, n, k, d, 4).wrap_log2_len == j


def test_device_mbasis_argument_checks():
    """pm_mbasis_u32 and its workspace query reject bad arguments before any
    device work."""
    assert B.pm_mbasis_workspace_bytes(3, 5, 2, 4) == 4 * 3 * 5 * 2 * 4
    assert B.pm_mbasis_workspace_bytes(1, 256, 128, 2) is None        # LDS too small
    lib = B.lib()
    one = ctypes.c_void_p(16)
    for p, count, m, n, sigma, want in [((1 << 31) + 11, 1, 2, 1, 1, B.PM_ERANGE),
                                        (1, 1, 2, 1, 1, B.PM_ERANGE),
                                        (97, 0, 2, 1, 1, B.PM_EINVAL),
                                        (97, 1, 0, 1, 1, B.PM_EINVAL),
                                        (97, 1, 2, 1, 0, B.PM_EINVAL)]:
        got = lib.pm_mbasis_u32(p, count, m, n, sigma, one, 1 << 20, one, one, one, one,
                                1 << 20, None)
        assert got == want, (p, count, m, n, sigma)
    # a workspace that is too small or misaligned
    assert lib.pm_mbasis_u32(97, 1, 2, 1, 1, one, 2, one, one, one, ctypes.c_void_p(256), 4,
                             None) == B.PM_EWORKSPACE
    assert lib.pm_mbasis_u32(97, 1, 2, 1, 1, one, 2, one, one, one, ctypes.c_void_p(8), 1 << 20,
                             None) == B.PM_EWORKSPACE
    # a stride shorter than one instance
    assert lib.pm_mbasis_u32(97, 1, 2, 1, 3, one, 5, one, one, one, ctypes.c_void_p(256),
                             1 << 20, None) == B.PM_EINVAL


def test_tables_attach_and_negation_reject_bad_arguments():
    """Checks that run before the device is touched."""
    L = B.lib()
    assert L.pm_tables_attach(None, 1 << 20) == B.PM_EINVAL
    assert L.pm_tables_attach(ctypes.c_void_p((1 << 20) + 16), 1 << 20) == B.PM_EINVAL
    assert L.pm_tables_attach(ctypes.c_void_p(1 << 20), 255) == B.PM_EINVAL
    X, Y = 1 << 20, 2 << 20
    assert L.pm_neg_mod(97, None, Y, 4, 4, None) == B.PM_EINVAL
    assert L.pm_neg_mod(97, X, Y, 4, 2, None) == B.PM_EINVAL          # elem_bytes
    assert L.pm_neg_mod(1, X, Y, 4, 4, None) == B.PM_EINVAL            # p < 2
    assert L.pm_neg_mod(1 << 32, X, Y, 4, 4, None) == B.PM_ERANGE
    assert L.pm_neg_mod(1 << 62, X, Y, 4, 8, None) == B.PM_ERANGE
    assert L.pm_neg_mod(97, X, X + 4, 4, 4, None) == B.PM_EINVAL      # partial overlap
    assert L.pm_neg_mod(97, X + 4, Y, 4, 8, None) == B.PM_EINVAL      # misaligned
    assert L.pm_neg_mod(97, X, Y, 0, 4, None) == B.PM_OK               # nothing to do


def _enomem_calls():
    """(name, call) for every entry point whose host code allocates before it
    touches the device; pointers are never dereferenced."""
    A, Bp, C, WS = 1 << 20, 2 << 20, 3 << 20, 64 << 20
    p = 998244353
    L = B.lib()
    info = B.pm_plan_info()
    out = ctypes.c_uint64(0)
    prods = B.products_array([(4, 4, 4, 16, A, Bp, C), (8, 4, 2, 100, A, Bp, C + (1 << 16)),
                              (2, 2, 2, 9, A, Bp, C + (2 << 16))])
    wins = B.windows_array([(4, 4, 4, 16, 32, 16, 16, A, Bp, C),
                            (2, 3, 2, 5, 9, 5, 4, A, Bp, C + (1 << 16))])
    F = (ctypes.c_uint64 * 8)(*range(8))
    sh = (ctypes.c_int64 * 2)(0, 0)
    P = (ctypes.c_uint64 * 32)()
    rd = (ctypes.c_int64 * 2)()
    M = (ctypes.c_uint64 * 4)(1, 2, 3, 5)
    Mi = (ctypes.c_uint64 * 4)()
    ws_big = 1 << 40
    return [
        ("pm_plan", lambda: L.pm_plan(p, 4, 4, 4, 16, 4, ctypes.byref(info))),
        ("pm_workspace_bytes", lambda: L.pm_workspace_bytes(p, 4, 4, 4, 16, 4, ctypes.byref(out))),
        ("pm_tables_bytes", lambda: L.pm_tables_bytes(p, 4, 4, 4, 16, 4, ctypes.byref(out))),
        ("pm_tables_attach", lambda: L.pm_tables_attach(ctypes.c_void_p(WS), 1 << 20)),
        ("pm_mul_u32", lambda: L.pm_mul_u32(p, 4, 4, 4, 16, A, Bp, C, WS, ws_big, None)),
        ("pm_mul_u64", lambda: L.pm_mul_u64(p, 4, 4, 4, 16, A, Bp, C, WS, ws_big, None)),
        ("pm_mul_noalloc", lambda: L.pm_mul_noalloc(p, 4, 4, 4, 16, 4, A, Bp, C, None)),
        ("pm_middle_plan", lambda: L.pm_middle_plan(p, 2, 2, 2, 5, 9, 5, 4, 4,
                                                    ctypes.byref(info))),
        ("pm_middle_u32", lambda: L.pm_middle_u32(p, 2, 2, 2, 5, 9, 5, 4, A, Bp, C, WS, ws_big,
                                                  None)),
        ("pm_middle_u64", lambda: L.pm_middle_u64(p, 2, 2, 2, 5, 9, 5, 4, A, Bp, C, WS, ws_big,
                                                  None)),
        ("pm_eval_bytes", lambda: L.pm_eval_bytes(p, 0, 4, 4, 16, 4, ctypes.byref(out))),
        ("pm_eval_u32", lambda: L.pm_eval_u32(p, 0, 4, 4, 16, A, WS, ws_big, None)),
        ("pm_eval_u64", lambda: L.pm_eval_u64(p, 0, 4, 4, 16, A, WS, ws_big, None)),
        ("pm_mul_vdm_u32", lambda: L.pm_mul_vdm_u32(1000000007, 4, 4, 4, 16, A, Bp, C, WS,
                                                    ws_big, None)),
        ("pm_batched_workspace_bytes", lambda: L.pm_batched_workspace_bytes(
            p, 3, prods, 4, ctypes.byref(out))),
        ("pm_mul_batched_u32", lambda: L.pm_mul_batched_u32(p, 3, prods, WS, ws_big, None)),
        ("pm_mul_batched_u64", lambda: L.pm_mul_batched_u64(p, 3, prods, WS, ws_big, None)),
        ("pm_middle_batched_workspace_bytes", lambda: L.pm_middle_batched_workspace_bytes(
            p, 2, wins, 4, ctypes.byref(out))),
        ("pm_middle_batched_u32", lambda: L.pm_middle_batched_u32(p, 2, wins, WS, ws_big, None)),
        ("pm_middle_batched_u64", lambda: L.pm_middle_batched_u64(p, 2, wins, WS, ws_big, None)),
        ("pm_mbasis_host", lambda: L.pm_mbasis_host(97, 2, 1, 4, F, sh, P, rd)),
        ("pm_matinv_host", lambda: L.pm_matinv_host(97, 2, M, Mi)),
    ]


@pytest.mark.parametrize("name", [n for n, _ in _enomem_calls()])
def test_entry_points_return_enomem_on_injected_allocation_failure(name):
    """The library's host allocation points throw std::bad_alloc when the
    test hook arms them; every entry point must turn that into PM_ENOMEM
    (no exception crosses the C ABI) and enqueue nothing."""
    call = dict(_enomem_calls())[name]
    L = B.lib()
    assert L.pm_debug_fail_alloc(0) == B.PM_OK
    try:
        assert call() == B.PM_ENOMEM
    finally:
        L.pm_debug_fail_alloc(-1)
    # disarmed: host-only entry points succeed again
    if name in ("pm_plan", "pm_workspace_bytes", "pm_tables_bytes", "pm_middle_plan",
                "pm_eval_bytes", "pm_batched_workspace_bytes",
                "pm_middle_batched_workspace_bytes", "pm_mbasis_host", "pm_matinv_host"):
        assert call() == B.PM_OK


def test_tables_bytes_covers_every_route():
    """pm_tables_bytes counts one twiddle table per (prime, length) of the
    plan, the wrapped form's two plans, and the Vandermonde tables."""
    direct = B.pm_tables_bytes(998244353, 8, 8, 8, 256, 4)
    crt = B.pm_tables_bytes((1 << 62) - 57, 8, 8, 8, 256, 8)
    assert 0 < direct < crt
    assert crt == direct * B.pm_plan((1 << 62) - 57, 8, 8, 8, 256, 8).num_primes or crt > direct
    wrapped = B.pm_tables_bytes(998244353, 128, 8, 128, 4740, 4)
    plain = B.pm_tables_bytes(998244353, 8, 8, 8, 4096, 4)      # same L = 2^13, not wrapped
    assert B.pm_plan(998244353, 128, 8, 128, 4740, 4).wrap_log2_len == 13
    assert wrapped > plain
    vdm = B.pm_tables_bytes(1000000007, 8, 8, 8, 64, 4)        # routed to Vandermonde
    N = 2 * 64 - 1
    assert vdm >= 4 * N * 64 + 4 * N * N


def test_noalloc_rejects_products_beyond_its_scratch():
    """pm_mul_noalloc refuses, before touching a device, a product whose
    workspace exceeds its 56 MiB static scratch, and bad element sizes."""
    L = B.lib()
    A, Bp, C = 1 << 20, 2 << 20, 3 << 20
    need = B.pm_workspace_bytes(2013265921, 64, 64, 32, 4096, 4)
    assert need > 56 << 20
    assert L.pm_mul_noalloc(2013265921, 64, 64, 32, 4096, 4, A, Bp, C, None) == B.PM_ESCRATCH
    assert L.pm_mul_noalloc(998244353, 4, 4, 4, 16, 2, A, Bp, C, None) == B.PM_EINVAL
    assert L.pm_mul_noalloc(998244353, 0, 4, 4, 16, 4, A, Bp, C, None) == B.PM_EINVAL
    assert B.status_str(B.PM_ESCRATCH).startswith("PM_ESCRATCH")
