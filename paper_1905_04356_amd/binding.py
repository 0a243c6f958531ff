"""ctypes binding of libpm (include/pm.h): the same entry points, same names.

Only argument marshalling happens here; every step of a product runs in the
HIP kernels of libpm.so. PyTorch supplies device memory and streams. If the
library is missing the calls raise: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpm.so")

PM_OK = 0
PM_EINVAL = -1
PM_ERANGE = -2
PM_ENOMEM = -3
PM_EWORKSPACE = -4
PM_EDEVICE = -5
PM_EUNSUPPORTED = -6
PM_EBUSY = -7
PM_ETABLES = -8
PM_ESCRATCH = -9

# Every symbol include/pm.h declares.
EXPORTS = ("pm_status_str", "pm_abi_version", "pm_plan", "pm_workspace_bytes",
           "pm_mul_u32", "pm_mul_u64", "pm_batched_workspace_bytes",
           "pm_mul_batched_u32", "pm_mul_batched_u64", "pm_eval_bytes", "pm_eval_u32",
           "pm_eval_u64", "pm_check_residues", "pm_profile_begin", "pm_profile_end",
           "pm_sync", "pm_middle_plan", "pm_middle_u32", "pm_middle_u64", "pm_mbasis_host",
           "pm_matinv_host", "pm_middle_batched_workspace_bytes", "pm_middle_batched_u32",
           "pm_middle_batched_u64", "pm_vdm_workspace_bytes", "pm_mul_vdm_u32",
           "pm_profile_pause", "pm_mbasis_workspace_bytes", "pm_mbasis_u32",
           "pm_tables_attach", "pm_tables_bytes", "pm_tables_reset", "pm_tables_info",
           "pm_neg_mod", "pm_debug_fail_alloc", "pm_mul_noalloc", "pm_tune_load",
           "pm_tune_info", "pm_geo_workspace_bytes", "pm_mul_geo_u32", "pm_probe_valu")

KERNEL_KINDS = ("ntt_fwd", "pointwise", "ntt_inv", "crt", "batched", "vdm_eval", "vdm_interp",
                "geo")


class PmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class pm_plan_info(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("log2_len", ctypes.c_int32),
                ("num_primes", ctypes.c_int32), ("pointwise", ctypes.c_int32),
                ("primes", ctypes.c_uint32 * 8), ("workspace_bytes", ctypes.c_uint64),
                ("wrap_log2_len", ctypes.c_int32), ("tune_entry", ctypes.c_int32),
                ("num_points", ctypes.c_int32)]


class pm_kernel_stats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double * 8), ("launches", ctypes.c_uint64 * 8)]


class pm_product(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("d", ctypes.c_int32), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("A_eval", ctypes.c_void_p),
                ("B_eval", ctypes.c_void_p)]


class pm_window_product(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("da", ctypes.c_int32), ("db", ctypes.c_int32), ("lo", ctypes.c_int32),
                ("len", ctypes.c_int32), ("pad", ctypes.c_int32), ("A", ctypes.c_void_p),
                ("B", ctypes.c_void_p), ("C", ctypes.c_void_p)]


_lib = None


def _start_torch_runtime() -> None:
    """PyTorch's wheel carries a HIP runtime of its own, while libpm.so links
    the system one, so a process that uses both holds two.  They cooperate
    when PyTorch's is loaded and initialised first; when libpm.so (and with
    it the system runtime) is loaded before PyTorch, libpm's first kernel
    launch fails with hipErrorOutOfMemory (pinned allocations refused with
    out-of-resources).  So PyTorch, where it is installed, starts first."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def lib():
    """Load libpm.so (built by paper_1905_04356_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1905_04356_amd.build`")
    _start_torch_runtime()
    L = ctypes.CDLL(LIB_PATH)
    i32, u32, u64, vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    L.pm_status_str.argtypes = [ctypes.c_int]
    L.pm_status_str.restype = ctypes.c_char_p
    L.pm_abi_version.argtypes = []
    L.pm_abi_version.restype = ctypes.c_int
    L.pm_plan.argtypes = [u64, i32, i32, i32, i32, i32, ctypes.POINTER(pm_plan_info)]
    L.pm_workspace_bytes.argtypes = [u64, i32, i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_mul_u32.argtypes = [u32, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_mul_u64.argtypes = [u64, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_batched_workspace_bytes.argtypes = [u64, i32, ctypes.POINTER(pm_product), i32,
                                             ctypes.POINTER(u64)]
    L.pm_mul_batched_u32.argtypes = [u32, i32, ctypes.POINTER(pm_product), vp, u64, vp]
    L.pm_mul_batched_u64.argtypes = [u64, i32, ctypes.POINTER(pm_product), vp, u64, vp]
    L.pm_check_residues.argtypes = [u64, vp, u64, i32, ctypes.POINTER(u64), vp, vp]
    L.pm_sync.argtypes = [vp]
    L.pm_eval_bytes.argtypes = [u64, i32, i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_eval_u32.argtypes = [u32, i32, i32, i32, i32, vp, vp, u64, vp]
    L.pm_eval_u64.argtypes = [u64, i32, i32, i32, i32, vp, vp, u64, vp]
    L.pm_middle_plan.argtypes = [u64, i32, i32, i32, i32, i32, i32, i32, i32,
                                 ctypes.POINTER(pm_plan_info)]
    L.pm_middle_u32.argtypes = [u32, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_middle_u64.argtypes = [u64, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_mbasis_host.argtypes = [u64, i32, i32, i32, vp, vp, vp, vp]
    L.pm_matinv_host.argtypes = [u64, i32, vp, vp]
    L.pm_middle_batched_workspace_bytes.argtypes = [u64, i32, ctypes.POINTER(pm_window_product),
                                                    i32, ctypes.POINTER(u64)]
    L.pm_middle_batched_u32.argtypes = [u32, i32, ctypes.POINTER(pm_window_product), vp, u64, vp]
    L.pm_middle_batched_u64.argtypes = [u64, i32, ctypes.POINTER(pm_window_product), vp, u64, vp]
    L.pm_vdm_workspace_bytes.argtypes = [u64, i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_mul_vdm_u32.argtypes = [u32, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_profile_begin.argtypes = []
    L.pm_profile_end.argtypes = [ctypes.POINTER(pm_kernel_stats)]
    L.pm_profile_pause.argtypes = [i32]
    L.pm_mbasis_workspace_bytes.argtypes = [i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_mbasis_u32.argtypes = [u32, i32, i32, i32, i32, vp, u64, vp, vp, vp, vp, u64, vp]
    L.pm_tables_attach.argtypes = [vp, u64]
    L.pm_tables_bytes.argtypes = [u64, i32, i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_tables_reset.argtypes = []
    L.pm_tables_info.argtypes = [ctypes.POINTER(u64), ctypes.POINTER(u64),
                                 ctypes.POINTER(i32)]
    L.pm_neg_mod.argtypes = [u64, vp, vp, u64, i32, vp]
    L.pm_debug_fail_alloc.argtypes = [i32]
    L.pm_mul_noalloc.argtypes = [u64, i32, i32, i32, i32, i32, vp, vp, vp, vp]
    L.pm_tune_load.argtypes = [ctypes.c_char_p]
    L.pm_tune_info.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.pm_geo_workspace_bytes.argtypes = [u64, i32, i32, i32, i32, ctypes.POINTER(u64)]
    L.pm_mul_geo_u32.argtypes = [u32, i32, i32, i32, i32, vp, vp, vp, vp, u64, vp]
    L.pm_probe_valu.argtypes = [u32, u32, vp, vp]
    for name in ("pm_tables_attach", "pm_tables_bytes", "pm_tables_reset", "pm_tables_info",
                 "pm_neg_mod", "pm_debug_fail_alloc", "pm_mul_noalloc", "pm_tune_load",
                 "pm_tune_info", "pm_geo_workspace_bytes", "pm_mul_geo_u32", "pm_probe_valu"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("pm_plan", "pm_workspace_bytes", "pm_mul_u32", "pm_mul_u64",
                 "pm_batched_workspace_bytes", "pm_mul_batched_u32", "pm_mul_batched_u64",
                 "pm_check_residues", "pm_sync", "pm_profile_begin", "pm_profile_end",
                 "pm_eval_bytes", "pm_eval_u32", "pm_eval_u64", "pm_middle_plan",
                 "pm_middle_u32", "pm_middle_u64", "pm_mbasis_host", "pm_matinv_host",
                 "pm_middle_batched_workspace_bytes", "pm_middle_batched_u32",
                 "pm_middle_batched_u64", "pm_vdm_workspace_bytes", "pm_mul_vdm_u32",
                 "pm_profile_pause", "pm_mbasis_workspace_bytes", "pm_mbasis_u32"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def status_str(status: int) -> str:
    return lib().pm_status_str(int(status)).decode()


def _check(status: int, what: str) -> None:
    if status != PM_OK:
        raise PmError(status, what)


# ---- thin wrappers with the C names (raw pointers as ints) -----------------

def pm_plan(p: int, m: int, n: int, k: int, d: int, elem_bytes: int) -> pm_plan_info:
    info = pm_plan_info()
    _check(lib().pm_plan(p, m, n, k, d, elem_bytes, ctypes.byref(info)), "pm_plan")
    return info


def pm_workspace_bytes(p: int, m: int, n: int, k: int, d: int, elem_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_workspace_bytes(p, m, n, k, d, elem_bytes, ctypes.byref(out)),
           "pm_workspace_bytes")
    return out.value


def pm_tables_attach(ptr: int, nbytes: int) -> int:
    return lib().pm_tables_attach(ptr, nbytes)


def pm_tables_bytes(p: int, m: int, n: int, k: int, d: int, elem_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_tables_bytes(p, m, n, k, d, elem_bytes, ctypes.byref(out)),
           "pm_tables_bytes")
    return out.value


def pm_tables_reset() -> None:
    _check(lib().pm_tables_reset(), "pm_tables_reset")


def pm_tables_info() -> tuple[int, int, int]:
    """(bytes attached, bytes carved, tables) on the current device."""
    a, u, t = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_int32(0)
    _check(lib().pm_tables_info(ctypes.byref(a), ctypes.byref(u), ctypes.byref(t)),
           "pm_tables_info")
    return a.value, u.value, t.value


def pm_probe_valu(blocks, iters, out, stream) -> int:
    return lib().pm_probe_valu(blocks, iters, out, stream)


def pm_neg_mod(p, X, Y, count, elem_bytes, stream) -> int:
    return lib().pm_neg_mod(p, X, Y, count, elem_bytes, stream)


def pm_mul_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream)


def pm_mul_u64(p, m, n, k, d, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_u64(p, m, n, k, d, A, B, C, ws, ws_bytes, stream)


def products_array(prods) -> ctypes.Array:
    """(m, n, k, d, A_ptr, B_ptr, C_ptr[, A_eval_ptr, B_eval_ptr]) tuples ->
    pm_product[count] (evaluation pointers None/0 when absent)."""
    arr = (pm_product * max(1, len(prods)))()
    for i, t in enumerate(prods):
        m, n, k, d, a, b, c = t[:7]
        ae = t[7] if len(t) > 7 else None
        be = t[8] if len(t) > 8 else None
        arr[i] = pm_product(m, n, k, d, a, b, c, ae or None, be or None)
    return arr


def pm_batched_workspace_bytes(p: int, prods_arr, count: int, elem_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_batched_workspace_bytes(p, count, prods_arr, elem_bytes,
                                            ctypes.byref(out)), "pm_batched_workspace_bytes")
    return out.value


def pm_mul_batched_u32(p, count, prods_arr, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_batched_u32(p, count, prods_arr, ws, ws_bytes, stream)


def pm_mul_batched_u64(p, count, prods_arr, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_batched_u64(p, count, prods_arr, ws, ws_bytes, stream)


def pm_check_residues(p: int, x_ptr: int, count: int, elem_bytes: int, ws_ptr: int,
                      stream) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_check_residues(p, x_ptr, count, elem_bytes, ctypes.byref(out), ws_ptr,
                                   stream), "pm_check_residues")
    return out.value


def pm_sync(stream) -> None:
    _check(lib().pm_sync(stream), "pm_sync")


def pm_profile_begin() -> None:
    _check(lib().pm_profile_begin(), "pm_profile_begin")


def pm_profile_pause(paused: bool) -> None:
    _check(lib().pm_profile_pause(1 if paused else 0), "pm_profile_pause")


def pm_profile_end() -> dict:
    """{kind: (total_ms, launches)} for the kernels launched since begin."""
    st = pm_kernel_stats()
    _check(lib().pm_profile_end(ctypes.byref(st)), "pm_profile_end")
    return {name: (st.total_ms[i], int(st.launches[i]))
            for i, name in enumerate(KERNEL_KINDS)}


def pm_eval_bytes(p: int, role: int, rows: int, cols: int, d: int, elem_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_eval_bytes(p, role, rows, cols, d, elem_bytes, ctypes.byref(out)),
           "pm_eval_bytes")
    return out.value


def pm_eval_u32(p, role, rows, cols, d, X, X_eval, eval_bytes, stream) -> int:
    return lib().pm_eval_u32(p, role, rows, cols, d, X, X_eval, eval_bytes, stream)


def pm_eval_u64(p, role, rows, cols, d, X, X_eval, eval_bytes, stream) -> int:
    return lib().pm_eval_u64(p, role, rows, cols, d, X, X_eval, eval_bytes, stream)


def pm_middle_plan(p: int, m: int, n: int, k: int, da: int, db: int, lo: int, length: int,
                   elem_bytes: int) -> pm_plan_info:
    info = pm_plan_info()
    _check(lib().pm_middle_plan(p, m, n, k, da, db, lo, length, elem_bytes,
                                ctypes.byref(info)), "pm_middle_plan")
    return info


def pm_middle_u32(p, m, n, k, da, db, lo, length, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_middle_u32(p, m, n, k, da, db, lo, length, A, B, C, ws, ws_bytes, stream)


def pm_middle_u64(p, m, n, k, da, db, lo, length, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_middle_u64(p, m, n, k, da, db, lo, length, A, B, C, ws, ws_bytes, stream)


def pm_mbasis_host(p: int, F, sigma: int, shift):
    """M-Basis on the host: F a (>= sigma, m, n) integer array of residues,
    shift m integers -> (P as a (sigma+1, m, m) uint64 array, rdeg list)."""
    import numpy as np
    F = np.ascontiguousarray(np.asarray(F)[:sigma], dtype=np.uint64)
    _, m, n = F.shape
    sh = np.ascontiguousarray(shift, dtype=np.int64)
    P = np.zeros((sigma + 1, m, m), dtype=np.uint64)
    rd = np.zeros(m, dtype=np.int64)
    _check(lib().pm_mbasis_host(p, m, n, sigma, F.ctypes.data, sh.ctypes.data, P.ctypes.data,
                                rd.ctypes.data), "pm_mbasis_host")
    return P, [int(x) for x in rd]


def pm_mbasis_workspace_bytes(count: int, m: int, n: int, sigma: int) -> int | None:
    """Workspace bytes of pm_mbasis_u32, or None when the shape does not fit
    the device elimination."""
    out = ctypes.c_uint64(0)
    st = lib().pm_mbasis_workspace_bytes(count, m, n, sigma, ctypes.byref(out))
    if st == PM_EUNSUPPORTED:
        return None
    _check(st, "pm_mbasis_workspace_bytes")
    return out.value


def pm_matinv_host(p: int, M):
    """Inverse of a square matrix mod a prime p (host), as a uint64 array."""
    import numpy as np
    M = np.ascontiguousarray(np.asarray(M), dtype=np.uint64)
    n = M.shape[0]
    out = np.zeros((n, n), dtype=np.uint64)
    _check(lib().pm_matinv_host(p, n, M.ctypes.data, out.ctypes.data), "pm_matinv_host")
    return out


def windows_array(wins) -> ctypes.Array:
    """(m, n, k, da, db, lo, len, A_ptr, B_ptr, C_ptr) tuples -> pm_window_product[count]."""
    arr = (pm_window_product * max(1, len(wins)))()
    for i, (m, n, k, da, db, lo, ln, a, b, c) in enumerate(wins):
        arr[i] = pm_window_product(m, n, k, da, db, lo, ln, 0, a, b, c)
    return arr


def pm_middle_batched_workspace_bytes(p: int, arr, count: int, elem_bytes: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_middle_batched_workspace_bytes(p, count, arr, elem_bytes, ctypes.byref(out)),
           "pm_middle_batched_workspace_bytes")
    return out.value


def pm_middle_batched_u32(p, count, arr, ws, ws_bytes, stream) -> int:
    return lib().pm_middle_batched_u32(p, count, arr, ws, ws_bytes, stream)


def pm_middle_batched_u64(p, count, arr, ws, ws_bytes, stream) -> int:
    return lib().pm_middle_batched_u64(p, count, arr, ws, ws_bytes, stream)


def pm_vdm_workspace_bytes(p: int, m: int, n: int, k: int, d: int) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().pm_vdm_workspace_bytes(p, m, n, k, d, ctypes.byref(out)),
           "pm_vdm_workspace_bytes")
    return out.value


def pm_mul_vdm_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_vdm_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream)


def pm_mul_geo_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream) -> int:
    return lib().pm_mul_geo_u32(p, m, n, k, d, A, B, C, ws, ws_bytes, stream)


_tune_epoch = 0


def tune_epoch() -> int:
    """Counts the tables installed through tune_load (sizes that the
    launch shapes decide are cached per epoch)."""
    return _tune_epoch


def tune_load(text: str | None) -> None:
    """Install a tuning table (JSON text); None re-reads the default file,
    "" removes the table (defaults).  Raises on an invalid table."""
    global _tune_epoch
    st = lib().pm_tune_load(None if text is None else text.encode())
    _tune_epoch += 1
    if st != PM_OK:
        raise PmError(st, "pm_tune_load")


def tune_info() -> tuple[int, int]:
    """(entries, source) of the installed tuning table."""
    e, s = ctypes.c_int32(0), ctypes.c_int32(0)
    st = lib().pm_tune_info(ctypes.byref(e), ctypes.byref(s))
    if st != PM_OK:
        raise PmError(st, "pm_tune_info")
    return e.value, s.value


def pm_geo_workspace_bytes(p: int, m: int, n: int, k: int, d: int) -> int | None:
    """Workspace of pm_mul_geo_u32, or None when the product is not eligible."""
    out = ctypes.c_uint64(0)
    st = lib().pm_geo_workspace_bytes(p, m, n, k, d, ctypes.byref(out))
    return out.value if st == PM_OK else None
