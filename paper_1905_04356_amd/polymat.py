"""Torch-facing helpers over the C ABI: allocate outputs and workspaces with
PyTorch, pass raw pointers and the current stream to libpm.

Tensors are coefficient-major: A has shape (d, m, n), B (d, n, k), and the
product C has shape (2d-1, m, k), dtype torch.uint32 (p < 2^32) or
torch.uint64 (p < 2^62), on a GPU device.
"""
from __future__ import annotations

import contextlib

import torch

from . import binding as _b


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


@contextlib.contextmanager
def _on_stream(stream, *inputs, cur=None):
    """Launch on `stream` (None: the current stream, `cur` if given).  For
    another stream, that stream first waits for the current stream's work
    (which produced the inputs), the inputs are marked as in use on it, and
    tensors allocated inside the block (outputs, workspaces) belong to it."""
    if stream is None:
        yield
        return
    if cur is None:
        cur = torch.cuda.current_stream()
    if stream == cur:
        yield
        return
    stream.wait_stream(cur)
    for t in inputs:
        if t is not None:
            t.record_stream(stream)
    with torch.cuda.stream(stream):
        yield


# ---- device tables -----------------------------------------------------------
# libpm allocates no device memory: its tables live in regions that PyTorch
# allocates here and registers once per device (pm_tables_attach), kept
# alive for the life of the process.

TABLE_REGION_BYTES = 64 << 20
_regions: dict = {}


def _dev_index(device) -> int:
    d = torch.device(device) if device is not None else torch.device("cuda")
    return d.index if d.index is not None else torch.cuda.current_device()


def attach_tables(device=None, nbytes: int = TABLE_REGION_BYTES) -> None:
    """Register `nbytes` of device memory on `device` as a table region."""
    idx = _dev_index(device)
    nbytes = max(int(nbytes), 256)
    with torch.cuda.device(idx):
        buf = torch.empty(nbytes, dtype=torch.uint8, device=torch.device("cuda", idx))
        st = _b.pm_tables_attach(buf.data_ptr(), nbytes)
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_tables_attach")
    _regions.setdefault(idx, []).append(buf)


def reset_tables(device=None) -> None:
    """Forget the tables and regions of `device` (no work may be in flight)."""
    idx = _dev_index(device)
    with torch.cuda.device(idx):
        torch.cuda.synchronize()
        _b.pm_tables_reset()
    _regions.pop(idx, None)


def _with_tables(device, call, need_bytes: int = 0) -> int:
    """call() -> pm_status, with a table region attached on first use and
    another one when the attached regions are full (the library enqueues
    nothing before reporting that)."""
    idx = _dev_index(device)
    if idx not in _regions:
        attach_tables(idx, max(TABLE_REGION_BYTES, need_bytes))
    st = call()
    if st == _b.PM_ETABLES:
        attach_tables(idx, max(TABLE_REGION_BYTES, 2 * need_bytes))
        st = call()
    return st


def _elem_bytes(t: torch.Tensor) -> int:
    if t.dtype == torch.uint32:
        return 4
    if t.dtype == torch.uint64:
        return 8
    raise TypeError(f"expected torch.uint32 or torch.uint64 residues, got {t.dtype}")


class Workspace:
    """A growable device byte buffer reused across calls on one stream."""

    def __init__(self, device=None):
        self.device = torch.device(device or "cuda")
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws: dict = {}


def _workspace(device) -> Workspace:
    key = str(device)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def plan(p: int, m: int, n: int, k: int, d: int, elem_bytes: int = 4):
    return _b.pm_plan(p, m, n, k, d, elem_bytes)


_sizes: dict = {}


def _product_sizes(p: int, m: int, n: int, k: int, d: int, eb: int) -> tuple[int, int]:
    """(workspace bytes, table bytes) of a product, cached per shape and
    tuning table (each query plans the product in the library)."""
    key = (p, m, n, k, d, eb, _b.tune_epoch())
    got = _sizes.get(key)
    if got is None:
        if len(_sizes) > 4096:
            _sizes.clear()
        got = (_b.pm_workspace_bytes(p, m, n, k, d, eb), _b.pm_tables_bytes(p, m, n, k, d, eb))
        _sizes[key] = got
    return got


def mul(p: int, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
        workspace: Workspace | None = None, stream=None) -> torch.Tensor:
    """C = A B mod p on the GPU (asynchronous on `stream`)."""
    if A.dim() != 3 or B.dim() != 3:
        raise ValueError("A and B must be (d, rows, cols)")
    d, m, n = A.shape
    d2, n2, k = B.shape
    if d2 != d or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    eb = _elem_bytes(A)
    if B.dtype != A.dtype:
        raise TypeError("A and B must have the same dtype")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be GPU tensors")
    A = A.contiguous()
    B = B.contiguous()
    cur = torch.cuda.current_stream()
    sptr = int((stream if stream is not None else cur).cuda_stream)
    with _on_stream(stream, A, B, cur=cur):
        if out is None:
            out = torch.empty((2 * d - 1, m, k), dtype=A.dtype, device=A.device)
        ws_bytes, tab_bytes = _product_sizes(p, m, n, k, d, eb)
        ws = (workspace or _workspace(A.device)).get(ws_bytes)
        fn = _b.pm_mul_u32 if eb == 4 else _b.pm_mul_u64
        st = _with_tables(A.device, lambda: fn(
            p, m, n, k, d, A.data_ptr(), B.data_ptr(), out.data_ptr(), ws.data_ptr(),
            ws.numel(), sptr), tab_bytes)
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_mul")
    return out


def middle(p: int, A: torch.Tensor, B: torch.Tensor, lo: int, length: int,
           out: torch.Tensor | None = None, workspace: Workspace | None = None,
           stream=None) -> torch.Tensor:
    """Coefficients lo .. lo+length-1 of A B mod p (A: (da, m, n), B: (db, n, k));
    the middle product of F in K[x]_c and G in K[x]_{c+d} is
    middle(p, F, G, c, d)."""
    if A.dim() != 3 or B.dim() != 3:
        raise ValueError("A and B must be (coefficients, rows, cols)")
    da, m, n = A.shape
    db, n2, k = B.shape
    if n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    eb = _elem_bytes(A)
    if B.dtype != A.dtype:
        raise TypeError("A and B must have the same dtype")
    if not (A.is_cuda and B.is_cuda):
        raise ValueError("A and B must be GPU tensors")
    A = A.contiguous()
    B = B.contiguous()
    with _on_stream(stream, A, B):
        if out is None:
            out = torch.empty((length, m, k), dtype=A.dtype, device=A.device)
        need = _b.pm_middle_plan(p, m, n, k, da, db, lo, length, eb).workspace_bytes
        ws = (workspace or _workspace(A.device)).get(need)
        fn = _b.pm_middle_u32 if eb == 4 else _b.pm_middle_u64
        st = _with_tables(A.device, lambda: fn(
            p, m, n, k, da, db, lo, length, A.data_ptr(), B.data_ptr(), out.data_ptr(),
            ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_middle")
    return out


def middle_batched(p: int, As, Bs, windows, outs=None, workspace: Workspace | None = None,
                   stream=None):
    """[coefficients lo_i .. lo_i+len_i-1 of A_i B_i mod p] in one batched call;
    windows: list of (lo, len)."""
    if not (len(As) == len(Bs) == len(windows)):
        raise ValueError("As, Bs and windows differ in length")
    if not As:
        return []
    eb = _elem_bytes(As[0])
    As = [A.contiguous() for A in As]
    Bs = [B.contiguous() for B in Bs]
    with _on_stream(stream, *As, *Bs):
        if outs is None:
            outs = [torch.empty((ln, A.shape[1], B.shape[2]), dtype=A.dtype, device=A.device)
                    for A, B, (lo, ln) in zip(As, Bs, windows)]
        wins = []
        for A, B, C, (lo, ln) in zip(As, Bs, outs, windows):
            da, m, n = A.shape
            db, n2, k = B.shape
            if n2 != n or _elem_bytes(A) != eb or _elem_bytes(B) != eb:
                raise ValueError("inconsistent batch member")
            wins.append((m, n, k, da, db, lo, ln, A.data_ptr(), B.data_ptr(), C.data_ptr()))
        arr = _b.windows_array(wins)
        need = _b.pm_middle_batched_workspace_bytes(p, arr, len(wins), eb)
        ws = (workspace or _workspace(As[0].device)).get(need)
        fn = _b.pm_middle_batched_u32 if eb == 4 else _b.pm_middle_batched_u64
        st = _with_tables(As[0].device, lambda: fn(p, len(wins), arr, ws.data_ptr(), ws.numel(),
                                                   _stream_ptr(stream)))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_middle_batched")
    return outs


def mul_vdm(p: int, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
            workspace: Workspace | None = None, stream=None) -> torch.Tensor:
    """C = A B mod p by Vandermonde evaluation/interpolation on the matrix
    cores (uint32, p prime below 2^31, 2d - 1 <= p, 2d - 1 < 4096)."""
    d, m, n = A.shape
    d2, n2, k = B.shape
    if d2 != d or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    if A.dtype != torch.uint32 or B.dtype != torch.uint32:
        raise TypeError("mul_vdm takes torch.uint32 residues")
    A = A.contiguous()
    B = B.contiguous()
    with _on_stream(stream, A, B):
        if out is None:
            out = torch.empty((2 * d - 1, m, k), dtype=A.dtype, device=A.device)
        need = _b.pm_vdm_workspace_bytes(p, m, n, k, d)
        ws = (workspace or _workspace(A.device)).get(need)
        N = 2 * d - 1
        st = _with_tables(A.device, lambda: _b.pm_mul_vdm_u32(
            p, m, n, k, d, A.data_ptr(), B.data_ptr(), out.data_ptr(), ws.data_ptr(),
            ws.numel(), _stream_ptr(stream)), 4 * N * (d + N + 2) + 1024)
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_mul_vdm")
    return out


def mul_geo(p: int, A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
            workspace: Workspace | None = None, stream=None) -> torch.Tensor:
    """C = A B mod p by evaluation and interpolation at a geometric
    progression (uint32, p prime below 2^31, 2d - 1 <= p - 1)."""
    d, m, n = A.shape
    d2, n2, k = B.shape
    if d2 != d or n2 != n:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    if A.dtype != torch.uint32 or B.dtype != torch.uint32:
        raise TypeError("mul_geo takes torch.uint32 residues")
    A = A.contiguous()
    B = B.contiguous()
    need = _b.pm_geo_workspace_bytes(p, m, n, k, d)
    if need is None:
        raise _b.PmError(_b.PM_EUNSUPPORTED, "pm_mul_geo_u32")
    with _on_stream(stream, A, B):
        if out is None:
            out = torch.empty((2 * d - 1, m, k), dtype=A.dtype, device=A.device)
        ws = (workspace or _workspace(A.device)).get(need)
        N = 2 * d - 1
        st = _with_tables(A.device, lambda: _b.pm_mul_geo_u32(
            p, m, n, k, d, A.data_ptr(), B.data_ptr(), out.data_ptr(), ws.data_ptr(),
            ws.numel(), _stream_ptr(stream)), 32 * N + (4 << 20))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_mul_geo")
    return out


def mbasis_fits(p: int, m: int, n: int, sigma: int) -> bool:
    """Whether pm_mbasis_u32 takes this shape and modulus."""
    return 2 <= p < (1 << 31) and _b.pm_mbasis_workspace_bytes(1, m, n, sigma) is not None


def mbasis(p: int, F: torch.Tensor, sigma: int, shifts: torch.Tensor,
           workspace: Workspace | None = None, stream=None):
    """Algorithm M-Basis on the device (pm_mbasis_u32) for a stack of
    instances: F (count, >= sigma, m, n) uint32 residues, shifts (count, m)
    int64 on the device -> (P (count, sigma+1, m, m) uint32, rdeg (count, m)
    int64), the same as pm_mbasis_host instance by instance."""
    if F.dim() != 4 or F.dtype != torch.uint32 or not F.is_cuda:
        raise ValueError("F must be a (count, >= sigma, m, n) uint32 GPU tensor")
    count, _, m, n = F.shape
    F = F[:, :sigma].contiguous()
    shifts = shifts.to(device=F.device, dtype=torch.int64).contiguous()
    if tuple(shifts.shape) != (count, m):
        raise ValueError("shifts must be (count, m)")
    need = _b.pm_mbasis_workspace_bytes(count, m, n, sigma)
    if need is None:
        raise _b.PmError(_b.PM_EUNSUPPORTED, "pm_mbasis_u32")
    with _on_stream(stream, F, shifts):
        P = torch.empty((count, sigma + 1, m, m), dtype=torch.uint32, device=F.device)
        rd = torch.empty((count, m), dtype=torch.int64, device=F.device)
        ws = (workspace or _workspace(F.device)).get(need)
        st = _b.lib().pm_mbasis_u32(p, count, m, n, sigma, F.data_ptr(), sigma * m * n,
                                    shifts.data_ptr(), P.data_ptr(), rd.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream_ptr(stream))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_mbasis_u32")
    return P, rd


def evaluate(p: int, X: torch.Tensor, role: int, stream=None) -> torch.Tensor:
    """Evaluations of one operand (role 0: left factor A, 1: right factor B)
    as a device byte tensor, reusable by every product with the same p,
    contraction length and degree bound (pass it to mul_batched)."""
    d, rows, cols = X.shape
    eb = _elem_bytes(X)
    X = X.contiguous()
    nbytes = _b.pm_eval_bytes(p, role, rows, cols, d, eb)
    with _on_stream(stream, X):
        out = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        fn = _b.pm_eval_u32 if eb == 4 else _b.pm_eval_u64
        st = _with_tables(X.device, lambda: fn(p, role, rows, cols, d, X.data_ptr(),
                                               out.data_ptr(), nbytes, _stream_ptr(stream)))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_eval")
    return out


def mul_batched(p: int, As, Bs, outs=None, workspace: Workspace | None = None,
                stream=None, A_evals=None, B_evals=None):
    """[A_i B_i mod p] for lists of tensors, in one batched call. A_evals /
    B_evals: optional lists of evaluate() results (or None entries)."""
    if len(As) != len(Bs):
        raise ValueError("As and Bs differ in length")
    if not As:
        return []
    eb = _elem_bytes(As[0])
    A_evals = A_evals or [None] * len(As)
    B_evals = B_evals or [None] * len(As)
    with _on_stream(stream, *As, *Bs, *A_evals, *B_evals):
        if outs is None:
            outs = [torch.empty((2 * A.shape[0] - 1, A.shape[1], B.shape[2]), dtype=A.dtype,
                                device=A.device) for A, B in zip(As, Bs)]
        prods = []
        for A, B, C, Ae, Be in zip(As, Bs, outs, A_evals, B_evals):
            d, m, n = A.shape
            if (B.shape[0] != d or B.shape[1] != n or _elem_bytes(B) != eb
                    or _elem_bytes(A) != eb):
                raise ValueError("inconsistent batch member")
            prods.append((m, n, B.shape[2], d, A.data_ptr(), B.data_ptr(), C.data_ptr(),
                          Ae.data_ptr() if Ae is not None else None,
                          Be.data_ptr() if Be is not None else None))
        arr = _b.products_array(prods)
        need = _b.pm_batched_workspace_bytes(p, arr, len(prods), eb)
        ws = (workspace or _workspace(As[0].device)).get(need)
        fn = _b.pm_mul_batched_u32 if eb == 4 else _b.pm_mul_batched_u64
        st = _with_tables(As[0].device, lambda: fn(p, len(prods), arr, ws.data_ptr(),
                                                   ws.numel(), _stream_ptr(stream)))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_mul_batched")
    return outs


def neg(p: int, X: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """-X mod p elementwise on the GPU (pm_neg_mod); out may be X (in place)."""
    eb = _elem_bytes(X)
    X = X.contiguous()
    with _on_stream(stream, X):
        if out is None:
            out = torch.empty_like(X)
        st = _b.pm_neg_mod(p, X.data_ptr(), out.data_ptr(), X.numel(), eb, _stream_ptr(stream))
    if st != _b.PM_OK:
        raise _b.PmError(st, "pm_neg_mod")
    return out
