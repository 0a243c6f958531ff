"""Algorithm PM-Basis (Section 3, "Approximant bases") with its polynomial
products on the GPU.

PM-Basis(F, sigma, s): below the threshold T it is M-Basis, on the host
(pm_mbasis_host), or on the device (pm_mbasis_u32, one workgroup per
instance) for families of at least `device_leaf_min` same-shape instances
in lockstep (32-bit residues mod p < 2^31, shapes whose elimination fits
the LDS): one elimination is a serial chain that a host core runs faster,
but the device runs many at once; above it,
    P1 = PM-Basis(F mod x^c, c, s)            c = ceil(sigma / 2)
    R  = MiddleProduct(P1, F, c, sigma - c)   coefficients c .. sigma-1 of P1 F
    P2 = PM-Basis(R, sigma - c, rdeg_s(P1))
    return P2 P1
The residual and the product run through pm_middle (the residual on a
transform of about sigma points instead of 1.5 sigma). Bases stay on the
device; a device leaf sends only its row degrees to the host (they steer
the recursion), a host leaf its input and output.
The shifts follow the predictable-degree property: the row degrees
rdeg_s(P2 P1) equal rdeg_{rdeg_s(P1)}(P2), so deg(P) <= max rdeg - min s
bounds the coefficients kept.
"""
from __future__ import annotations

import concurrent.futures
import os
import time

import numpy as np
import torch

from . import binding as _b
from . import polymat


def _trim_host(P: np.ndarray) -> np.ndarray:
    D = P.shape[0]
    while D > 1 and not P[D - 1].any():
        D -= 1
    return P[:D]


class PMBasis:
    """One PM-Basis computation mod a prime p (residues as torch.uint32 for
    p < 2^32, torch.uint64 otherwise)."""

    def __init__(self, p: int, threshold: int = 16, stream=None, device_leaf_min: int = 16):
        if threshold < 1:
            raise ValueError("threshold must be >= 1")
        self.p = p
        self.T = threshold
        self.device_leaf_min = device_leaf_min
        self.stream = stream
        self.ws = None
        self.leaves = 0
        self.products = 0
        self.leaf_seconds = 0.0   # host time in the leaves (copies included)

    def _device_leaf(self, F: torch.Tensor, sigma: int, count: int = 1) -> bool:
        return (count >= self.device_leaf_min and F.dtype == torch.uint32 and
                polymat.mbasis_fits(self.p, F.shape[1], F.shape[2], sigma))

    def _device_leaves(self, Fs, sigma: int, ss):
        """M-Basis of same-shape instances in one pm_mbasis_u32 call; their
        row degrees are read back (one small copy)."""
        if self.ws is None:
            self.ws = polymat.Workspace(Fs[0].device)
        stack = torch.stack([F[:sigma] for F in Fs])
        sh = torch.tensor(ss, dtype=torch.int64, device=Fs[0].device)
        P, rd = polymat.mbasis(self.p, stack, sigma, sh, workspace=self.ws, stream=self.stream)
        if self.stream is not None:
            self.stream.synchronize()
        rds = rd.tolist()
        # each basis in an allocation of its own: the products take 16-byte
        # aligned operands, which views into the stack need not be
        return [self._bound(P[i], rds[i], ss[i]).clone() for i in range(len(Fs))], rds

    def _leaf(self, F: torch.Tensor, sigma: int, s: list[int]):
        t0 = time.perf_counter()
        if self._device_leaf(F, sigma):
            (P,), (rd,) = self._device_leaves([F], sigma, [s])
            self.leaves += 1
            self.leaf_seconds += time.perf_counter() - t0
            return P, rd
        Fh = F[:sigma].to("cpu").numpy().astype(np.uint64)
        P, rd = _b.pm_mbasis_host(self.p, Fh, sigma, s)
        P = _trim_host(P)
        self.leaves += 1
        out = torch.from_numpy(P.astype(np.uint64 if F.dtype == torch.uint64 else np.uint32)
                               ).to(F.device)
        self.leaf_seconds += time.perf_counter() - t0
        return out, rd

    def _bound(self, P: torch.Tensor, rd: list[int], s: list[int]) -> torch.Tensor:
        keep = max(rd) - min(s) + 1
        return P[:max(1, min(P.shape[0], keep))]

    def _run(self, F: torch.Tensor, sigma: int, s: list[int]):
        if sigma <= self.T:
            return self._leaf(F, sigma, s)
        c = (sigma + 1) // 2
        d = sigma - c
        P1, s1 = self._run(F[:c], c, s)
        if self.ws is None:
            self.ws = polymat.Workspace(F.device)
        R = polymat.middle(self.p, P1, F[:sigma], c, d, workspace=self.ws, stream=self.stream)
        P2, s2 = self._run(R, d, s1)
        P = polymat.middle(self.p, P2, P1, 0, P2.shape[0] + P1.shape[0] - 1,
                           workspace=self.ws, stream=self.stream)
        self.products += 2
        return self._bound(P, s2, s), s2

    def __call__(self, F: torch.Tensor, sigma: int, shift) -> tuple[torch.Tensor, list[int]]:
        """F: (>= sigma, m, n) residues on the GPU; shift: m integers.
        Returns (P, rdeg): P (deg+1, m, m) on the GPU, an s-ordered weak Popov
        approximant basis of (F, sigma), and rdeg_s(P)."""
        if F.dim() != 3 or F.shape[0] < sigma or sigma < 1:
            raise ValueError("F must be (>= sigma, m, n) with sigma >= 1")
        s = [int(x) for x in shift]
        if len(s) != F.shape[1]:
            raise ValueError("one shift per row of F")
        P, rd = self._run(F.contiguous(), sigma, s)
        # exact trim of trailing zero coefficients (one reduction on the device)
        signed = torch.int64 if P.dtype == torch.uint64 else torch.int32
        nz = torch.nonzero(P.reshape(P.shape[0], -1).view(signed).ne(0).any(dim=1))
        D = int(nz.max().item()) + 1 if nz.numel() else 1
        return P[:D].contiguous(), rd


def pmbasis(p: int, F: torch.Tensor, sigma: int, shift, threshold: int = 16, stream=None):
    """PM-Basis(F, sigma, shift) mod p; see PMBasis."""
    return PMBasis(p, threshold, stream)(F, sigma, shift)


class PMBasisMany(PMBasis):
    """Several independent PM-Basis computations of the same order, run in
    lockstep: at every node of the recursion the residuals of all instances
    are one pm_middle_batched call, and so are their basis products, so the
    batched phase kernels carry the whole family (shapes and degrees may
    differ between instances)."""

    def __init__(self, p: int, threshold: int = 16, stream=None, workers: int | None = None,
                 device_leaf_min: int = 16):
        super().__init__(p, threshold, stream, device_leaf_min)
        self.workers = workers or min(16, os.cpu_count() or 1)
        self.pool = None

    def _leaves(self, Fs, sigma: int, ss):
        """The instances' leaves are independent: on the device, instances of
        one shape share a pm_mbasis_u32 call; on the host, the eliminations
        run on a thread pool (the C calls release the interpreter lock)."""
        t0 = time.perf_counter()
        Ps, rds = [None] * len(Fs), [None] * len(Fs)
        shapes = {}
        for i, F in enumerate(Fs):
            shapes.setdefault((F.shape[1], F.shape[2]), []).append(i)
        groups, host = [], []
        for idx in shapes.values():
            if self._device_leaf(Fs[idx[0]], sigma, len(idx)):
                groups.append(idx)
            else:
                host.extend(idx)
        host.sort()
        for idx in groups:
            P, rd = self._device_leaves([Fs[i] for i in idx], sigma, [ss[i] for i in idx])
            for j, i in enumerate(idx):
                Ps[i], rds[i] = P[j], rd[j]
        if host:
            hosts = [Fs[i][:sigma].to("cpu").numpy().astype(np.uint64) for i in host]
            if self.pool is None:
                self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=self.workers)
            res = list(self.pool.map(lambda a: _b.pm_mbasis_host(self.p, a[0], sigma, a[1]),
                                     zip(hosts, [ss[i] for i in host])))
            npdt = np.uint64 if Fs[0].dtype == torch.uint64 else np.uint32
            for i, (P, rd) in zip(host, res):
                Ps[i] = torch.from_numpy(_trim_host(P).astype(npdt)).to(Fs[i].device)
                rds[i] = rd
        self.leaves += len(Fs)
        self.leaf_seconds += time.perf_counter() - t0
        return Ps, rds

    def _run_many(self, Fs, sigma: int, ss):
        if sigma <= self.T:
            return self._leaves(Fs, sigma, ss)
        c = (sigma + 1) // 2
        d = sigma - c
        P1s, s1s = self._run_many([F[:c] for F in Fs], c, ss)
        if self.ws is None:
            self.ws = polymat.Workspace(Fs[0].device)
        Rs = polymat.middle_batched(self.p, P1s, [F[:sigma] for F in Fs], [(c, d)] * len(Fs),
                                    workspace=self.ws, stream=self.stream)
        P2s, s2s = self._run_many(Rs, d, s1s)
        Ps = polymat.middle_batched(self.p, P2s, P1s,
                                    [(0, a.shape[0] + b.shape[0] - 1) for a, b in zip(P2s, P1s)],
                                    workspace=self.ws, stream=self.stream)
        self.products += 2 * len(Fs)
        return [self._bound(P, s2, s) for P, s2, s in zip(Ps, s2s, ss)], s2s

    def __call__(self, Fs, sigma: int, shifts):
        """Fs: list of (>= sigma, m_i, n_i) GPU tensors; shifts: one list per
        instance.  Returns a list of (P, rdeg), as PMBasis does for each."""
        if not Fs or len(Fs) != len(shifts):
            raise ValueError("one shift list per series")
        ss = [[int(x) for x in s] for s in shifts]
        for F, s in zip(Fs, ss):
            if F.dim() != 3 or F.shape[0] < sigma or len(s) != F.shape[1]:
                raise ValueError("each F must be (>= sigma, m, n) with m shifts")
        Ps, rds = self._run_many([F.contiguous() for F in Fs], sigma, ss)
        out = []
        for P, rd in zip(Ps, rds):
            signed = torch.int64 if P.dtype == torch.uint64 else torch.int32
            nz = torch.nonzero(P.reshape(P.shape[0], -1).view(signed).ne(0).any(dim=1))
            D = int(nz.max().item()) + 1 if nz.numel() else 1
            out.append((P[:D].contiguous(), rd))
        return out
