"""Truncated inverse S = A^{-1} mod x^N of a square polynomial matrix by
Newton iteration, with its products on the GPU.

Section 4 of Hyun, Neiger, Schost (ISSAC 2019), "Lifting techniques":
before Dixon's lifting, the truncated inverse of A (A(0) invertible) is
computed by matrix Newton iteration (Schulz).  With A X_k = I + x^k E
mod x^{2k}, one doubling step is
    X_{2k} = X_k - x^k (X_k E mod x^k),
where E is coefficients k .. 2k-1 of A X_k: a middle product (Section 2),
then a truncated product.  Both run through pm_middle, on transforms of
about 2k points.  X_1 = A(0)^{-1} comes from pm_matinv_host.  The
iteration keeps -A (negated once by pm_neg_mod) so that each update is a
concatenation.

Dixon's algorithm then multiplies by S again and again: S is a multiplier
class (Section 2, "Polynomial matrix multiplication").  `evaluations`
computes its evaluations once (pm_eval_*) for use as pm_product.A_eval.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as _b
from . import polymat


def truncated_inverse(p: int, A: torch.Tensor, N: int, stream=None) -> torch.Tensor:
    """S = A^{-1} mod x^N, A: (da, n, n) residues on the GPU (uint32 for
    p < 2^32, uint64 otherwise), p prime, A(0) invertible mod p.
    Returns (N, n, n) on the same device."""
    if A.dim() != 3 or A.shape[1] != A.shape[2] or N < 1:
        raise ValueError("A must be (da, n, n) and N >= 1")
    dev, dt = A.device, A.dtype
    npdt = np.uint64 if dt == torch.uint64 else np.uint32
    A0 = A[0].to("cpu").numpy().astype(np.uint64)
    with polymat._on_stream(stream, A):
        # everything below is ordered on one stream: `stream` or the current one
        X = torch.from_numpy(_b.pm_matinv_host(p, A0).astype(npdt)).to(dev)[None].contiguous()
        if N == 1:
            return X
        n = A.shape[1]
        # -A mod p (pm_neg_mod), zero-padded to N coefficients
        negA = torch.zeros((max(N, A.shape[0]), n, n), dtype=dt, device=dev)
        polymat.neg(p, A.contiguous(), out=negA[:A.shape[0]])
        negA = negA[:N]
        ws = polymat.Workspace(dev)
        k = 1
        while k < N:
            k2 = min(2 * k, N)
            h = k2 - k
            negE = polymat.middle(p, negA[:k2], X, k, h, workspace=ws)
            Y = polymat.middle(p, X, negE, 0, h, workspace=ws)
            X = torch.cat([X, Y], dim=0)
            k = k2
    return X


def evaluations(p: int, S: torch.Tensor, stream=None) -> torch.Tensor:
    """Evaluations of S as a left factor (a multiplier class), for products
    S B with B of the same coefficient count, through pm_product.A_eval."""
    return polymat.evaluate(p, S, 0, stream=stream)
