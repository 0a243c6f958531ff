"""Seeded synthetic inputs: uniform residues, batched shape draws, 60-bit moduli.

This module holds input generation only. It contains none of the arithmetic
of polynomial-matrix multiplication, and it imports nothing else from this
package, so both the GPU path and the CPU oracle can be fed from it.

The paper measures on random matrices of polynomials over F_p (Section 2,
"Polynomial matrix multiplication", timing table; Section 1, "Experiments").
Every draw here comes from one counter-based generator: the splitmix64
finaliser of Steele, Lea and Flood (OOPSLA 2014), applied to a key derived from
(seed, stream) plus a Weyl sequence. Any element can be regenerated on its own
from (seed, stream, index).

Layouts follow the library's convention: a polynomial matrix with `rows` x
`cols` entries of `deg` coefficients is stored coefficient-major, element
(c, i, j) at offset (c * rows + i) * cols + j.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

# Stream identifiers: tensor A or B of product number `product`.
TENSOR_A = 0
TENSOR_B = 1


def mix64(z: int) -> int:
    """splitmix64 finaliser on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def _mix64_np(z: np.ndarray) -> np.ndarray:
    """Vectorised splitmix64 finaliser; numpy uint64 products wrap mod 2^64."""
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(_M1)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def _mulhi64_np(a: np.ndarray, b: int) -> np.ndarray:
    """floor(a * b / 2^64) for uint64 arrays a and a scalar b < 2^64."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0 = a & m32
    a1 = a >> s32
    b0 = np.uint64(b & 0xFFFFFFFF)
    b1 = np.uint64(b >> 32)
    t = a0 * b0
    k = t >> s32
    t = a1 * b0 + k
    w1 = t & m32
    w2 = t >> s32
    t = a0 * b1 + w1
    k = t >> s32
    return a1 * b1 + w2 + k


def stream_key(seed: int, stream: int) -> int:
    """Key of one generator stream: mix(seed xor mix(stream + 1))."""
    return mix64((seed & MASK64) ^ mix64(stream + 1))


def product_stream(product: int, tensor: int) -> int:
    """Stream number of operand `tensor` (TENSOR_A/TENSOR_B) of a product."""
    return 2 * product + tensor


def uniform_residues(seed: int, stream: int, count: int, p: int,
                     start: int = 0) -> np.ndarray:
    """`count` residues in [0, p) as uint64: element e is
    floor(mix(key + (e + 1) * GOLDEN) * p / 2^64), e = start .. start+count-1.
    """
    if not (2 <= p < (1 << 64)):
        raise ValueError("modulus out of range")
    key = np.uint64(stream_key(seed, stream))
    with np.errstate(over="ignore"):
        e = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = key + e * np.uint64(GOLDEN)
        return _mulhi64_np(_mix64_np(z), p)


def _to_i64(v: int) -> int:
    """A 64-bit pattern as a signed Python int (for torch.int64 constants)."""
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def uniform_residues_torch(seed: int, stream: int, count: int, p: int, device,
                           start: int = 0):
    """Same values as uniform_residues, computed with torch int64 tensors on
    `device` (wrapping products and logical shifts give the unsigned bits).
    Returns an int64 tensor holding values in [0, p), p < 2^63."""
    import torch
    if not (2 <= p < (1 << 63)):
        raise ValueError("modulus out of range")

    def lsr(x, s):
        return (x >> s) & ((1 << (64 - s)) - 1)

    m32 = 0xFFFFFFFF
    key = _to_i64(stream_key(seed, stream))
    e = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = e * _to_i64(GOLDEN) + key
    z = (z ^ lsr(z, 30)) * _to_i64(_M1)
    z = (z ^ lsr(z, 27)) * _to_i64(_M2)
    z = z ^ lsr(z, 31)
    a0 = z & m32
    a1 = lsr(z, 32)
    p0, p1 = p & m32, p >> 32
    t = a0 * p0
    k = lsr(t, 32)
    t = a1 * p0 + k
    w1 = t & m32
    w2 = lsr(t, 32)
    t = a0 * p1 + w1
    k = lsr(t, 32)
    return a1 * p1 + w2 + k


def polymat_torch(seed: int, product: int, tensor: int, p: int, deg: int, rows: int,
                  cols: int, device, dtype=None):
    """polymat() generated on `device`; dtype torch.uint32 (default) or
    torch.uint64."""
    import torch
    dtype = dtype or torch.uint32
    x = uniform_residues_torch(seed, product_stream(product, tensor), deg * rows * cols, p,
                               device)
    if dtype == torch.uint32:
        x = x.to(torch.int32).view(torch.uint32)
    else:
        x = x.view(torch.uint64)
    return x.reshape(deg, rows, cols)


def uniform_residue_at(seed: int, stream: int, index: int, p: int) -> int:
    """Scalar version of uniform_residues for one index (pure Python ints)."""
    z = (stream_key(seed, stream) + (index + 1) * GOLDEN) & MASK64
    return (mix64(z) * p) >> 64


def polymat(seed: int, product: int, tensor: int, p: int, deg: int, rows: int,
            cols: int, dtype=np.uint32) -> np.ndarray:
    """A seeded polynomial matrix, shape (deg, rows, cols), coefficient-major."""
    x = uniform_residues(seed, product_stream(product, tensor),
                         deg * rows * cols, p)
    return x.astype(dtype).reshape(deg, rows, cols)


class _Stream:
    """Sequential draws from one counter-based stream."""

    def __init__(self, seed: int, stream: int):
        self.key = stream_key(seed, stream)
        self.ctr = 0

    def next_u64(self) -> int:
        self.ctr += 1
        return mix64(self.key + self.ctr * GOLDEN)

    def uniform_int(self, n: int) -> int:
        return (self.next_u64() * n) >> 64

    def uniform_01(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


# Stream used for batched shape draws and serving traces (separate from the
# operand streams, which are numbered 2*product + tensor >= 0).
SHAPE_STREAM = (1 << 62) + 1
ARRIVAL_STREAM = (1 << 62) + 2
SAMPLE_STREAM = (1 << 62) + 3
PRIME_STREAM = (1 << 62) + 4

DIMS = (4, 8, 16, 32, 64, 128)
MK_PAIRS = tuple((m, k) for m in DIMS for k in DIMS if k <= m)  # 21 pairs


def batched_shapes(seed: int, count: int, log2_dmin: float = 5.0,
                   log2_dmax: float = 13.0) -> list[tuple[int, int, int, int]]:
    """Shapes (m, n, k, d) of a batch: (m, k) uniform over the 21 pairs of
    {4,...,128} with k <= m, n uniform over the six values, and
    d = round(2^u) with u uniform in [log2_dmin, log2_dmax]."""
    s = _Stream(seed, SHAPE_STREAM)
    out = []
    for _ in range(count):
        m, k = MK_PAIRS[s.uniform_int(len(MK_PAIRS))]
        n = DIMS[s.uniform_int(len(DIMS))]
        u = log2_dmin + (log2_dmax - log2_dmin) * s.uniform_01()
        d = int(round(2.0 ** u))
        out.append((m, n, k, d))
    return out


def sample_pairs(seed: int, rows: int, cols: int, count: int) -> list[tuple[int, int]]:
    """`count` distinct (i, j) pairs drawn without replacement (partial
    Fisher-Yates over the rows*cols indices, driven by the seeded stream)."""
    total = rows * cols
    count = min(count, total)
    s = _Stream(seed, SAMPLE_STREAM)
    perm = {}
    picked = []
    for t in range(count):
        r = t + s.uniform_int(total - t)
        vt, vr = perm.get(t, t), perm.get(r, r)
        perm[t], perm[r] = vr, vt
        picked.append(vr)
    return [(v // cols, v % cols) for v in picked]


def poisson_arrivals(seed: int, rate: float, duration: float) -> list[float]:
    """Arrival times of a Poisson process of the given rate on [0, duration)."""
    s = _Stream(seed, ARRIVAL_STREAM)
    t, out = 0.0, []
    while True:
        u = s.uniform_01()
        t += -math.log1p(-u) / rate
        if t >= duration:
            return out
        out.append(t)


# --- 60-bit modulus selection ---------------------------------------------

def _is_probable_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (first 13 prime bases)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for q in small:
        if n % q == 0:
            return n == q
    dd, s = n - 1, 0
    while dd % 2 == 0:
        dd //= 2
        s += 1
    for a in small:
        x = pow(a, dd, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _v2(x: int) -> int:
    return (x & -x).bit_length() - 1


def seeded_prime_60(seed: int, max_v2: int = 11) -> int:
    """A 60-bit prime with no large power-of-two roots of unity: start at
    c0 = 2^59 | (mix(key) >> 5) | 1 and step by 2 to the first prime c with
    v2(c - 1) <= max_v2 (so no 2^12-point transform exists mod c)."""
    c = (1 << 59) | (mix64(stream_key(seed, PRIME_STREAM)) >> 5) | 1
    while not (_is_probable_prime(c) and _v2(c - 1) <= max_v2):
        c += 2
    return c
