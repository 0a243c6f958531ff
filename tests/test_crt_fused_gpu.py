"""CRT mode with the last inverse pass and the Chinese remaindering in one
kernel, and with each forward first pass computed for all primes from one
read of the input: products and coefficient windows for 2 to 5 primes, 32-
and 64-bit moduli, 3- and 4-stage first passes, full and three-quarter
lengths, equal to the oracle coefficient by coefficient and to per-prime
first passes and separate reconstruction (global knobs crt_fused = 0,
col_fwd_mp = 0)."""
from __future__ import annotations

import json
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


@pytest.fixture(autouse=True)
def _restore_table():
    yield
    torch.cuda.synchronize()
    Bd.tune_load(None)


def load(split, fused, maxr=4):
    Bd.tune_load(json.dumps({"format": "pm-tune-1",
                             "global": {"split_min_log": 8, "crt_fused": fused,
                                        "col_fwd_mp": fused, "vdm_max_d": 0},
                             "entries": [{"knobs": {"split": split, "maxr": maxr}}]}))


CASES = [  # (p, dtype, m, n, k, d, split, primes)
    (1048573, np.uint32, 4, 6, 3, 700, 4, 2),             # 2^20 - 3
    (4294967291, np.uint32, 5, 3, 4, 500, 3, 3),          # 2^32 - 5
    (4294967291, np.uint32, 3, 4, 5, 600, 4, 3),          # three-quarter
    (17592186044399, np.uint64, 4, 4, 4, 1000, 4, 4),     # 2^44 - 17
    (17592186044399, np.uint64, 3, 5, 2, 300, 3, 4),
    (1152921504606846883, np.uint64, 4, 3, 4, 700, 4, 5),  # three-quarter
    (1152921504606846883, np.uint64, 2, 3, 3, 1000, 3, 5),
    (1152921504606846883, np.uint64, 3, 3, 3, 1024, 4, 5),  # full 4-stage: not fused
]


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_fused_reconstruction_equals_the_oracle(ci):
    p, dt, m, n, k, d, split, primes = CASES[ci]
    eb = 4 if dt == np.uint32 else 8
    load(split, 1)
    info = Bd.pm_plan(p, m, n, k, d, eb)
    assert info.mode == 1 and info.num_primes == primes, (info.mode, info.num_primes)
    say(f"[crt] case {ci} p={p} {m}x{n}x{k} d={d} split={split} primes={primes} "
        f"pts={info.num_points}")
    A = I.polymat(900 + ci, 0, I.TENSOR_A, p, d, m, n, dt)
    B = I.polymat(900 + ci, 0, I.TENSOR_B, p, d, n, k, dt)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    Bd.pm_profile_begin()
    C1 = polymat.mul(p, tA, tB)
    st = Bd.pm_profile_end()
    fused = st["crt"][1] == 0
    assert fused == (not (split == 4 and primes == 5 and info.num_points == 1 << info.log2_len))
    # a coefficient window (middle product) through the same kernel
    lo, ln = d // 3, d
    W1 = polymat.middle(p, tA, tB, lo, ln)
    load(split, 0)
    C0 = polymat.mul(p, tA, tB)
    W0 = polymat.middle(p, tA, tB, lo, ln)
    torch.cuda.synchronize()
    assert torch.equal(C0, C1) and torch.equal(W0, W1)
    ref = O.polymatmul(p, A, B)
    got = C1.cpu().numpy().astype(np.uint64)
    bad = np.argwhere(got != ref)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:3].tolist()}"
    assert np.array_equal(W1.cpu().numpy().astype(np.uint64), ref[lo:lo + ln])
