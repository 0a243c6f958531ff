"""The tuning table (launch shapes per prime class, transform length and shape
bucket): parsing, matching, global knobs, rejection of invalid tables, and the
fall-back to the defaults when the file is missing or invalid. Host only."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

from paper_1905_04356_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
P31 = 2013265921
P30 = 998244353


@pytest.fixture(autouse=True)
def _restore_table():
    yield
    B.tune_load(None)


def table(entries=(), glob=None):
    t = {"format": "pm-tune-1", "entries": list(entries)}
    if glob is not None:
        t["global"] = glob
    return json.dumps(t)


def test_no_table_means_defaults():
    B.tune_load("")
    assert B.tune_info() == (0, 0)
    info = B.pm_plan(P31, 64, 64, 32, 4096, 4)
    assert info.tune_entry == -1 and info.pointwise == 1


def test_entries_match_by_class_length_and_bucket_first_match_wins():
    B.tune_load(table([
        {"prime_class": "direct_ge30", "log2_len": 13, "m_log2": 6, "n_log2": 6, "k_log2": 5,
         "knobs": {"pointwise": 0, "blk_nt": 512}, "us": 123.4},
        {"prime_class": "direct_ge30", "log2_len": 13, "knobs": {"maxr": 3}},
        {"prime_class": "crt", "knobs": {"colvec_fwd": 1}},
        {"knobs": {"reg_tile": 0}},
    ]))
    assert B.tune_info() == (4, 2)
    c2 = B.pm_plan(P31, 64, 64, 32, 4096, 4)
    assert c2.tune_entry == 0 and c2.pointwise == 0
    # same class and length, other bucket: the second entry
    assert B.pm_plan(P31, 8, 8, 8, 4096, 4).tune_entry == 1
    # q < 2^30: not direct_ge30, so the catch-all entry
    assert B.pm_plan(P30, 64, 64, 32, 4096, 4).tune_entry == 3
    # CRT modulus
    assert B.pm_plan((1 << 61) - 1, 4, 4, 4, 100, 8).tune_entry == 2
    # shape buckets are ceil(log2): 33..64 -> 6, 17..32 -> 5
    assert B.pm_plan(P31, 40, 50, 20, 4096, 4).tune_entry == 0
    assert B.pm_plan(P31, 40, 50, 17, 4096, 4).tune_entry == 0
    assert B.pm_plan(P31, 40, 50, 16, 4096, 4).tune_entry == 1


@pytest.mark.parametrize("knobs", [{"maxr": 2, "split": 3}, {"maxr": 3}, {"split": 0},
                                   {"split": 2, "maxr": 4}, {"split": 5}])
def test_pass_structure_knobs_keep_the_twiddle_count(knobs):
    """Any pass structure needs sum_i S_i (2^r_i - 1) = L - 1 twiddles per
    direction (the sum telescopes), so the table size of a length does not
    depend on the knobs; the plan reports the entry it used."""
    B.tune_load(table([{"knobs": knobs}]))
    for logL in (9, 12, 13, 15):
        d = 1 << (logL - 1)
        want = -(-2 * ((1 << logL) - 1) * 8 // 256) * 256
        assert B.pm_tables_bytes(P31, 8, 8, 8, d, 4) == want
        assert B.pm_plan(P31, 8, 8, 8, d, 4).tune_entry == 0


def test_global_knobs_move_the_wrapped_length_rule():
    """The wrap rule's size bound is a global knob: lowering it lets a small
    product with a small top take the wrapped form."""
    B.tune_load("")
    m, n, k, d = 8, 8, 8, 1100                 # 2d - 1 = 2199 = 2^11 + 151
    assert B.pm_plan(P30, m, n, k, d, 4).wrap_log2_len == 0
    # (three-quarter transforms off: they take over this top otherwise)
    B.tune_load(table(glob={"wrap_min_work_log": 0, "trunc34": 0}))
    assert B.pm_plan(P30, m, n, k, d, 4).wrap_log2_len == 11
    B.tune_load(table(glob={"wrap_min_work_log": 0, "wrap_top_div": 64, "trunc34": 0}))
    assert B.pm_plan(P30, m, n, k, d, 4).wrap_log2_len == 0   # 151 > 2048 / 64


def test_three_quarter_transforms_are_planned_for_whole_products_in_the_band():
    """Whole products with L/2 < 2d - 1 <= 3L/4 on split transforms take 3L/4
    points (the workspace shrinks with them); 2d - 1 above the band, unsplit
    lengths, coefficient windows and the knob set to 0 keep L points; with
    the knob at 2 the three-quarter transform replaces the wrapped form."""
    B.tune_load("")
    for d, L, pts in [(1025, 4096, 3072), (1536, 4096, 3072), (1537, 4096, 4096),
                      (2049, 8192, 6144), (3072, 8192, 6144), (4096, 8192, 8192)]:
        info = B.pm_plan(P31, 16, 16, 8, d, 4)
        assert (1 << info.log2_len, info.num_points) == (L, pts), d
    full = B.pm_plan(P31, 16, 16, 8, 1500, 4)
    B.tune_load(table(glob={"trunc34": 0}))
    off = B.pm_plan(P31, 16, 16, 8, 1500, 4)
    assert off.num_points == 4096 and full.num_points == 3072
    assert 3 * off.workspace_bytes == 4 * full.workspace_bytes
    # unsplit transforms: no
    B.tune_load(table([{"knobs": {"split": 0}}]))
    assert B.pm_plan(P31, 16, 16, 8, 1500, 4).num_points == 4096
    # CRT moduli too (every prime's transform)
    B.tune_load("")
    crt = B.pm_plan((1 << 61) - 1, 4, 4, 4, 1500, 8)
    assert crt.mode == 1 and crt.num_points == 3072
    # where both apply, the wrapped form keeps the small tops: t <= 2^j / 8 for
    # L <= 2^13, every top of its band above; the knob at 2: never wrapped
    B.tune_load(table(glob={"wrap_min_work_log": 0}))
    assert B.pm_plan(P30, 8, 8, 8, 1200, 4).wrap_log2_len == 0     # t = 351 > 2^11 / 8
    assert B.pm_plan(P30, 8, 8, 8, 1050, 4).wrap_log2_len == 11    # t = 51
    assert B.pm_plan(P30, 8, 8, 8, 4300, 4).wrap_log2_len == 13    # L = 2^14, t = 407
    assert B.pm_plan(P30, 8, 8, 8, 4300, 4).num_points == 12288
    B.tune_load(table(glob={"wrap_min_work_log": 0, "wrap_top_div_tr": 4}))
    assert B.pm_plan(P30, 8, 8, 8, 1200, 4).wrap_log2_len == 11
    B.tune_load(table(glob={"wrap_min_work_log": 0, "trunc34": 2}))
    w = B.pm_plan(P30, 8, 8, 8, 1050, 4)
    assert w.wrap_log2_len == 0 and w.num_points == 3072


def test_every_global_knob_is_accepted():
    glob = {"lds_log": 14, "split_min_log": 11, "blk_pad": 0, "batch_tile_log": 14,
            "batch_pw_work": 8192, "batch_pw_pipe_pts": 16, "batch_direct_max": 2,
            "batch_graph": 1, "wrap_min_log": 10, "wrap_top_div": 4, "wrap_min_work_log": 25,
            "vdm_max_d": 64, "min_wg": 512, "min_wg_unsplit": 256, "trunc34": 1,
            "wrap_top_div_tr": 8, "wrap_tr_max_log": 13, "crt_fused": 1,
            "batch_single_min_log": 25, "col_fwd_mp": 1, "lazy": 1}
    B.tune_load(table(glob=glob))
    assert B.tune_info()[0] == 0
    # the defaults, so plans are those of no table
    def plan():
        x = B.pm_plan(P31, 64, 64, 32, 4096, 4)
        return [list(v) if f == "primes" else v
                for f, v in ((f[0], getattr(x, f[0])) for f in x._fields_)]

    c2 = plan()
    B.tune_load("")
    assert plan() == c2


@pytest.mark.parametrize("bad", [
    "{",                                                             # not JSON
    "[]",                                                            # not an object
    '{"format": "pm-tune-2", "entries": []}',                        # unknown format
    table([{"knobs": {"blk_nt": 300}}]),                             # bad value
    table([{"knobs": {"colvec_fwd": 3}}]),
    table([{"knobs": {"split": 1}}]),
    table([{"knobs": {"no_such_knob": 1}}]),                         # unknown knob
    table([{"prime_class": "big", "knobs": {}}]),                    # bad class
    table([{"log2_len": -1, "knobs": {}}]),                          # bad selector
    table([{"knobs": {"maxr": 3.5}}]),                               # not an integer
    table(glob={"wrap_top_div": 0}),                                 # bad global
    table(glob={"nope": 1}),
    table(glob={"trunc34": 3}),
    table(glob={"min_wg_unsplit": -1}),
    table([{"knobs": {"split": 6}}]),
    table([{"knobs": {}}]) + "x",                                    # trailing text
])
def test_invalid_tables_are_rejected_and_the_current_one_stays(bad):
    B.tune_load(table([{"knobs": {"reg_tile": 0}}]))
    with pytest.raises(B.PmError) as e:
        B.tune_load(bad)
    assert e.value.status == B.PM_EINVAL
    assert B.tune_info() == (1, 2)


def test_vandermonde_route_is_reported():
    B.tune_load("")
    assert B.pm_plan(1000000007, 4, 4, 4, 16, 4).mode == 2   # d <= 64, eligible prime
    assert B.pm_plan(1000000007, 4, 4, 4, 100, 4).mode == 1
    assert B.pm_plan(1000000007, 4, 4, 4, 16, 8).mode == 1   # u64: no Vandermonde route
    B.tune_load(table(glob={"vdm_max_d": 0}))
    assert B.pm_plan(1000000007, 4, 4, 4, 16, 4).mode == 1


def _fresh_process_info(env_table):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1905_04356_amd import binding as B\n"
            "print(B.tune_info(), B.pm_plan(%d, 64, 64, 32, 4096, 4).tune_entry)\n"
            % (ROOT, P31))
    env = dict(os.environ, PM_TUNE_TABLE=env_table)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    return out.stdout.strip(), out.stderr


def test_table_file_is_read_on_first_use_with_fallback(tmp_path):
    good = tmp_path / "good.json"
    good.write_text(table([{"prime_class": "direct_ge30", "knobs": {"blk_nt": 512}}]))
    out, _ = _fresh_process_info(str(good))
    assert out == "(1, 1) 0"
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "pm-tune-1", "entries": [{"knobs": {"blk_nt": 7}}]}')
    out, err = _fresh_process_info(str(bad))
    assert out == "(0, -1) -1" and "ignoring tuning table" in err
    out, _ = _fresh_process_info(str(tmp_path / "missing.json"))
    assert out == "(0, 0) -1"
    out, _ = _fresh_process_info("")                  # empty: no table at all
    assert out == "(0, 0) -1"


def test_committed_table_parses():
    """The table shipped beside libpm.so is valid (when present)."""
    path = os.path.join(ROOT, "paper_1905_04356_amd", "tune_table.json")
    if not os.path.exists(path):
        pytest.skip("no tuning table committed")
    B.tune_load(open(path).read())
    entries, source = B.tune_info()
    assert entries >= 1 and source == 2


def test_whole_length_entries_take_the_knobs_most_buckets_chose():
    from paper_1905_04356_amd.tune import common_knobs
    big = {"blk_nt": 512, "blk_tile_log": 14}
    assert common_knobs([big, big, dict(big, maxr=3), dict(big, pw_small_lds=0)]) == big
    # one bucket of four kept the defaults: 3/4 still agree
    assert common_knobs([big, big, big, {}]) == big
    # two of four: no whole-length entry
    assert common_knobs([big, big, {}, {"split": 3}]) == {}
    assert common_knobs([{"split": 3}, {"split": 3}, {"split": 3}, {"split": 2}]) == {"split": 3}
