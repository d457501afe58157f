"""Host logic of the autotuner's variant choice and of the bench's profile
lookup (no GPU: only the decision rules are exercised)."""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1902_08318_amd import tune  # noqa: E402


def _samples(**by_name):
    return {name: {"batch": list(b), "single": list(s)} for name, (b, s) in by_name.items()}


BASE = ([100, 101, 99, 100, 102, 100, 101], [150, 151, 149, 150, 152, 150, 151])


def test_default_kept_when_no_variant_is_clearly_faster():
    s = _samples(default=BASE, naive_classify=([120] * 7, [170] * 7),
                 xor_loop=([99, 100, 98, 99, 100, 99, 99], [149] * 7), direct_flatten=([130] * 7, [200] * 7))
    name, reason = tune.choose_variant(s)
    assert name == "default" and "no variant" in reason


def test_win_on_one_workload_only_is_not_enough():
    s = _samples(default=BASE, naive_classify=([80] * 7, [160] * 7), xor_loop=([110] * 7, [160] * 7),
                 direct_flatten=([130] * 7, [200] * 7))
    assert tune.choose_variant(s)[0] == "default"


def test_win_within_the_spread_is_not_enough():
    # median 5% faster, but one round time overlaps the default's fastest round
    s = _samples(default=BASE, naive_classify=([95, 95, 95, 95, 95, 95, 99.5], [142] * 7),
                 xor_loop=([120] * 7, [170] * 7), direct_flatten=([130] * 7, [200] * 7))
    assert tune.choose_variant(s)[0] == "default"


def test_clear_win_on_every_workload_is_taken():
    s = _samples(default=BASE, naive_classify=([120] * 7, [170] * 7), xor_loop=([90] * 7, [135] * 7),
                 direct_flatten=([130] * 7, [200] * 7))
    name, reason = tune.choose_variant(s)
    assert name == "xor_loop" and "xor_loop" in reason


def test_fastest_of_several_winners():
    s = _samples(default=BASE, naive_classify=([95, 94, 95, 95, 95, 95, 95], [140] * 7),
                 xor_loop=([90] * 7, [135] * 7), direct_flatten=([130] * 7, [200] * 7))
    assert tune.choose_variant(s)[0] == "xor_loop"


def test_profile_lookup_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_hash()
    prof = tmp_path / "p.md"
    prof.write_text(f"sha256[:16]: `{h}`\ntraffic_bytes_per_launch (variant default): 123\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.profiled_traffic("default") == 123
    assert bench.profiled_traffic("xor_loop") is None
    prof.write_text("sha256[:16]: `0123456789abcdef`\ntraffic_bytes_per_launch (variant default): 123\n")
    assert bench.profiled_traffic("default") is None
