"""Host-side tools of bench.py: algorithmic byte counts, the code hash that
ties counter summaries to the kernels, and the committed traffic summary
(no GPU)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_pass_bytes_per_velocity_node():
    # 9 plane-set passes (read 1 + write 1, read 2 + write 2, read 2 + write 1)
    # and 7 FP64 moment-set passes of 4 fields over 128 planes
    cells = 1000
    for elem, per_vn in ((8, 9 * 8 + 7 * 4 * 8 / 128), (4, 9 * 4 + 7 * 4 * 8 / 128)):
        pb = bench.pass_bytes(128, cells, elem, 4)
        assert abs(sum(pb.values()) / (128 * cells) - per_vn) < 1e-12
        assert pb["stage4"] > pb["stage5"] > pb["stage3"]


def test_code_hash_ignores_comments_only():
    src = "int f(int x) {  // one\n    /* two\n       lines */\n    return x + 1;\n}\n"
    same = "// header\nint f(int x) {\n    return x + 1;   \n}\n\n"
    other = "int f(int x) {\n    return x + 2;\n}\n"
    strip = bench._strip_comments
    assert strip(src) == strip(same)
    assert strip(src) != strip(other)


def test_committed_traffic_summary_matches_the_kernels():
    t = bench.read_traffic(4096)
    if not t:
        pytest.skip("the traffic summary was taken on other kernel code")
    assert set(t) == {f"{p} stage{k}" for p in ("f64", "f32") for k in (3, 4, 5)}
    for key, traffic in t.items():
        prec, stage = key.split()
        alg = bench.pass_bytes(128, 4096 * 4096, 8 if prec == "f64" else 4, 4)[stage]
        assert 1.0 <= traffic / alg < 2.0, (key, traffic / alg)
    assert bench.read_traffic(1024) == {}


def test_valu_peak_from_unit_counts():
    # 256 CUs x 4 SIMDs x 16 lanes per cycle at 2.4 GHz
    assert abs(bench.VALU_PEAK_T - 39.3216) < 1e-9


def test_committed_instruction_mix_matches_the_kernels():
    v = bench.read_valu_per_vn(4096)
    if not v:
        pytest.skip("the instruction-mix summary was taken on other kernel code")
    assert set(v) == {f"{p} stage{k}" for p in ("f64", "f32") for k in (3, 4, 5)}
    # tens of lane-instructions per velocity node; stage 4 (two outputs, E^n
    # at the own cells) the most
    for prec in ("f64", "f32"):
        assert 50 < v[f"{prec} stage3"] < v[f"{prec} stage4"] < 200
    assert bench.read_valu_per_vn(1024) == {}
