"""Host-side logic of bench.py (no GPU): the issue-model peaks against cycle
counts worked out by hand, the counter-summary parser and its source-hash gate,
and the refusal of several GPUs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
import bench  # noqa: E402

S = 256 * 4 * 2.4e9  # SIMD cycles per second


def test_compiled_dimensions():
    assert [bench.dpad(d) for d in (1, 2, 3, 4, 5, 7, 9, 13, 17, 33, 64)] == [1, 2, 3, 4, 6, 8, 12, 16, 24, 48, 64]


def test_product_peaks_by_hand(monkeypatch):
    monkeypatch.delenv("KRR_KMVP_VALU", raising=False)
    monkeypatch.delenv("KRR_KMVP_MG32", raising=False)
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    # FP32 d = 3, symmetric kernel: one 32x32x16 f16 op (32) + 16 x (exp2 8 + 2 FMAs 8) + 24 per
    # 1024 exponentials (2048 pair terms)
    assert bench.product_peak(3)[0] == pytest.approx(S * 2048 / (32 + 256 + 24))
    assert bench.product_peak(3)[2] == "k_kmvp_mhs<3, FP32>"
    # d = 8 (symmetric): ceil(26 / 16) = 2 f16 ops per 1024 exponentials
    assert bench.product_peak(8)[0] == pytest.approx(S * 2048 / (2 * 32 + 256 + 24))
    assert bench.product_peak(8)[2] == "k_kmvp_mhs<8, FP32>"
    # d = 12 (symmetric): ceil(38 / 16) = 3 ops
    assert bench.product_peak(12)[0] == pytest.approx(S * 2048 / (3 * 32 + 256 + 24))
    # d = 16: symmetric only with groups of 8 tiles or more (N = 2e5: 782 tiles, groups of 8)
    assert bench.sym_group_tiles(200_000) == 8 and bench.sym_group_tiles(100_000) == 4
    assert bench.product_peak(16, n=200_000)[2] == "k_kmvp_mhs<16, FP32>"
    assert bench.product_peak(16, n=200_000)[0] == pytest.approx(S * 2048 / (4 * 32 + 256 + 24))
    assert bench.product_peak(16, n=100_000)[2] == "k_kmvp_mh<16, FP32>"
    # the one-sided split-f16 kernel (d = 16, or KRR_KMVP_SYM=0): 1024 pairs per kc x 32 + 16 x 12
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    assert bench.product_peak(4)[0] == pytest.approx(S * 1024 / 224)
    assert bench.product_peak(3)[0] == pytest.approx(S * 1024 / 224)
    monkeypatch.delenv("KRR_KMVP_SYM")
    # FP32 d = 16: ceil(52 / 16) = 4 ops
    assert bench.product_peak(16)[0] == pytest.approx(S * 1024 / (4 * 32 + 192))
    # FP64 d = 3, symmetric kernel: per 1024 exponentials (2048 pair terms) four
    # 16x16x4 FP64 ops (64 each) + 16 x (9 x 4 + 2 x 4) (4096-entry table) + 24
    monkeypatch.delenv("KRR_KMVP_SYM", raising=False)
    assert bench.product_peak(3, "fp64")[0] == pytest.approx(S * 2048 / (256 + 704 + 24))
    # FP64 d = 8: the 256-entry table, 11 instructions
    assert bench.product_peak(8, "fp64")[0] == pytest.approx(S * 2048 / (4 * 3 * 64 + 16 * 52 + 24))
    # FP64 d = 16 (symmetric): five chunks of 4 over d + 1 = 17 coordinates
    assert bench.product_peak(16, "fp64")[0] == pytest.approx(S * 2048 / (4 * 5 * 64 + 16 * 52 + 24))
    # the one-sided FP64 kernel (KRR_KMVP_SYM=0): 1024 pairs per 256 + 16 x (36 + 4)
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    assert bench.product_peak(3, "fp64")[0] == pytest.approx(S * 1024 / (256 + 640))
    assert bench.product_peak(8, "fp64")[0] == pytest.approx(S * 1024 / (4 * 3 * 64 + 768))
    monkeypatch.delenv("KRR_KMVP_SYM")
    # FP32 d = 20 runs at D = 24: ceil(74 / 16) = 5 ops; d = 41 at D = 48: 10 ops
    assert bench.product_peak(20)[0] == pytest.approx(S * 1024 / (5 * 32 + 192))
    assert bench.product_peak(41, "bf16")[0] == pytest.approx(S * 1024 / (10 * 32 + 192))
    # FP64 at d = 41 runs at D = 48: 4 x 13 FP64 ops + 16 x (11 x 4 + 4)
    assert bench.product_peak(41, "fp64")[0] == pytest.approx(S * 1024 / (52 * 64 + 768))
    # FP32 beyond d = 48 runs at D = 64 on the FP32 matrix cores: 4 x 17 ops + 16 x (8 + 4)
    assert bench.product_peak(60)[0] == pytest.approx(S * 1024 / (68 * 32 + 192))
    # VALU kernel on request: 64 pairs per (d + 1) FMAs + exp2
    monkeypatch.setenv("KRR_KMVP_VALU", "1")
    assert bench.product_peak(20)[0] == pytest.approx(S * 64 / (21 * 4 + 8))
    monkeypatch.delenv("KRR_KMVP_VALU")
    monkeypatch.setenv("KRR_KMVP_MG32", "1")
    assert bench.product_peak(3)[0] == pytest.approx(S * 1024 / (4 * 32 + 192))
    # Matern d = 8, symmetric: two f16 ops + 16 x (sqrt 8 + exp2 8 + 4 FMA-class ops) + 24 per
    # 2048 terms; one-sided (KRR_KMVP_SYM=0): two f16 ops + 16 x (sqrt 8 + exp2 8 + 2 FMAs) per 1024
    monkeypatch.delenv("KRR_KMVP_MG32")
    assert bench.matern_peak(8)[0] == pytest.approx(S * 2048 / (64 + 512 + 24))
    assert bench.matern_peak(8)[2] == "k_kmvp_mhs<8, FP32, matern>"
    monkeypatch.setenv("KRR_KMVP_SYM", "0")
    assert bench.matern_peak(8)[0] == pytest.approx(S * 1024 / (64 + 384))
    monkeypatch.delenv("KRR_KMVP_SYM")
    # 16-RHS product d = 4: one 16x16x32 f16 op + 4 exp2 + four 16x16x4 FP32 ops per 4096 pair-RHS
    assert bench.multi_peak(4)[0] == pytest.approx(S * 4096 / (16 + 32 + 128))


def test_traffic_parser_and_hash_gate(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    (tmp_path / "profiles" / "c.txt").write_text("x\ntraffic: bytes_per_launch=12345 source_hash=abc\n")
    assert bench.read_traffic("c.txt") == 12345.0
    (tmp_path / "profiles" / "d.txt").write_text("traffic: bytes_per_launch=12345 source_hash=zzz\n")
    assert bench.read_traffic("d.txt") is None  # kernel changed since the counters were taken
    assert bench.read_traffic("missing.txt") is None


def test_committed_counters_match_kernel_source():
    # the committed counter summary is the one the bench line's traffic figure uses
    v = bench.read_traffic("kmvp_fp32_d3_kriging_counters.txt")
    assert v is None or v > 3.6e6  # at least the algorithmic bytes when current


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
