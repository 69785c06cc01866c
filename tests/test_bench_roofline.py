"""The benchmark's roofline arithmetic (no GPU): the algorithmic bytes per
block-window follow the staged design of the scope table (block and halo
read, block written, W; the staged block, the sum tree's build and per event
the descent and dirty paths in LDS), `frac` is the larger term and `bound`
names it, and the one-GPU bench refuses other GPU counts."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_staged_hbm_bytes():
    # 16x16 spin flip: 256 + 64 read, 256 written, 4 bytes of W
    assert bench.hbm_bytes_staged("flip", 16, 1) == 580
    # 32x32 pair events also write the halo back
    assert bench.hbm_bytes_staged("zgb", 32, 1) == 2 * (1024 + 128) + 4
    assert bench.hbm_bytes_staged("flip", 16, 1000) == 580 * 1000


def test_method_lds_bytes():
    # per block-window: staging 320, 256 leaves x 8, 255 inner nodes x 24
    assert bench.lds_bytes("flip", 16, 1, 0) == 320 + 8 * 256 + 24 * 255 == 8488
    # per event: descent 16 log2(256) = 128, five dirty paths of 8 + 24 * 8
    assert bench.lds_bytes("flip", 16, 0, 1) == 128 + 5 * 200 == 1128
    # pair events: eight dirty paths on 32x32 blocks (log2 1024 = 10)
    assert bench.lds_bytes("zgb", 32, 0, 1) == 160 + 8 * (8 + 240)


def test_resident_variant_bytes():
    # 1024^2, 16x16: lattice read and written once, 28 counter bytes per block,
    # 64 edge bytes per block-window
    assert bench.resident_bytes(16, 2000 * 2048, 1 << 20, 1) == 2 * (1 << 20) + 28 * 4096 + 64 * 2000 * 2048


class _FakeTiming:
    def __init__(self, ms, n):
        self.ms, self.n = ms, n

    def fskmc_ctx_read_kernel_timing(self, ctx):
        return self.ms, self.n


def test_frac_is_the_larger_term_and_names_it():
    obs = [{"block_windows": 4096000, "events": 4975732}]
    rl = bench.roofline(_FakeTiming(6.3, 1), None, "flip", 16, obs, 1, "k", symbol=None, resident_sites=1 << 20)
    hbm = bench.hbm_bytes_staged("flip", 16, 4096000) / 6.3e-3 / 1e9
    lds = bench.lds_bytes("flip", 16, 4096000, 4975732) / 6.3e-3 / 1e9
    assert rl["hbm"]["achieved"] == pytest.approx(hbm) and rl["lds"]["achieved"] == pytest.approx(lds)
    assert rl["bound"] == "lds" and rl["frac"] == pytest.approx(lds / bench.LDS_PEAK_GBS)
    assert rl["frac"] == max(rl["hbm"]["frac"], rl["lds"]["frac"])
    assert rl["variant"]["hbm_bytes_per_launch"] == bench.resident_bytes(16, 4096000, 1 << 20, 1)
    assert bench.LDS_PEAK_GBS == pytest.approx(78643.2) and bench.HBM_PEAK_GBS == 8000.0


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
