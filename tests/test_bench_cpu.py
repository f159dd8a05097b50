"""Host-side logic of bench.py: flop and byte accounting, the choice of roofline, the stored
HBM-traffic lookup and the one-GPU guard.  CPU only."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N256 = (256, 256, 256)
KERNEL = {"precision": "fp32", "structure": "even_odd_bwd", "tile_cfg": 4, "t_loader": False,
          "prologue": "exp_euler_update_otf", "epilogue": "store"}


def test_flop_counts():
    N = 256.0 ** 3
    assert bench.mode_product_flop(N256, "dense") == 4 * 256 * N == bench.method_flop(N256)
    # even/odd: 4 (me^2 + mo^2) N / n + 2N with me = mo = 128
    assert bench.mode_product_flop(N256, "even_odd_bwd") == 4 * (2 * 128 * 128) * N / 256 + 2 * N
    # odd length: me = 4, mo = 3
    assert bench.mode_product_flop((7, 7), "even_odd_fwd") == 4 * (16 + 9) * 49 / 7 + 2 * 49


def test_byte_counts():
    N = 256.0 ** 3
    plain = dict(KERNEL, prologue="none")
    assert bench.mode_product_bytes(N256, plain, 8) == 2 * 8 * N
    assert bench.mode_product_bytes(N256, KERNEL, 8) == 4 * 8 * N
    assert bench.mode_product_bytes(N256, dict(KERNEL, prologue="exp_euler_update"), 8) == 5 * 8 * N
    assert bench.mode_product_bytes(N256, dict(plain, epilogue="exp_euler"), 16) == 4 * 16 * N


def test_roofline_choice():
    flop = bench.mode_product_flop(N256, "even_odd_bwd")
    upd = bench.roofline_of(KERNEL, flop, bench.mode_product_bytes(N256, KERNEL, 8), 0.151, "fp32")
    assert upd["bound"] == "hbm" and upd["unit"] == "GB/s"
    assert abs(upd["frac"] - 4 * 8 * 256.0 ** 3 / 0.151e-3 / 8e12) < 1e-12
    plain = dict(KERNEL, prologue="none")
    pl = bench.roofline_of(plain, flop, bench.mode_product_bytes(N256, plain, 8), 0.096, "fp32")
    assert pl["bound"] == "mfma" and pl["peak"] == 157.3
    assert 0.5 < pl["frac"] < 0.6


def test_stored_traffic_follows_the_source_hash(monkeypatch):
    value = bench.stored_traffic(KERNEL)
    if value is not None:  # present for the committed sources
        assert 0.9 * 4 * 8 * 256 ** 3 < value < 1.2 * 4 * 8 * 256 ** 3
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.stored_traffic(KERNEL) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
