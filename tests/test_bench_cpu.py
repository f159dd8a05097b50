"""Host-side logic of bench.py: flop and byte accounting, the choice of roofline, the stored
HBM-traffic lookup and the one-GPU guard.  CPU only."""
import json
import os
import subprocess
import sys

import numpy as np
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


def test_temporal_error_estimate():
    """Richardson estimate on synthetic samples of a first-order trajectory: u_tau = u* + c tau."""
    rng = np.random.default_rng(0)
    idx = np.arange(64)
    ustar = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    c = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    tau = 1e-3
    g = {k: {"idx": idx, "val": ustar + c * tau / k, "tau": tau / k} for k in (1, 2, 4)}
    t = bench.temporal_error(g[1], g[2], g[4])
    exact = np.linalg.norm(c * tau)
    assert abs(t["rel_l2"] - exact / np.linalg.norm(g[2]["val"])) < 1e-12
    assert abs(t["successive_difference_ratio"] - 2.0) < 1e-12
    assert abs(t["rel_l2_vs_extrapolated"] - exact / np.linalg.norm(ustar)) < 1e-12
    assert bench.temporal_error(g[1], {"idx": idx[::-1], "val": g[2]["val"]}) is None


def test_equal_accuracy_selection():
    v = {"fp64": {"steps_per_s": 100.0, "rel_l2_vs_fp64_oracle_at_T": 1e-14},
         "fp32": {"steps_per_s": 180.0, "rel_l2_vs_fp64_oracle_at_T": 3e-7},
         "bf16x3": {"steps_per_s": 200.0, "rel_l2_vs_fp64_oracle_at_T": 8e-6}}
    sp = bench.equal_accuracy(v, {"rel_l2": 1e-5})
    assert sp == {"fp64": 1.0, "fp32": 1.8}
    assert bench.equal_accuracy(v, None) is None
