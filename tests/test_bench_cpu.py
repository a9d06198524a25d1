"""CPU: the arithmetic behind bench.py's JSON line (algorithmic bytes, the
roofline fraction, the certificate tally) and its refusal of several GPUs,
checked against values worked out by hand."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1802_08557_amd import workloads as W  # noqa: E402


def two_lps():
    # LP 0: 3 x 2, rows <=, <=, >= (b > 0): one surplus column.
    # LP 1: 2 x 2, rows <= with b < 0 (flips to >=) and >= with b < 0 (flips to <=).
    A = np.ones(3 * 2 + 2 * 2)
    b = np.array([1.0, 2.0, 3.0, -1.0, -2.0])
    c = np.ones(4)
    sense = np.array([0, 0, 1, 0, 1], np.int8)
    return W.Batch(A, b, c, sense, np.array([3, 2], np.int32), np.array([2, 2], np.int32))


def test_surplus_columns_follow_sign_normalisation():
    assert bench.surplus_columns(two_lps()).tolist() == [1, 1]


def test_algorithmic_bytes_by_placement():
    bt = two_lps()
    stats = np.zeros((2, 8), np.int32)
    stats[0, 0], stats[0, 1], stats[0, 6] = 1, 2, 1  # 3 pivots, wavefront kernel (LDS)
    stats[1, 1], stats[1, 6] = 4, 2                  # 4 pivots, device-memory slot
    lds, hbm, io, piv = bench.algorithmic_bytes(bt, stats, 8)
    # LP 0: m x N = 3 x 3 cells, built once and read + written per pivot.
    assert lds == 8 * 9 * (1 + 2 * 3)
    # LP 1: (m + 1) x (N + 1) = 3 x 4 cells in device memory, plus the inputs
    # and outputs of both LPs.
    io_want = sum(8 * (m * n + m + n) + m + 8 * n + 8 + 4 + 32 for m, n in ((3, 2), (2, 2)))
    assert io == io_want
    assert hbm == 8 * 12 * (1 + 2 * 4) + io_want
    assert piv == 3.5


def test_roofline_fraction_and_bound():
    peaks = {"lds_read_write": 70e12, "lds_read": 120e12}
    r = bench.roofline({"k": 2.0}, "k", 7e10, 1e9, peaks, "no-such-workload")
    assert r["bound"] == "lds"
    assert r["achieved"] == pytest.approx(7e10 / 2e-3 / 1e9)
    assert r["frac"] == pytest.approx(7e10 / 2e-3 / 70e12)
    assert r["lds_frac_vs_read_peak"] == pytest.approx(7e10 / 2e-3 / 120e12)
    assert r["traffic"] is None  # no counters for this workload
    r = bench.roofline({"k": 1.0}, "k", 1e9, 4e9, peaks, "no-such-workload")
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(4e9 / 1e-3 / 8e12)


def test_certified_count():
    stats = np.zeros((6, 8), np.int32)
    stats[:, 5] = [3, 1, 4, 16, 8, 0]  # optimal, primal only, ray, Phase I, singular, none
    assert bench.certified_count(stats) == 3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
