"""CPU checks of bench.py's host logic: the one-GPU refusal, the algorithmic
work model of the dominant kernels and the staleness check of the
counter-measured traffic."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "one MI355X" in r.stderr


def test_algorithmic_work_model():
    """T255, 64 states: FLOPs 2 (nlat/2) sum_m (M-m+2) columns, bytes as
    counted in the kernels' design (table once, operands and results once)."""
    import bench
    nrows = (bench.M + 1) * (bench.M + 4) // 2
    f_syn, b_syn = bench.algorithmic_work("legendre_synth", 64)
    assert f_syn == 2.0 * (bench.NLAT // 2) * nrows * 12 * 64
    assert f_syn == pytest.approx(9.78e9, rel=1e-3)
    f_ana, _ = bench.algorithmic_work("legendre_anal", 64)
    assert f_ana == pytest.approx(6.52e9, rel=1e-3)
    f_ring, b_ring = bench.algorithmic_work("ring_tendency", 64)
    assert f_ring == 0.0 and b_ring == pytest.approx(1.007e9, rel=1e-3)
    # the mixed modes move 4-byte values
    assert bench.algorithmic_work("ring_tendency", 64, 1)[1] == pytest.approx(b_ring / 2)


def test_measured_traffic_goes_stale(monkeypatch):
    """Counter figures are reported only for the sources they were taken on."""
    import bench
    key = ("ring_tendency", 0)
    byts, srcs = bench.MEASURED_TRAFFIC[key]
    fresh = bench.measured_traffic(*key)
    assert fresh in (None, byts)
    stale = dict(srcs)
    stale[next(iter(stale))] = "0" * 16
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, key, (byts, stale))
    assert bench.measured_traffic(*key) is None
    assert bench.measured_traffic("no_such_kernel") is None
