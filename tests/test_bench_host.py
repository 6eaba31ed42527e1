"""Host logic of bench.py (no GPU): the refusal of more than one GPU, the algorithmic byte table,
the LDS-atomic floor of the deposition and the gating of the recorded HBM traffic on the kernel
sources."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_algorithmic_bytes():
    N, M, Np, s = 8 * 8 * 8, 8 * 8 * 5, 100, 4
    assert bench.stage_bytes("psatd_update", N, M, Np, s) == 39 * s * M  # 11 spectra + 5 tables in, 6 out
    assert bench.stage_bytes("deposit_reduce", N, M, Np, s) == 5 * N * s
    assert bench.stage_bytes("clear_sources", N, M, Np, s) == 0
    assert bench.stage_bytes("fft_inverse", N, M, Np, s) == 6 * (2 * s * M + s * N)


def test_lds_atomic_floor():
    # cubic FP32: 64 64-bit and 128 32-bit lane operations per particle on each of 256 CUs
    r32, r64 = 14.5 * 2.4e9, 9.9 * 2.4e9
    per_cu = 1000
    expected = per_cu * (64 / r64 + 128 / r32) * 1e3
    assert bench.deposit_lds_floor_ms(256 * per_cu, 3, "f32", r32, r64) == pytest.approx(expected)
    # FP64 (CIC): four 64-bit words per node, 8 nodes
    assert bench.deposit_lds_floor_ms(256, 1, "f64", r32, r64) == pytest.approx(32 / r64 * 1e3)


def test_recorded_traffic_is_gated_on_the_kernel_sources(monkeypatch):
    v = bench.recorded_traffic("deposit")
    assert v is None or v > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.recorded_traffic("deposit") is None
    assert bench.recorded_traffic("deposit", "laser128") is None


def test_checkpoint_interval_of_the_reverse_mode():
    """The forward+backward legs store every step's state when the states fit the memory given to
    them (nothing is recomputed), else take the smallest interval whose checkpoints and one
    recomputed segment fit."""
    from types import SimpleNamespace

    from paper_2106_12919_amd import autograd as pag

    pic = SimpleNamespace(shape=(64, 64, 128), dtype="f32")
    n = 2_097_152
    s = pag.state_bytes(pic, n)
    assert s == 7 * 64 * 64 * 128 * 4 + 4 * n + 6 * n * 4  # n is a multiple of 64: no row padding
    # 60 steps: k = 1 holds 60 states; k > 1 holds ceil(60 / k) + k + 1 (2: 33, 3: 24, 4: 20, 6: 17)
    assert pag.checkpoint_interval(pic, n, 60, 60 * s) == 1
    assert pag.checkpoint_interval(pic, n, 60, 59 * s) == 2
    assert pag.checkpoint_interval(pic, n, 60, 20 * s) == 4
    assert pag.checkpoint_interval(pic, n, 60, 16 * s) == 6  # none fits: the fewest held (17, first at k = 6)
    assert pag.checkpoint_interval(SimpleNamespace(shape=(8, 8, 8), dtype="f64"), 100, 5, 1e12) == 1
