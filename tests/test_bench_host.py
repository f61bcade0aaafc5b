"""Host-side logic of bench.py (no GPU): the one-GPU guard, the roofline arithmetic and the
counter-traffic lookup that is tied to the GEMM source it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _stats(launches, ms, flops, byts):
    return {"timed_launches": launches, "timed_ms": ms, "timed_flops": flops,
            "timed_bytes": byts}


def test_roofline_arithmetic():
    # 100 launches in 10 ms with 1e9 flops in all: 1e7 flops per 100 us = 0.1 TFLOP/s
    roof = bench._roof("gemm", _stats(100, 10.0, 1e9, 5e8), 1.0)
    assert roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    assert roof["avg_launch_us"] == pytest.approx(100.0)
    assert roof["achieved"] == pytest.approx(0.1)
    assert roof["peak"] == bench.PEAK_FP64_MFMA_TFLOPS
    assert roof["frac"] == pytest.approx(0.1 / bench.PEAK_FP64_MFMA_TFLOPS)
    assert roof["alg_flops_per_launch"] == pytest.approx(1e7)
    assert roof["alg_bytes_per_launch"] == pytest.approx(5e6)
    assert roof["traffic"] is None
    f32 = bench._roof("gemm", _stats(100, 10.0, 1e9, 5e8), 1.0, fp32=True, traffic=123.0)
    assert f32["peak"] == bench.PEAK_FP32_MFMA_TFLOPS and f32["traffic"] == 123.0
    assert bench._roof("gemm", _stats(0, 0.0, 0.0, 0.0), 1.0) is None
    # the Householder family: vector ALU, FP32 peak in the FP32 form
    qr = bench._roof("tsqr_qr", _stats(10, 1.0, 1e8, 1e7), 1.0, fp32=True)
    assert qr["bound"] == "alu" and qr["peak"] == bench.PEAK_FP32_VECTOR_TFLOPS
    assert bench._roof("tsqr_qr", _stats(10, 1.0, 1e8, 1e7), 1.0)["peak"] == \
        bench.PEAK_FP64_VECTOR_TFLOPS


def test_step_roofline_arithmetic():
    # 3e12 flops and 2e11 bytes per step in 2 s: 1.5 TFLOP/s and 100 GB/s
    r = bench._step_roof(3e12, 2e11, 2.0, fp32=True)
    assert r["achieved"] == pytest.approx(1.5) and r["peak"] == bench.PEAK_FP32_MFMA_TFLOPS
    assert r["frac"] == pytest.approx(1.5 / bench.PEAK_FP32_MFMA_TFLOPS)
    assert r["hbm_achieved_gbs"] == pytest.approx(100.0)
    assert r["hbm_frac"] == pytest.approx(100.0 / bench.PEAK_HBM_GBS)
    assert bench._step_roof(3e12, 2e11, 2.0, fp32=False)["peak"] == bench.PEAK_FP64_MFMA_TFLOPS


def test_traffic_follows_the_gemm_source(tmp_path, monkeypatch):
    """The counter traffic is reported only while the GEMM source hashes to the value recorded
    with the counters (a summary written for the current source is read back; any change of
    the source makes it null)."""
    import hashlib
    sha = hashlib.sha256(open(bench.GEMM_SOURCE, "rb").read()).hexdigest()
    summary = tmp_path / "traffic.txt"
    summary.write_text(f"# counters\nbytes_per_launch: 12345678\nsource_sha256: {sha}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(summary))
    assert bench._gemm_traffic() == pytest.approx(12345678.0)
    other = tmp_path / "gemm.hip"
    other.write_text(open(bench.GEMM_SOURCE).read() + "\n// changed\n")
    monkeypatch.setattr(bench, "GEMM_SOURCE", str(other))
    assert bench._gemm_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench._gemm_traffic() is None
