"""Host logic of bench.py's measurement (no GPU): the algorithmic work per step and
per update, and the rule that a committed counter summary counts only while the
kernel source it was taken on is unchanged."""
import hashlib
import os

import pytest

import bench


def test_step_work_formulas():
    M = N = 512
    # each column of W (and V) read and written once, complex128
    assert bench.step_bytes(M, N) == 2 * 16 * (M * N + N * N)
    assert bench.step_bytes(M, N, jvec=0) == 2 * 16 * M * N
    # a sweep of N/8 - 1 steps does the scalar one-sided Jacobi's J(M, N) flops
    J = N * (N - 1) / 2 * (28 * M + 20 * N)
    assert bench.step_flops(M, N) * (N // 8 - 1) == pytest.approx(J, rel=1e-15)
    assert bench.step_flops(M, N) == pytest.approx(bench.jacobi_flops(M, N) / (N // 8 - 1), rel=1e-15)
    assert bench.step_flops(M, N, jvec=0) * (N // 8 - 1) == pytest.approx(N * (N - 1) / 2 * 28 * M, rel=1e-15)


def test_work_at_s_ref():
    # 2-site update at a = b = c = k = 256 with 10 sweeps: 32abc + 128ac + 10 J(2a, 2c) + 32ack
    a = b = c = k = 256
    J = (2 * c) * (2 * c - 1) / 2 * (28 * 2 * a + 20 * 2 * c)
    F = 32 * a * b * c + 128 * a * c + 10 * J + 32 * a * c * k
    w = bench.work_at_s_ref(100.0)
    assert w["flops_per_update"] == pytest.approx(F, rel=1e-15)
    assert w["achieved"] == pytest.approx(100.0 * F / 1e12, rel=1e-15)
    assert w["frac"] == pytest.approx(100.0 * F / bench.PEAK_FP64, rel=1e-15)


def test_counter_summary_hash_rule(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    summary = tmp_path / "summary.md"
    summary.write_text(f"# figures\n\nbytes_per_update_step: 1234\nkernels_hip_sha256: {digest}\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.measured(str(summary), "bytes_per_update_step") == 1234.0
    src.write_text("// kernel source, changed\n")
    assert bench.measured(str(summary), "bytes_per_update_step") is None
    assert bench.measured(str(tmp_path / "missing.md"), "bytes_per_update_step") is None


def test_committed_summaries_name_their_figures():
    for name, key in (("jacobi_step_chi256_dd_traffic.md", "bytes_per_update_step"),
                      ("jacobi_step_chi256_dd_fp64_ops.md", "fp64_flops_per_update_step")):
        text = open(os.path.join(bench.ROOT, "profiles", name)).read()
        assert f"{key}:" in text and "kernels_hip_sha256:" in text and "rocprofv3 --pmc" in text


def test_update_bytes():
    # 16 (2ab + 2bc + 2ak + 2kc) + 8a + 256 at a = b = c = k = 256: about 8.4 MB, x2 dd
    a = 256
    assert bench.update_bytes(a, False) == 16 * 8 * a * a + 8 * a + 256
    assert bench.update_bytes(a, True) == 2 * bench.update_bytes(a, False)
    assert 8.3e6 < bench.update_bytes(a, False) < 8.5e6


def test_roofline_totals(monkeypatch):
    # 46 updates x 11 sweeps of 63 steps in 145 ms over 3276 step launches, 20 updates/s
    monkeypatch.setattr(bench, "measured", lambda path, key: None)
    res = {"ktimes": {"jacobi": (145.0, 3276)}, "slot_sweeps": 46 * 11, "mean_sweeps": 11.0, "rate": 20.0}
    r = bench.roofline(res, 1, True)
    usteps = 46 * 11 * 63
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["flops_per_launch"] == pytest.approx(usteps * bench.step_flops(512, 512) / 3276, rel=1e-15)
    assert r["achieved"] == pytest.approx(usteps * bench.step_flops(512, 512) / 0.145 / 1e12, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] * 1e12 / bench.PEAK_FP64, rel=1e-12)
    assert r["avg_launch_us"] == pytest.approx(145e3 / 3276, rel=1e-12)
    assert r["traffic"] is None and r["executed"] is None
    assert r["hbm_algorithmic"]["achieved_GBps"] == pytest.approx(20.0 * bench.update_bytes(256, True) / 1e9)
    # counter figures per update-step scale to launches and to whole updates
    monkeypatch.setattr(bench, "measured", lambda path, key: 1e6 if "traffic" in path else 7e7)
    r = bench.roofline(res, 1, True)
    assert r["traffic"] == pytest.approx(1e6 * usteps / 3276, rel=1e-12)
    assert r["traffic_per_update"]["bytes"] == pytest.approx(1e6 * 11 * 63, rel=1e-12)
    assert r["executed"]["achieved"] == pytest.approx(7e7 * usteps / 0.145 / 1e12, rel=1e-12)
    assert bench.roofline({"ktimes": {"jacobi": (0.0, 0)}, "slot_sweeps": 0}, 1, True) is None
