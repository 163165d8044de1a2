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
    for name, key in (("jacobi_step_chi256_traffic.md", "bytes_per_update_step"),
                      ("jacobi_step_chi256_fp64_ops.md", "fp64_flops_per_update_step")):
        text = open(os.path.join(bench.ROOT, "profiles", name)).read()
        assert f"{key}:" in text and "kernels_hip_sha256:" in text and "rocprofv3 --pmc" in text


def test_roofline_totals():
    # 46 updates x 11 sweeps of 63 steps in 145 ms over 3276 step launches
    res = {"ktimes": {"jacobi": (145.0, 3276)}, "slot_sweeps": 46 * 11}
    r = bench.roofline(res, 1)
    usteps = 46 * 11 * 63
    assert r["bytes_per_launch"] == pytest.approx(usteps * bench.step_bytes(512, 512) / 3276, rel=1e-15)
    assert r["achieved"] == pytest.approx(usteps * bench.step_bytes(512, 512) / 0.145 / 1e9, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] * 1e9 / bench.PEAK_HBM, rel=1e-12)
    assert r["avg_launch_us"] == pytest.approx(145e3 / 3276, rel=1e-12)
    assert bench.roofline({"ktimes": {"jacobi": (0.0, 0)}, "slot_sweeps": 0}, 1) is None
