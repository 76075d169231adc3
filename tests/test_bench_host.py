"""Host-side pieces of bench.py (no GPU): the refusal of several GPUs, the
roofline arithmetic and the gating of committed traffic figures on the
device-source hash."""
import os
import subprocess
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_peaks():
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz, without and with packed FP32
    assert abs(bench.PEAK_VALU_NONPACKED_TFLOPS - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.05
    assert abs(bench.PEAK_FP32_TFLOPS - 2 * bench.PEAK_VALU_NONPACKED_TFLOPS) < 0.2


def test_default_line_is_the_largest_configuration():
    assert bench.HEADLINE == "config5"
    assert set(bench.BESIDE) == {"config4", "config2"}
    # bytes per eval of the d = 116 and d = 50 mixed-precision rows: x in FP32, y, the index
    assert bench.algorithmic_bytes_per_eval(116, True) == 472
    assert bench.algorithmic_bytes_per_eval(50, True) == 208


class _W:
    """The fields of a workload that the roofline reads."""
    def __init__(self, d, M, m, L, name):
        self.d, self.M, self.m, self.L, self.name = d, M, m, L, name


def test_roofline_resident_is_alu_bound():
    w = _W(20, 2048, 5000, 20, "poisson_n1e6_d20_fp32data")
    r = bench.roofline(w, True, 1.0, bench.MOVE_RESIDENT)
    evals = 2048 * 5000 * 21
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["flops_per_eval"] == 8 * 20 and r["evals_per_launch"] == evals
    assert abs(r["achieved"] - 160 * evals / 1e-3 / 1e12) < 0.01
    assert r["peak"] == 157.3
    assert abs(r["frac"] - r["achieved"] / bench.PEAK_FP32_TFLOPS) < 1e-3
    assert abs(r["frac_of_nonpacked_fp32_peak"] - r["achieved"] / 78.6) < 1e-3


def test_roofline_streaming_is_hbm_bound():
    w = _W(20, 2048, 5000, 20, "poisson_n1e6_d20_fp32data")
    r = bench.roofline(w, False, 2.0, bench.MOVE_STREAMING)
    evals = 2048 * 5000 * 21
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    # x (d values), y and the 4-byte index per eval, in doubles
    assert r["bytes_per_eval"] == 20 * 8 + 8 + 4
    assert abs(r["achieved"] - 172 * evals / 2e-3 / 1e9) < 0.1


def test_traffic_only_for_current_sources(tmp_path, monkeypatch):
    w = _W(20, 2048, 5000, 20, "poisson_n1e6_d20_fp32data")
    prof = tmp_path / "profiles"
    prof.mkdir()
    f = prof / "move_kernel_res_poisson_n1e6_d20_fp32data_mixed_traffic.txt"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "device_source_hash", lambda kernel: "abc")
    f.write_text("# header\ndevice_source_sha256 abc\ntraffic_bytes_per_launch 1234\n")
    assert bench.measured_traffic(w, "mixed", "move_kernel_res") == 1234.0
    # the a = 1 state's moves have a figure of their own, or none
    assert bench.measured_traffic(w, "mixed", "move_kernel_res", "a1") is None
    f.write_text("# header\ndevice_source_sha256 abc\ntraffic_bytes_per_launch 1234\n"
                 "traffic_bytes_per_launch_a1 5678\n")
    assert bench.measured_traffic(w, "mixed", "move_kernel_res") == 1234.0
    assert bench.measured_traffic(w, "mixed", "move_kernel_res", "a1") == 5678.0
    f.write_text("# header\ndevice_source_sha256 old\ntraffic_bytes_per_launch 1234\n")
    assert bench.measured_traffic(w, "mixed", "move_kernel_res") is None
    assert bench.measured_traffic(w, "fp64", "move_kernel") is None
    # each kernel's summary follows its own sources
    assert set(bench.DEVICE_SOURCES) >= {"move_kernel", "move_kernel_wide", "move_kernel_res"}
    assert "kernels_resident.hpp" not in bench.DEVICE_SOURCES["move_kernel_wide"]
