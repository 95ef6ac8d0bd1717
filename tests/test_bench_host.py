"""Host-side parts of bench.py (no GPU): the committed rocprofv3 counter
summary matches the current device sources, so the benchmark's `traffic`
and ALU figures are not silently dropped, and it holds the kernels the
benchmark's default line looks up; the byte accounting of each kernel."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_counter_summary_matches_sources_and_kernels():
    rows = bench._counter_rows()
    assert rows is not None, "profiles summary missing or taken for other device sources"
    for k in ("k_cpull<64, 8, 64, false, f32, false>",
              "k_fused<64, 8, 64, 4, false, f32, false, true>",
              "k_fused<64, 8, 32, 4, false, f32, false, false>", "k_pull<f32, false, f32>"):
        t = bench.measured_traffic(k)
        assert t is not None and t > 0, k
    for k in ("k_cpull<64, 8, 64, false, f32, false>",
              "k_fused<64, 8, 64, 4, false, f32, false, true>"):
        v = bench.measured_valu(k)
        assert v is not None and v > 0, k
        # lane operations per node of a 256^3 launch: several hundred
        assert 300 < v * 64 / 256 ** 3 < 2000, (k, v)


def test_byte_accounting():
    assert bench.kernel_bytes("fp32")["pull"] == 54 * 4 + 11 * 4
    assert bench.kernel_bytes("fp16")["fused"] == 11 * 4 + 2 * 8 + 52 * 2 + 2 * 8
    assert bench.COMPACT_BYTES["pull"] == bench.COMPACT_BYTES["fused"] == 112
    assert bench.d2q9_bytes("fp32") == 144 and bench.d2q9_bytes("fp16") == 96
    assert bench.step_bytes("fp32") == 432 and bench.step_bytes("bf16") == 216
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
