"""Host-only checks of the benchmark's roofline bookkeeping (no GPU): which
peak each kernel kind is priced against, and the transposes' HBM rate."""

import bench


def _prof():
    # kind: [launches, total ms, algorithmic flops, algorithmic bytes]
    return {"gemm_mfma": [10, 20.0, 1.6e12, 1e9], "gemm_split_fp16": [5, 5.0, 4e12, 2e9],
            "transpose": [14, 6.0, 0.0, 3.15e10]}


def test_fp32_kind_in_a_split_program_is_priced_at_the_fp32_peak():
    r = bench._roofline(_prof(), "split_fp16", "none")
    assert r["kernel"] == "gemm_mfma" and r["bound"] == "mfma"
    assert r["peak"] == bench.PEAK_FP32_TFLOPS
    assert abs(r["achieved"] - 1.6e12 / 20e-3 / 1e12) < 1e-9  # 80 TFLOP/s, one product per algorithmic one
    assert abs(r["frac"] - 80.0 / bench.PEAK_FP32_TFLOPS) < 1e-12


def test_split_kind_counts_three_hardware_products_at_the_16bit_peak():
    prof = _prof()
    prof["gemm_split_fp16"][1] = 50.0  # now the dominant kind
    r = bench._roofline(prof, "split_fp16", "none")
    assert r["kernel"] == "gemm_split_fp16" and r["bound"] == "mfma"
    assert r["peak"] == bench.PEAK_MFMA_TFLOPS["split_fp16"]
    assert abs(r["achieved"] - 3 * 4e12 / 50e-3 / 1e12) < 1e-9


def test_hbm_bound_kind_reports_bytes():
    # Few flops over many bytes: HBM-bound, achieved in GB/s against 8 TB/s.
    r = bench._roofline({"gemm_mfma": [1, 1.0, 1e6, 4e9]}, "c64", "none")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.PEAK_HBM_GBS
    assert abs(r["achieved"] - 4e9 / 1e-3 / 1e9) < 1e-6


def test_transpose_hbm_rate():
    t = bench._hbm_kind(_prof(), "transpose")
    assert t["bound"] == "hbm" and t["launches"] == 14
    assert abs(t["achieved"] - 3.15e10 / 6e-3 / 1e9) < 1e-6
    assert abs(t["frac"] - t["achieved"] / 8000.0) < 1e-12
    assert bench._hbm_kind(_prof(), "gemm_rows") is None
