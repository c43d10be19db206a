"""Host-side checks of the benchmark's contract (no GPU): one GPU only, and
the algorithmic byte / flop models it reports against."""
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_models_at_32_qubits():
    sys.path.insert(0, ROOT)
    import bench
    m = bench.model(16, 8, 8, 94849, 39960)
    assert m["dim"] == math.comb(16, 8) ** 2
    # gather model: (nnz + dim) 8 + 16 T bytes, 7.678 TB at 32 qubits
    assert abs(bench.hpsi_gather_bytes(m) / 1e12 - 7.678) < 0.01
    # the mixed pass: 2 flops per product, s_a s_b + s_a + s_b + 1 products per output
    flops, bound = bench.kernel_flops("k_mixed", m)
    assert bound == "alu" and abs(flops - 2 * m["dim"] * (64 * 64 + 64 + 64 + 1)) < 1
    r = bench.roofline("k_mixed", 218.0, m)
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-3
    assert abs(r["lds"]["achieved"] - flops / 2 * 16 / 0.218 / 1e12) < 0.05
    assert abs(bench.LDS_PEAK_TBS - 78.6432) < 1e-3
    # the same products on the FP64 matrix cores: same flops, bound by the
    # matrix peak (equal to the vector peak on this chip), no LDS-per-product figure
    f_m, b_m = bench.kernel_flops("k_mixed_m", m)
    assert b_m == "mfma" and f_m == flops
    r = bench.roofline("k_mixed_m", 76.8, m)
    assert r["bound"] == "mfma" and "lds" not in r and abs(r["achieved"] - flops / 0.0768 / 1e12) < 0.01
    # the transition values: 2 flops per (target, source) product, s_a + s_b (s_a + 1) per amplitude,
    # on the matrix cores or the vector ALU (1.40 TFLOP at 32 qubits either way)
    f_t, b_t = bench.kernel_flops("k_tdens_m", m)
    f_r, b_r = bench.kernel_flops("k_tdens_rows", m)
    assert b_t == "mfma" and b_r == "alu" and f_t == f_r
    assert abs(f_t - 2 * m["dim"] * (64 + 64 * 65)) < 1 and abs(f_t / 1e12 - 1.40) < 0.01
