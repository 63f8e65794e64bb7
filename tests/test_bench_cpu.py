"""The benchmark's host-side contract, checked without a GPU: more than one GPU is refused with a
message, the roofline byte/flop counts follow the per-point figures, and the committed
sustained peaks and traffic summaries are readable."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


@pytest.mark.parametrize("prec,es", [("fp64", 8), ("bf16x3", 4), ("fp32", 4), ("bf16", 2)])
def test_mode_stage_counts(prec, es):
    n = 256 ** 3
    N = dict(x_fwd=256, y_fwd=256, z_fwd_div=256, z_inv=256, y_inv=256, x_inv=256, x_fwd_rhs=256, z_inv_u=256)
    rl = bench.stage_roofline("y_fwd", 1.0, 1, N, n, prec)
    assert rl["algorithmic_flops"] == 2 * 256 * n                # 2N flops per point
    assert rl["algorithmic_bytes"] == 2 * es * n                 # one read and one write per point
    if prec == "bf16x3":
        rhs = bench.stage_roofline("x_fwd_rhs", 1.0, 1, N, n, prec)
        assert rhs["algorithmic_bytes"] == (8 + 4) * n            # FP64 right-hand side in, FP32 out
        # 64 flop/B is below the BF16 ridge (2500 TFLOP/s over 8 TB/s = 312.5 flop/B): HBM-bound,
        # frac = algorithmic bytes / time / 8 TB/s, and the issued MFMA work is six times the flops
        assert rl["bound"] == "hbm" and rl["peak"] == 8000.0
        assert abs(rl["achieved"] - 2 * es * n / 1e-3 / 1e9) < 1e-6 * rl["achieved"]
        assert rl["issued_flops_factor"] == 6 and abs(rl["issued_tflops"] - 6 * rl["algorithmic_tflops"]) < 1e-9


def test_streaming_stage_counts():
    n = 1000
    assert bench.stage_roofline("residual", 1.0, 1, {}, n, "bf16x3")["algorithmic_bytes"] == (4 + 8 + 4) * n
    assert bench.stage_roofline("update", 1.0, 1, {}, n, "bf16x3")["algorithmic_bytes"] == (4 + 4 + 8) * n
    assert bench.stage_roofline("residual", 1.0, 1, {}, n, "fp64")["algorithmic_bytes"] == (8 + 8 + 8) * n
    assert bench.stage_roofline("thomas", 1.0, 1, {}, n, "fp64")["algorithmic_bytes"] == 16 * n


def test_committed_peaks_and_traffic_readable():
    assert bench.sustained_peak("bf16x3", "mfma") > 0
    assert bench.sustained_peak("fp64", "mfma") > 0
    assert bench.sustained_peak("fp64", "hbm") > 0
    # the split-BF16 product contracts on the BF16 matrix cores: it is priced against the BF16
    # rate with its algorithmic flops; its six issued products per term are a separate factor
    assert bench.sustained_peak("bf16x3", "mfma") == bench.sustained_peak("bf16", "mfma")
    assert bench.MFMA_PEAK_TFLOPS["bf16x3"] == bench.MFMA_PEAK_TFLOPS["bf16"] == 2500.0
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        t = json.load(fh)
    assert t["bf16x3"]["z_fwd_div"]["bytes_per_launch"] > 0
