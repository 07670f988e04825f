"""Host-side checks of bench.py (no GPU): the one-GPU refusal and the
algorithmic-byte formulas behind its roofline, evaluated on the benchmark
block's sizes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_bytes_of_the_benchmark_block():
    """Each input read once, each output written once, for R = 429,884,
    C = 433,816, nnz = 4,012,517, kz = 32, FP32 (and BF16 operands)."""
    import bench
    R, C, nnz, kz = 429_884, 433_816, 4_012_517, 32
    a = bench.algorithmic_bytes(R, C, nnz, kz, 4)
    # gather: gmap (8 B) + source row + packed row per id
    assert a["gather_A"] == 8 * R + 2 * 4 * kz * R == 113_489_376
    assert a["gather_B"] == 8 * C + 2 * 4 * kz * C
    # fused: row structure, indices + values + outputs, A and B rows once, Y rows once
    assert a["sddmm_spmm"] == 4 * (R + 1) + 12 * nnz + 4 * kz * (R + C) + 4 * kz * R == 215_448_496
    assert a["sddmm"] == 4 * (R + 1) + 12 * nnz + 4 * kz * (R + C)
    assert a["spmm"] == 4 * (R + 1) + 8 * nnz + 4 * kz * C + 4 * kz * R
    # scatter-reduce: gmap + packed read + owner row read and written
    assert a["scatter"] == 8 * R + 12 * kz * R == 168_514_528
    b = bench.algorithmic_bytes(R, C, nnz, kz, 2)
    assert b["gather_A"] == 8 * R + (4 + 2) * kz * R          # FP32 source, bfloat16 packed
    assert a["sddmm_spmm"] - b["sddmm_spmm"] == 2 * kz * (R + C)
    # the step total the JSON line's step fraction divides by
    step = sum(a[k] for k in ("gather_A", "gather_B", "sddmm_spmm", "scatter"))
    assert round(step / 1e6, 1) == 612.0
