"""Host-side checks of bench.py that need no GPU: the one-GPU contract, the
flop model, and the counter-summary reader."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_flop_model():
    # Step 2 of the fast algorithm: 32 m n s p real flops; FFTs: 10 p log2 p per tube of each tensor
    f_gemm, f_fft = bench.flops(1024, 1024, 1024, 32)
    assert f_gemm == 32.0 * 1024 ** 3 * 32
    assert f_fft == pytest.approx(10.0 * 32 * 5 * 3 * 1024 ** 2)
    assert bench.flops(4, 5, 6, 1)[1] == 0.0


def test_traffic_only_for_matching_fingerprint():
    fp = bench.kernel_fingerprint()
    assert len(fp) == 40
    t = bench.measured_traffic("c3", "split_bf16")
    # the committed summary records the current kernel sources, or the bench reports no traffic
    with open(bench.COUNTER_SUMMARY) as fh:
        recorded = [ln.split()[3] for ln in fh if ln.startswith("traffic_bytes_per_launch:")]
    assert (t is not None) == (fp in recorded)
    assert bench.measured_traffic("c2", "split_bf16") is None
    assert bench.measured_traffic("c3", "fp32") is None


def test_tsvd_flop_model():
    # one complex SVD of the 2r x 2c matrix per pair, half for each self-paired frequency
    one = bench.svd_flops(2 * 256, 2 * 192)
    assert one == 4.0 * (4 * 512 ** 2 * 384 + 8 * 512 * 384 ** 2 + 9 * 384 ** 3)
    assert bench.tsvd_flops(256, 192, 1) == pytest.approx(0.5 * one)
    assert bench.tsvd_flops(192, 256, 16) == pytest.approx((7 + 1.0) * one)     # pairs 1..7, f = 0 and 8
    assert bench.tsvd_flops(256, 192, 15) == pytest.approx((7 + 0.5) * one)
