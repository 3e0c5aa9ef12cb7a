"""Host-side checks of bench.py: the one-GPU contract and the algorithmic byte
counts behind its roofline figures (no GPU needed)."""
import math
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_kernel_bytes_at_128_cubed():
    """Each hot kernel touches each of its arrays once: 128^3 FP64 has
    nh = 128 * 128 * 65 half-spectrum modes of 16 B and N = 128^3 reals."""
    n = (128, 128, 128)
    N = math.prod(n)
    nh = 128 * 128 * 65
    assert bench.kernel_bytes("col0_inv_scale_d", "fp64", n) == 2 * 16 * nh  # 34.1 MB
    assert bench.kernel_bytes("plane_inner", "fp64", n) == 2 * 16 * nh + 8 * N  # 50.9 MB
    assert bench.kernel_bytes("col0_fwd_update", "fp64", n) == 4 * 16 * nh  # 68.2 MB
    # FP32 spectra and Gamma' halve every term
    for k in ("col0_inv_scale_d", "plane_inner", "col0_fwd_update"):
        assert bench.kernel_bytes(k, "fp32", n) * 2 == bench.kernel_bytes(k, "fp64", n)
    # a Hessian-vector product's three passes move 40 N + 64 nh bytes in FP64,
    # three times the 24 N its method-level definition touches
    hv = sum(bench.kernel_bytes(k, "fp64", n) for k in ("plane_fwd_phys", "col0_fwd_mul_inv", "plane_inv_phys"))
    assert hv == 40 * N + 64 * nh
    assert abs(hv / (24 * N) - 3.02) < 0.01
    assert bench.kernel_bytes("not_a_kernel", "fp64", n) is None
