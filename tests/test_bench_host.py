"""Host-side logic of bench.py (CPU only): the roofline numerators and the one-GPU contract."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class _Desc:
    """The plan description of the MORFEO-like geometry: 6 laser + 3 natural stars, L = 9, M = 256."""
    M, J, L, groups = 256, 9, 9, 2
    group_size = (6, 3)
    B_complex_per_group = (129 * 256 * 9 * 6, 129 * 256 * 9 * 3)


def test_algorithmic_bytes_of_the_morfeo_step():
    ab = bench.algorithmic_bytes(_Desc, 69, 64)
    wf, out = 9 * 69 * 69 * 4, 9 * 256 * 256 * 4            # wavefronts in, layers out per frame
    B = (6 + 3) * 9 * 129 * 256 * 8                          # both groups' B, FP32 complex, read once
    assert (wf, out, B) == (171_396, 2_359_296, 21_399_552)
    assert ab["step"] == 64 * (wf + out) + B == 183_363_840
    assert ab["per_kernel"]["rows"] == 64 * wf
    assert ab["per_kernel"]["cols"] == 6 * 9 * 129 * 256 * 8
    assert ab["per_kernel"]["out"] == 64 * out + 9 * 6 * 256 * 256 * 4


def test_algorithmic_flops_follow_the_table_1_model():
    af = bench.algorithmic_flops(_Desc, 1)
    fft = 2.5 * 256 * 256 * 16                               # benchFFT: 2.5 N log2 N, N = M^2
    fwd, inv, app = 9 * fft, 2 * 9 * fft, 8 * 9 * 9 * 129 * 256
    assert abs(af["step"] - (fwd + inv + app)) < 1.0
    assert abs(af["step"] - 92.18e6) < 0.01e6
    assert abs(sum(af["per_kernel"].values()) - af["step"]) < 1.0


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
