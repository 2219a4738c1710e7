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
    B_lgs = 128 * 256 * 9 * 6 * 8                            # laser group's FP32 B, columns below Nyquist
    basis = 9 * 6 * 256 * 256 * 4                            # natural-star basis images, FP32
    assert (wf, out, B_lgs, basis) == (171_396, 2_359_296, 14_155_776, 14_155_776)
    assert ab["per_kernel"] == {"rows": 64 * wf, "cols": B_lgs, "out": 64 * out + basis}
    assert ab["step"] == 64 * (wf + out) + B_lgs + basis
    # the paper's algorithm: both groups' B over the half spectrum instead of the basis images
    assert ab["method_step"] == 64 * (wf + out) + (6 + 3) * 9 * 129 * 256 * 8 == 183_363_840


def test_flops_credit_each_kernel_with_the_work_it_performs():
    af = bench.algorithmic_flops(_Desc, 69, 1)
    c1 = 5 * 256 * 8                                         # benchFFT, complex 256-point transform
    rows = 6 * 35 * c1 + 6 * 9 * 69 * 69                     # 35 packed row pairs per laser star + moments
    cols = (6 + 9) * 128 * c1 + 8 * 9 * 6 * 128 * 256 + 8 * 6 * 128 * 256
    out = 9 * 128 * c1 + 2 * 6 * 9 * 256 * 256              # C2R rows + 6 basis multiply-adds per pixel
    assert (rows, cols, out) == (2_407_494, 35_389_440, 18_874_368)
    assert {k: round(v) for k, v in af["per_kernel"].items()} == {"rows": rows, "cols": cols, "out": out}
    assert abs(af["step"] - (rows + cols + out)) < 1.0
    # Table 1 for the whole method: 9 forward + 2 x 9 inverse real 2-D transforms + the apply
    fft = 2.5 * 256 * 256 * 16
    assert abs(af["method_step"] - (9 * fft + 2 * 9 * fft + 8 * 9 * 9 * 129 * 256)) < 1.0
    assert abs(af["method_step"] - 92.18e6) < 0.01e6
    # the 64-frame column pass: 2.265 GFLOP
    assert abs(bench.algorithmic_flops(_Desc, 69, 64)["per_kernel"]["cols"] - 2.2649e9) < 1e5


def test_single_kind_asterism_transforms_every_star():
    class D:
        M, J, L, groups = 64, 4, 2, 1
        group_size = (4, 0)
        B_complex_per_group = (33 * 64 * 2 * 4, 0)
    af = bench.algorithmic_flops(D, 33, 1)
    c1 = 5 * 64 * 6
    assert round(af["per_kernel"]["rows"]) == 4 * 17 * c1
    assert round(af["per_kernel"]["cols"]) == (4 + 2) * 32 * c1 + 8 * 2 * 4 * 32 * 64
    assert round(af["per_kernel"]["out"]) == 2 * 32 * c1
    assert bench.algorithmic_bytes(D, 33, 1)["per_kernel"]["out"] == 2 * 64 * 64 * 4


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_metapupil_masks():
    """The learned filter's pupil-masked metric counts each layer's metapupil: the union over guide stars of
    the aperture's footprint at the layer's height (Sec. 2: star g sees layer l through c_g r + theta_g h_l)."""
    import numpy as np
    import synth
    geo = synth.preset("C1")
    masks = bench.metapupil_masks(geo)
    pupil = geo.pupil().astype(bool)
    M, n = geo.M, geo.n
    p0 = (M - n + 1) // 2
    # ground layer: every footprint is the pupil itself, placed like the zero extension
    ground = np.zeros((M, M), dtype=bool)
    ground[p0:p0 + n, p0:p0 + n] = pupil
    assert np.array_equal(masks[0], ground)
    # one star on axis: the metapupil is the pupil at every height
    on_axis = geo.replace(stars=[(0.0, 0.0, 0)])
    for m in bench.metapupil_masks(on_axis):
        assert np.array_equal(m, ground)
    # stars whose lines of sight shift the footprint by whole pixels at 6 km: the union of the shifted pupils
    t = geo.pitch / geo.heights[1]                          # one pixel at the second layer
    stars = [(3 * t, 0.0, 0), (0.0, -5 * t, 0), (-2 * t, 4 * t, 0)]
    masks = bench.metapupil_masks(geo.replace(stars=stars))
    want = np.zeros((M, M), dtype=bool)
    for sx, sy, _ in stars:
        want |= np.roll(np.roll(ground, int(round(sx / t)), axis=0), int(round(sy / t)), axis=1)
    assert np.array_equal(masks[0], ground)
    assert np.array_equal(masks[1], want)
