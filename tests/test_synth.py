"""The seeded input generators: determinism and agreement of the data simulators with the oracle's
forward operators (the simulators feed the benchmark, which must not call the oracle)."""
import numpy as np

import synth
from oracle import safr as O


def test_periodic_wavefronts_equal_oracle_fourier_forward():
    geo = synth.preset("C1").replace(n=64)
    truth = synth.periodic_layers(geo, 7)
    c = O.cone_coefficients(geo.heights, 0, geo.h_lgs)
    want = O.forward_fourier(truth, O.layer_shifts(geo.stars, geo.heights, c, geo.pitch))
    got = synth.periodic_wavefronts(geo, truth)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_periodic_frames_noise_scales_with_eta_and_is_seeded():
    geo = synth.preset("C1").replace(n=64)
    truth, (w0, w1, w2) = synth.periodic_frames(geo, [3, 4], [0.0, 0.01, 0.02])
    truth2, (w1b,) = synth.periodic_frames(geo, [3, 4], [0.01])
    assert np.array_equal(truth, truth2) and np.array_equal(w1, w1b)
    n1 = w1.astype(np.float64) - w0
    n2 = w2.astype(np.float64) - w0
    assert np.allclose(n2, 2 * n1, rtol=0, atol=1e-5 * np.abs(w0).max())
    rms = np.sqrt(np.mean(w0.astype(np.float64) ** 2, axis=(2, 3)))
    ratio = np.sqrt(np.mean(n1 ** 2, axis=(2, 3))) / rms
    assert np.all(np.abs(ratio - 0.01) < 0.001)


def test_mixed_size_instances_are_seeded_and_cover_the_three_sizes():
    a = synth.c5_instances(64)
    assert a == synth.c5_instances(64) and len(a) == 64
    assert set(a) == set(synth.C5_SIZES)


def test_mlp_init_is_seeded_and_shaped():
    p = synth.mlp_init(3)
    assert p.dtype == np.float32 and p.size == sum(int(np.prod(s)) for s in synth.MLP_SHAPES) == 8705
    assert np.array_equal(p, synth.mlp_init(3)) and not np.array_equal(p, synth.mlp_init(4))
