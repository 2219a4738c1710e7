"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

Holds workload presets and a data simulator only; none of the reconstruction
method's arithmetic lives here.
"""
from .configs import (ARCSEC, LGS, NGS, Geometry, PRESETS, circular_pupil, preset,  # noqa: F401
                      c1, c2, c3, c5_small, c5_mid, c5_big, C5_SIZES, c5_instances)
from .atmosphere import (frame, frames, random_wavefronts, rng_for, simulate_wavefronts,  # noqa: F401
                         truth_layers, truth_screens, vk_screen)
from .learning import (MLP_SHAPES, learn_draws, mlp_init, periodic_frames, periodic_layers,  # noqa: F401
                       periodic_wavefronts, vk_amplitude)  # noqa: F401,E402
