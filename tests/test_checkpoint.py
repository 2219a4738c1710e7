"""Learned-filter checkpoint files (flat float32 + JSON metadata), CPU only."""
import json

import numpy as np
import pytest

from paper_2510_19542_amd import learn as Lrn


def test_round_trip_with_adam_state(tmp_path):
    rng = np.random.default_rng(1)
    p, m, v = rng.standard_normal((3, Lrn.N_PARAMS)).astype(np.float32)
    v = np.abs(v)
    path = str(tmp_path / "c.bin")
    Lrn.save_checkpoint(path, p, m, v, 42, geometry="C1", eta=[0.005, 0.05])
    p2, m2, v2, n, meta = Lrn.load_checkpoint(path)
    assert np.array_equal(p2, p) and np.array_equal(m2, m) and np.array_equal(v2, v)
    assert n == 42 and meta == {"geometry": "C1", "eta": [0.005, 0.05]}
    info = json.load(open(path + ".json"))
    assert info["blocks"] == ["params", "adam_m", "adam_v"] and info["n_params"] == Lrn.N_PARAMS
    assert sum(int(np.prod(s)) for s in info["param_shapes"]) == Lrn.N_PARAMS
    raw = np.fromfile(path, dtype="<f4")
    assert raw.size == 3 * Lrn.N_PARAMS and np.array_equal(raw[:Lrn.N_PARAMS], p)


def test_rejects_mismatched_files(tmp_path):
    path = str(tmp_path / "c.bin")
    with pytest.raises(ValueError):
        Lrn.save_checkpoint(path, np.zeros(10, np.float32))
    Lrn.save_checkpoint(path, np.zeros(Lrn.N_PARAMS, np.float32))
    np.zeros(Lrn.N_PARAMS + 3, np.float32).tofile(path)        # truncated or padded payload
    with pytest.raises(ValueError):
        Lrn.load_checkpoint(path)
