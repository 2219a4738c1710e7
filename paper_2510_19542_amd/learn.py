"""Learned spectral filter: binding of the GPU trainer and the training driver.

The network and the training objective are described in include/safr.h.  The
driver only orchestrates: it draws seeded random inputs (through ``synth``),
hands them to the trainer (which applies the tomography operator and computes
the statistics on the GPU) and runs Adam steps on shuffled minibatches.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import safr as S

N_PARAMS = S.SAFR_MLP_PARAMS
SHAPES = [(64, 4), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)]


def _lib():
    L = S.lib()
    if not getattr(L, "_learn_bound", False):
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        fp = ctypes.POINTER(ctypes.c_float)
        L.safr_trainer_create.argtypes = [ctypes.POINTER(S.safr_geometry), i, ctypes.POINTER(d), ctypes.POINTER(d),
                                          fp, i, ctypes.POINTER(vp), vp]
        L.safr_trainer_add_frames.argtypes = [vp, i, vp, vp, fp, vp]
        L.safr_trainer_set_params.argtypes = [vp, fp]
        L.safr_trainer_get_params.argtypes = [vp, fp]
        L.safr_trainer_get_state.argtypes = [vp, fp, fp, ctypes.POINTER(i)]
        L.safr_trainer_set_state.argtypes = [vp, fp, fp, i]
        L.safr_trainer_step.argtypes = [vp, i, ctypes.POINTER(i), ctypes.c_float, ctypes.POINTER(d), vp]
        L.safr_trainer_gradient.argtypes = [vp, i, ctypes.POINTER(i), fp, ctypes.POINTER(d), vp]
        L.safr_trainer_frames.argtypes = [vp]
        L.safr_trainer_frames.restype = i
        L.safr_trainer_destroy.argtypes = [vp]
        L.safr_trainer_destroy.restype = None
        L.safr_mlp_infer.argtypes = [fp, vp, i, d, vp, vp]
        L.safr_trainer_optimal_filter.argtypes = [vp, i, ctypes.POINTER(i), fp, ctypes.POINTER(d), vp]
        L.safr_trainer_tikhonov_loss.argtypes = [vp, i, ctypes.POINTER(i), d, ctypes.POINTER(d), vp]
        for name in ("safr_trainer_create", "safr_trainer_add_frames", "safr_trainer_set_params",
                     "safr_trainer_get_params", "safr_trainer_get_state", "safr_trainer_set_state",
                     "safr_trainer_step", "safr_trainer_gradient", "safr_mlp_infer",
                     "safr_trainer_optimal_filter", "safr_trainer_tikhonov_loss"):
            getattr(L, name).restype = ctypes.c_int
        L._learn_bound = True
    return L


def _geometry_struct(geo, keep):
    st = np.asarray(geo.stars, dtype=np.float64).reshape(-1, 3)
    arr = (S.safr_star * len(st))(*[S.safr_star(float(a), float(b), int(k)) for a, b, k in st])
    keep.append(arr)
    g = S.safr_geometry()
    g.n, g.M, g.pitch, g.J = int(geo.n), int(geo.M), float(geo.pitch), len(st)
    g.stars = arr
    g.h_lgs = float(geo.h_lgs)
    g.beta, g.alpha_tt, g.filter, g.noise = float(geo.beta), float(geo.alpha_tt), 0, 0.0
    return g


def init_params(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters (the shared input generator's draw)."""
    import synth
    return synth.mlp_init(seed)


class Trainer:
    """GPU trainer of the learned filter for one geometry (see safr_trainer_* in safr.h)."""

    def __init__(self, geo, amp: np.ndarray, max_frames: int, stream=None):
        L = _lib()
        keep = []
        g = _geometry_struct(geo, keep)
        h = np.ascontiguousarray(np.asarray(geo.heights, dtype=np.float64))
        w = np.ascontiguousarray(np.asarray(geo.weights, dtype=np.float64))
        a = np.ascontiguousarray(np.asarray(amp, dtype=np.float32))
        out = ctypes.c_void_p()
        S._check(L.safr_trainer_create(ctypes.byref(g), len(h), h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), int(max_frames),
                                       ctypes.byref(out), S._stream(stream)))
        self.handle = out.value
        self.geo = geo
        self.stream = stream

    def close(self):
        if self.handle:
            _lib().safr_trainer_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def frames(self) -> int:
        return int(_lib().safr_trainer_frames(ctypes.c_void_p(self.handle)))

    def add_frames(self, zl, zn, eta):
        """zl, zn: device complex64 tensors [F][L][Kh][M], [F][J][Kh][M]; eta: host array [F]."""
        e = np.ascontiguousarray(np.asarray(eta, dtype=np.float32))
        S._check(_lib().safr_trainer_add_frames(ctypes.c_void_p(self.handle), int(zl.shape[0]), S._ptr(zl),
                                                S._ptr(zn), e.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                S._stream(self.stream)))

    def set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        S._check(_lib().safr_trainer_set_params(ctypes.c_void_p(self.handle),
                                                p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        p = np.empty(N_PARAMS, dtype=np.float32)
        S._check(_lib().safr_trainer_get_params(ctypes.c_void_p(self.handle),
                                                p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def get_state(self):
        """(first moments, second moments, steps taken) of Adam."""
        m = np.empty(N_PARAMS, dtype=np.float32)
        v = np.empty(N_PARAMS, dtype=np.float32)
        n = ctypes.c_int()
        fp = ctypes.POINTER(ctypes.c_float)
        S._check(_lib().safr_trainer_get_state(ctypes.c_void_p(self.handle), m.ctypes.data_as(fp),
                                               v.ctypes.data_as(fp), ctypes.byref(n)))
        return m, v, int(n.value)

    def set_state(self, m, v, step: int):
        m = np.ascontiguousarray(np.asarray(m, dtype=np.float32))
        v = np.ascontiguousarray(np.asarray(v, dtype=np.float32))
        fp = ctypes.POINTER(ctypes.c_float)
        S._check(_lib().safr_trainer_set_state(ctypes.c_void_p(self.handle), m.ctypes.data_as(fp),
                                               v.ctypes.data_as(fp), int(step)))

    def save(self, path: str, **meta):
        """Checkpoint: parameters and Adam state (see save_checkpoint)."""
        m, v, n = self.get_state()
        save_checkpoint(path, self.get_params(), m, v, n, **meta)

    def load(self, path: str):
        """Restore a checkpoint written by save (parameters first: that resets the Adam state)."""
        params, m, v, n, _ = load_checkpoint(path)
        self.set_params(params)
        if m is not None:
            self.set_state(m, v, n)

    def step(self, frames, lr: float, want_loss: bool = False) -> Optional[float]:
        f = np.ascontiguousarray(np.asarray(frames, dtype=np.int32))
        loss = ctypes.c_double()
        S._check(_lib().safr_trainer_step(ctypes.c_void_p(self.handle), len(f),
                                          f.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(lr),
                                          ctypes.byref(loss) if want_loss else None, S._stream(self.stream)))
        return float(loss.value) if want_loss else None

    def gradient(self, frames):
        f = np.ascontiguousarray(np.asarray(frames, dtype=np.int32))
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        S._check(_lib().safr_trainer_gradient(ctypes.c_void_p(self.handle), len(f),
                                              f.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                              g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss),
                                              S._stream(self.stream)))
        return g, float(loss.value)


    def optimal_filter(self, frames, want_phi: bool = False):
        """Training objective of the closed-form optimal filter factors on these frames (the lower bound of
        every filter's), and optionally the factors [r][H] (see safr_trainer_optimal_filter)."""
        f = np.ascontiguousarray(np.asarray(frames, dtype=np.int32))
        loss = ctypes.c_double()
        phi = None
        if want_phi:
            r = min(self.geo.J, self.geo.L)
            phi = np.empty((r, (self.geo.M // 2 + 1) * self.geo.M), dtype=np.float32)
        S._check(_lib().safr_trainer_optimal_filter(
            ctypes.c_void_p(self.handle), len(f), f.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            phi.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if phi is not None else None, ctypes.byref(loss),
            S._stream(self.stream)))
        return (float(loss.value), phi) if want_phi else float(loss.value)

    def tikhonov_loss(self, frames, alpha: float) -> float:
        """Training objective of Tikhonov's filter factors s^2 / (s^2 + alpha) on these frames."""
        f = np.ascontiguousarray(np.asarray(frames, dtype=np.int32))
        loss = ctypes.c_double()
        S._check(_lib().safr_trainer_tikhonov_loss(ctypes.c_void_p(self.handle), len(f),
                                                   f.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(alpha),
                                                   ctypes.byref(loss), S._stream(self.stream)))
        return float(loss.value)

    def network_loss(self, params, frames, batch: int = 50) -> float:
        """Training objective of the network `params` on these frames (batch losses averaged; the
        parameters and the Adam state of this trainer are replaced)."""
        self.set_params(params)
        f = np.asarray(frames, dtype=np.int32)
        tot = 0.0
        for b in range(0, len(f), batch):
            part = f[b:b + batch]
            tot += self.gradient(part)[1] * len(part)
        return tot / len(f)


def add_seeded_frames(trainer: Trainer, first: int, count: int, chunk: int = 500, eta_range=(0.005, 0.05)):
    """Frames first .. first+count-1 drawn with synth.learn_draws, uploaded chunk by chunk."""
    import torch

    import synth
    for s in range(first, first + count, chunk):
        c = min(chunk, first + count - s)
        zl, zn, eta = synth.learn_draws(trainer.geo, s, c, eta_range=eta_range)
        trainer.add_frames(torch.from_numpy(zl.astype(np.complex64)).cuda(),
                           torch.from_numpy(zn.astype(np.complex64)).cuda(), eta)


def train(geo, frames: int = 20000, epochs: int = 3, batch: int = 16, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0, eta_range=(0.005, 0.05)):
    """Train the learned filter on `frames` method-generated frames; returns (params, loss history)."""
    import synth
    tr = Trainer(geo, synth.vk_amplitude(geo).reshape(geo.L, -1), frames)
    add_seeded_frames(tr, 0, frames, eta_range=eta_range)
    tr.set_params(init_params(seed))
    rng = np.random.default_rng([19542, 4, seed, 8])
    hist = []
    step = 0
    for ep in range(epochs):
        order = rng.permutation(frames)
        for b in range(0, frames - batch + 1, batch):
            want = log_every > 0 and step % log_every == 0
            loss = tr.step(order[b:b + batch], lr * (0.5 ** ep), want_loss=want)
            if want:
                hist.append((ep, step, loss))
            step += 1
    params = tr.get_params()
    tr.close()
    return params, hist


def save_checkpoint(path: str, params, m=None, v=None, step: int = 0, **meta):
    """Flat little-endian float32 file `path` (parameters, then the Adam moments if given) and the JSON
    metadata `path`.json (layout, sizes, step count and any caller fields)."""
    import json
    arrays = [np.asarray(params, dtype="<f4").ravel()]
    if m is not None:
        arrays += [np.asarray(m, dtype="<f4").ravel(), np.asarray(v, dtype="<f4").ravel()]
    for a in arrays:
        if a.size != N_PARAMS:
            raise ValueError(f"expected {N_PARAMS} values, got {a.size}")
    np.concatenate(arrays).tofile(path)
    info = {"format": "safr learned-filter checkpoint", "dtype": "float32 little-endian",
            "n_params": N_PARAMS, "blocks": ["params"] + (["adam_m", "adam_v"] if m is not None else []),
            "param_shapes": [list(sh) for sh in SHAPES], "adam_step": int(step), "meta": meta}
    with open(path + ".json", "w") as f:
        json.dump(info, f, indent=1)


def load_checkpoint(path: str):
    """(params, adam_m or None, adam_v or None, adam_step, metadata) from save_checkpoint's files."""
    import json
    with open(path + ".json") as f:
        info = json.load(f)
    if info.get("n_params") != N_PARAMS:
        raise ValueError("checkpoint holds a different network")
    flat = np.fromfile(path, dtype="<f4")
    blocks = info["blocks"]
    if flat.size != N_PARAMS * len(blocks):
        raise ValueError("checkpoint size does not match its metadata")
    parts = {b: flat[i * N_PARAMS:(i + 1) * N_PARAMS].astype(np.float32) for i, b in enumerate(blocks)}
    return parts["params"], parts.get("adam_m"), parts.get("adam_v"), int(info.get("adam_step", 0)), info["meta"]


def mlp_infer(params, feats, rows: int, noise: float, phi, stream=None):
    """BF16 inference of the network on device feature rows (see safr_mlp_infer)."""
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    S._check(_lib().safr_mlp_infer(p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), S._ptr(feats), int(rows),
                                   float(noise), S._ptr(phi), S._stream(stream)))
