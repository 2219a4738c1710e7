"""Thin Python binding of the SAFR C ABI (include/safr.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library ``libsafr.so``.  Device buffers are passed as torch tensors (or raw
device pointers); streams as ``torch.cuda.Stream`` objects, raw handles or None
(the current torch stream).  The library must be built (``build.py``); importing
works without it, but every call raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsafr.so")

SAFR_OK, SAFR_ERR_ARG, SAFR_ERR_GEOMETRY, SAFR_ERR_DOMAIN = 0, -1, -2, -3
SAFR_ERR_UNSUPPORTED, SAFR_ERR_NUMERIC, SAFR_ERR_DEVICE, SAFR_ERR_STATE = -4, -5, -6, -7
SAFR_NGS, SAFR_LGS = 0, 1
SAFR_FILTER_TIKHONOV, SAFR_FILTER_MLP, SAFR_FILTER_TSVD = 0, 1, 2
SAFR_FP32, SAFR_BF16X3 = 0, 1
SAFR_OPT_GRAPH, SAFR_OPT_ROW_TEAMS, SAFR_OPT_OUT_ROWS, SAFR_OPT_MFMA_FRAMES, SAFR_OPT_COL_FRAMES = 0, 1, 2, 3, 4
SAFR_OPT_COL_PREFETCH, SAFR_OPT_OUT_FRAMES, SAFR_OPT_COL_TOGETHER, SAFR_OPT_CHECK_FINITE = 5, 6, 7, 8
SAFR_OPT_DEADLINE_US, SAFR_OPT_COL_MFMA, SAFR_OPT_SEQ_FRAMES, SAFR_OPT_FUSED = 9, 10, 11, 12
SAFR_MAX_LAYERS = 16
SAFR_MLP_PARAMS = 8705

EXPORTED = [
    "safr_precompute", "safr_reconstruct", "safr_reconstruct_batched", "safr_workspace_size",
    "safr_set_workspace", "safr_plan_info", "safr_export_B", "safr_set_option", "safr_time_stages",
    "safr_autotune", "safr_destroy", "safr_last_error",
    "safr_multi_create", "safr_multi_execute", "safr_multi_autotune", "safr_multi_destroy",
    "safr_polc", "safr_loop_step", "safr_strehl", "safr_update_alpha", "safr_import_B", "safr_deadline_stats",
    "safr_reconstruct_batched_static", "safr_static_workspace_bytes",
    # learned filter (bound in learn.py)
    "safr_trainer_create", "safr_trainer_add_frames", "safr_trainer_set_params", "safr_trainer_get_params",
    "safr_trainer_get_state", "safr_trainer_set_state",
    "safr_trainer_step", "safr_trainer_gradient", "safr_trainer_frames", "safr_trainer_destroy", "safr_mlp_infer",
    "safr_trainer_optimal_filter", "safr_trainer_tikhonov_loss",
]


class SafrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"SAFR status {status}: {message}")
        self.status = status


class safr_star(ctypes.Structure):
    _fields_ = [("ax", ctypes.c_double), ("ay", ctypes.c_double), ("kind", ctypes.c_int)]


class safr_geometry(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("M", ctypes.c_int), ("pitch", ctypes.c_double),
        ("J", ctypes.c_int), ("stars", ctypes.POINTER(safr_star)),
        ("h_lgs", ctypes.c_double), ("pupil", ctypes.POINTER(ctypes.c_ubyte)),
        ("beta", ctypes.c_double), ("alpha_tt", ctypes.c_double), ("filter", ctypes.c_int),
        ("mlp", ctypes.POINTER(ctypes.c_float)), ("noise", ctypes.c_double),
        ("alpha_weight", ctypes.POINTER(ctypes.c_double)),
    ]


class safr_plan_desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("M", ctypes.c_int), ("J", ctypes.c_int), ("L", ctypes.c_int),
        ("groups", ctypes.c_int), ("group_size", ctypes.c_int * 2), ("group_kind", ctypes.c_int * 2),
        ("c", ctypes.c_double * SAFR_MAX_LAYERS), ("layer_pitch", ctypes.c_double * SAFR_MAX_LAYERS),
        ("B_complex_per_group", ctypes.c_size_t * 2),
    ]


class safr_deadline_info(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_ulonglong), ("misses", ctypes.c_ulonglong), ("last_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("period_us", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libsafr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2510_19542_amd/build.py")
    # torch ships its own HIP runtime with the same soname; loading it first makes the
    # library bind to that one runtime, so torch's streams and allocations are valid in it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    L.safr_precompute.argtypes = [ctypes.POINTER(safr_geometry), i, ctypes.POINTER(d), ctypes.POINTER(d), d,
                                  ctypes.POINTER(vp), vp]
    L.safr_reconstruct.argtypes = [vp, vp, vp, vp]
    L.safr_reconstruct_batched.argtypes = [vp, i, vp, vp, i, vp]
    L.safr_workspace_size.argtypes = [vp, i, i, ctypes.POINTER(sz)]
    L.safr_set_workspace.argtypes = [vp, vp, sz]
    L.safr_plan_info.argtypes = [vp, ctypes.POINTER(safr_plan_desc)]
    L.safr_export_B.argtypes = [vp, i, ctypes.POINTER(d), sz]
    L.safr_set_option.argtypes = [vp, i, i]
    L.safr_time_stages.argtypes = [vp, i, vp, vp, i, i, vp, ctypes.POINTER(d)]
    L.safr_autotune.argtypes = [vp, i, vp, vp, i, i, vp, ctypes.POINTER(i)]
    L.safr_destroy.argtypes = [vp]
    L.safr_destroy.restype = None
    L.safr_last_error.restype = ctypes.c_char_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.safr_multi_create.argtypes = [pp, ctypes.POINTER(i), i, i, ctypes.POINTER(vp)]
    L.safr_multi_execute.argtypes = [vp, pp, pp, vp]
    L.safr_multi_autotune.argtypes = [vp, pp, pp, i, vp]
    L.safr_multi_destroy.argtypes = [vp]
    L.safr_multi_destroy.restype = None
    L.safr_polc.argtypes = [vp, i, vp, vp, ctypes.c_float, vp, vp]
    L.safr_loop_step.argtypes = [vp, i, vp, vp, ctypes.c_float, vp, vp]
    L.safr_strehl.argtypes = [vp, i, i, ctypes.POINTER(d), vp, vp, ctypes.c_float, vp, vp, vp]
    L.safr_update_alpha.argtypes = [vp, d, d, i, ctypes.POINTER(d), vp]
    L.safr_import_B.argtypes = [vp, i, ctypes.POINTER(d), sz, vp]
    L.safr_reconstruct_batched_static.argtypes = [vp, i, vp, vp, i, vp]
    L.safr_static_workspace_bytes.argtypes = []
    L.safr_static_workspace_bytes.restype = sz
    L.safr_deadline_stats.argtypes = [vp, ctypes.POINTER(safr_deadline_info), i, vp]
    for name in EXPORTED[:EXPORTED.index("safr_trainer_create")]:
        if name not in ("safr_destroy", "safr_last_error", "safr_multi_destroy", "safr_static_workspace_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def safr_last_error() -> str:
    return lib().safr_last_error().decode()


def _check(status: int):
    if status != SAFR_OK:
        raise SafrError(status, safr_last_error())


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(s) -> int:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


class Plan:
    """Owns a safr_plan; released on close() or garbage collection."""

    def __init__(self, handle: int):
        self.handle = handle
        self.desc = safr_plan_info(self)

    def close(self):
        if self.handle:
            lib().safr_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return ctypes.c_void_p(self.handle)


def safr_precompute(*, n: int, M: int, pitch: float, stars: Sequence, h_lgs: float, heights, weights,
                    alpha: float, alpha_tt: float, beta: float, pupil=None, filter: int = SAFR_FILTER_TIKHONOV,
                    mlp=None, noise: float = 0.0, alpha_weight=None, stream=None) -> Plan:
    """Alg. 2 on the GPU (see safr.h); returns a Plan.  alpha_weight: optional (M, M) per-frequency
    multipliers of alpha (point-symmetric)."""
    L = lib()
    st = np.asarray(stars, dtype=np.float64).reshape(-1, 3)
    arr = (safr_star * len(st))(*[safr_star(float(a), float(b), int(k)) for a, b, k in st])
    g = safr_geometry()
    g.n, g.M, g.pitch, g.J = int(n), int(M), float(pitch), len(st)
    g.stars = arr
    g.h_lgs = float(h_lgs)
    keep = []
    if pupil is not None:
        pb = np.ascontiguousarray(np.asarray(pupil, dtype=np.uint8).reshape(n, n))
        keep.append(pb)
        g.pupil = pb.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
    g.beta, g.alpha_tt, g.filter, g.noise = float(beta), float(alpha_tt), int(filter), float(noise)
    if mlp is not None:
        mb = np.ascontiguousarray(np.asarray(mlp, dtype=np.float32).ravel())
        keep.append(mb)
        g.mlp = mb.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    if alpha_weight is not None:
        aw = np.ascontiguousarray(np.asarray(alpha_weight, dtype=np.float64).reshape(M, M))
        keep.append(aw)
        g.alpha_weight = aw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = np.ascontiguousarray(np.asarray(heights, dtype=np.float64))
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    out = ctypes.c_void_p()
    _check(L.safr_precompute(ctypes.byref(g), len(h), h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(alpha),
                             ctypes.byref(out), _stream(stream)))
    return Plan(out.value)


def precompute_geometry(geo, stream=None, **kw) -> Plan:
    """safr_precompute for an object with the fields of a workload preset."""
    args = dict(n=geo.n, M=geo.M, pitch=geo.pitch, stars=geo.stars, h_lgs=geo.h_lgs, heights=geo.heights,
                weights=geo.weights, alpha=geo.alpha, alpha_tt=geo.alpha_tt, beta=geo.beta, pupil=geo.pupil())
    args.update(kw)
    return safr_precompute(stream=stream, **args)


def safr_reconstruct(plan: Plan, wavefronts, layers, stream=None):
    _check(lib().safr_reconstruct(plan._as_parameter_, _ptr(wavefronts), _ptr(layers), _stream(stream)))


def safr_reconstruct_batched(plan: Plan, frames: int, wavefronts, layers, precision: int = SAFR_FP32,
                             stream=None):
    _check(lib().safr_reconstruct_batched(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(layers),
                                          int(precision), _stream(stream)))


def safr_reconstruct_batched_static(plan: Plan, frames: int, wavefronts, layers, precision: int = SAFR_FP32,
                                    stream=None):
    """safr_reconstruct_batched with the library's static workspace (allocates nothing; see safr.h)."""
    _check(lib().safr_reconstruct_batched_static(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(layers),
                                                 int(precision), _stream(stream)))


def safr_static_workspace_bytes() -> int:
    return int(lib().safr_static_workspace_bytes())


def safr_workspace_size(plan: Plan, frames: int, precision: int = SAFR_FP32) -> int:
    out = ctypes.c_size_t()
    _check(lib().safr_workspace_size(plan._as_parameter_, int(frames), int(precision), ctypes.byref(out)))
    return int(out.value)


def safr_set_workspace(plan: Plan, workspace, nbytes: int):
    _check(lib().safr_set_workspace(plan._as_parameter_, _ptr(workspace), int(nbytes)))


def safr_set_option(plan: Plan, option: int, value: int):
    _check(lib().safr_set_option(plan._as_parameter_, int(option), int(value)))


def safr_time_stages(plan: Plan, frames: int, wavefronts, layers, precision: int = SAFR_FP32, iters: int = 20,
                     stream=None):
    """Milliseconds per launch of (row pass, column pass + apply, output pass): one batched call, then each
    stage's kernels `iters` times back to back between HIP events on the launch stream."""
    ms = (ctypes.c_double * 3)()
    _check(lib().safr_time_stages(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(layers), int(precision),
                                  int(iters), _stream(stream), ms))
    return [float(x) for x in ms]


def safr_autotune(plan: Plan, frames: int, wavefronts, layers, precision: int = SAFR_FP32, iters: int = 10,
                  stream=None):
    """Times the admissible block shapes of each stage and keeps the fastest; returns
    (row teams, output rows per block, column frames per block, output frames per block,
    column frames transformed together)."""
    ch = (ctypes.c_int * 5)()
    _check(lib().safr_autotune(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(layers), int(precision),
                               int(iters), _stream(stream), ch))
    return tuple(int(x) for x in ch)


def safr_update_alpha(plan: Plan, alpha: float, alpha_tt: float = 0.0, filter: int = SAFR_FILTER_TIKHONOV,
                      alpha_weight=None, stream=None):
    """Rebuild B for new regularisation parameters from the plan's kept SVDs (synchronises)."""
    M = plan.desc.M
    aw = None
    if alpha_weight is not None:
        aw = np.ascontiguousarray(np.asarray(alpha_weight, dtype=np.float64).reshape(M, M))
    _check(lib().safr_update_alpha(plan._as_parameter_, float(alpha), float(alpha_tt), int(filter),
                                   None if aw is None else aw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   _stream(stream)))


def safr_polc(plan: Plan, frames: int, wavefronts, layers, weight: float, out, stream=None):
    """Pseudo-open-loop data: out = pupil * (wavefronts + weight * A(layers)) for each frame."""
    _check(lib().safr_polc(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(layers), float(weight),
                           _ptr(out), _stream(stream)))


def safr_loop_step(plan: Plan, frames: int, wavefronts, a_in, gain: float, a_out, stream=None):
    """One closed-loop step: a_out = (1 - gain) a_in + gain * SAFR(POLC(wavefronts, a_in))."""
    _check(lib().safr_loop_step(plan._as_parameter_, int(frames), _ptr(wavefronts), _ptr(a_in), float(gain),
                                _ptr(a_out), _stream(stream)))


def safr_strehl(plan: Plan, frames: int, directions, open_loop, layers, scale: float, sr, var=None, stream=None):
    """Marechal Strehl ratios sr[f][d] (and residual variances var[f][d], rad^2) in science directions."""
    dirs = np.ascontiguousarray(np.asarray(directions, dtype=np.float64).reshape(-1, 2))
    _check(lib().safr_strehl(plan._as_parameter_, int(frames), len(dirs),
                             dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(open_loop), _ptr(layers),
                             float(scale), _ptr(sr), _ptr(var), _stream(stream)))


def safr_plan_info(plan: Plan) -> safr_plan_desc:
    d = safr_plan_desc()
    _check(lib().safr_plan_info(plan._as_parameter_, ctypes.byref(d)))
    return d


def safr_export_B(plan: Plan, group: int) -> np.ndarray:
    """FP64 B of one group as complex128 [k = 0..M/2][j = 0..M-1][l][g]."""
    d = plan.desc
    cnt = int(d.B_complex_per_group[group])
    buf = np.empty(2 * cnt, dtype=np.float64)
    _check(lib().safr_export_B(plan._as_parameter_, int(group), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               buf.size))
    z = buf[0::2] + 1j * buf[1::2]
    return z.reshape(d.M // 2 + 1, d.M, d.L, d.group_size[group])


def safr_import_B(plan: Plan, group: int, B, stream=None):
    """Replace one group's B by complex128 [k = 0..M/2][j = 0..M-1][l][g] (the layout of safr_export_B)
    and rebuild its FP32, BF16 and basis-image forms (synchronises)."""
    z = np.ascontiguousarray(np.asarray(B, dtype=np.complex128))
    flat = np.ascontiguousarray(z.view(np.float64).ravel())
    _check(lib().safr_import_B(plan._as_parameter_, int(group), flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               flat.size, _stream(stream)))


def safr_deadline_stats(plan: Plan, reset: bool = False, stream=None) -> dict:
    """Deadline monitor of the loop step: steps, misses (longer than the period), last and longest step [us]."""
    info = safr_deadline_info()
    _check(lib().safr_deadline_stats(plan._as_parameter_, ctypes.byref(info), int(bool(reset)), _stream(stream)))
    return {"steps": int(info.steps), "misses": int(info.misses), "last_us": float(info.last_us),
            "max_us": float(info.max_us), "period_us": float(info.period_us)}


class Multi:
    """A mixed-size batch: plans with their frame counts, executed in one graph launch."""

    def __init__(self, plans, frames, precision: int = SAFR_FP32):
        self.plans = list(plans)                 # keep the plans alive
        self.frames = [int(f) for f in frames]
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        fr = (ctypes.c_int * len(self.frames))(*self.frames)
        out = ctypes.c_void_p()
        _check(lib().safr_multi_create(arr, fr, len(self.plans), int(precision), ctypes.byref(out)))
        self.handle = out.value

    @staticmethod
    def _ptrs(bufs):
        return (ctypes.c_void_p * len(bufs))(*[_ptr(b) for b in bufs])

    def execute(self, wavefronts, layers, stream=None):
        _check(lib().safr_multi_execute(ctypes.c_void_p(self.handle), self._ptrs(wavefronts), self._ptrs(layers),
                                        _stream(stream)))

    def autotune(self, wavefronts, layers, iters: int = 5, stream=None):
        _check(lib().safr_multi_autotune(ctypes.c_void_p(self.handle), self._ptrs(wavefronts), self._ptrs(layers),
                                         int(iters), _stream(stream)))

    def close(self):
        if self.handle:
            lib().safr_multi_destroy(ctypes.c_void_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def safr_destroy(plan: Plan):
    plan.close()


def reconstruct(plan: Plan, wavefronts, precision: int = SAFR_FP32, workspace=None, stream=None):
    """Convenience: allocate the output (and, for several frames, a workspace) and reconstruct.

    wavefronts: device float32 tensor (J, n, n) or (F, J, n, n).  Returns (F?, L, M, M).
    """
    import torch
    d = plan.desc
    single = wavefronts.dim() == 3
    F = 1 if single else int(wavefronts.shape[0])
    out = torch.empty((F, d.L, d.M, d.M), dtype=torch.float32, device=wavefronts.device)
    if F > 1 or precision != SAFR_FP32:
        need = safr_workspace_size(plan, F, precision)
        if workspace is None:
            workspace = torch.empty(need + 256, dtype=torch.uint8, device=wavefronts.device)
        base = _ptr(workspace)
        aligned = (base + 255) & ~255
        safr_set_workspace(plan, aligned, need)
        safr_reconstruct_batched(plan, F, wavefronts, out, precision, stream)
        safr_set_workspace(plan, 0, 0)
    else:
        safr_reconstruct(plan, wavefronts, out, stream)
    return out[0] if single else out
