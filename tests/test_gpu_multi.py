"""Mixed-size batches: several plans executed in one graph launch.

* the bundle's results equal each plan's own batched reconstruction bit for bit
  (same kernels, same launch shapes), launched eagerly and replayed from its captured
  graph on a non-default stream, with eager work in between;
* the mixed-size workload (64 instances of three sizes, 16 frames each, learned
  filter at eta = 2%) against the FP64 oracle on sampled frames of every size:
  relative L2 <= 1e-4 per frame.
"""
import collections

import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu


def _setup():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available()
    S.lib()
    return torch, S


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _mixed32():
    rng = np.random.default_rng(5)
    h = np.array([0.0, 3000.0, 8000.0])
    stars = [(float(x), float(y), k) for (x, y), k in zip(rng.uniform(-1.5e-4, 1.5e-4, (5, 2)), [1, 1, 1, 0, 0])]
    return synth.Geometry(name="mixed32", n=19, M=32, pitch=0.5, diameter=9.0, obstruction=0.1, stars=stars,
                          h_lgs=90e3, heights=h, weights=np.array([0.5, 0.3, 0.2]), alpha=5e-3, alpha_tt=1e-3,
                          beta=1.5, truth_heights=h, truth_fracs=np.ones(3) / 3, r0=0.15, L0=25.0, eta=0.01,
                          config_id=77)


@pytest.mark.parametrize("precision", ["FP32", "BF16X3"])
@pytest.mark.parametrize("mode", ["eager", "graph"])
def test_bundle_equals_single_plans(precision, mode):
    """eager: the legacy stream (launched directly); graph: a non-default stream, where the first call captures
    the entries as parallel branches of one graph and later calls replay it."""
    torch, S = _setup()
    prec = getattr(S, "SAFR_" + precision)
    geos = [synth.preset("C5-Mid"), synth.preset("C5-S"), _mixed32(), synth.preset("C5-S")]
    frames = [3, 5, 7, 2]
    plans = [S.precompute_geometry(g) for g in geos[:3]]
    plans.append(plans[1])                       # one plan serving two entries
    wf = [torch.from_numpy(synth.random_wavefronts(g, f, seed=i)).cuda() for i, (g, f) in enumerate(zip(geos, frames))]
    want = [S.reconstruct(p, x, precision=prec).cpu().numpy() for p, x in zip(plans, wf)]
    m = S.Multi(plans, frames, precision=prec)
    outs = [torch.full((f, g.L, g.M, g.M), float("nan"), device="cuda") for g, f in zip(geos, frames)]
    stream = torch.cuda.Stream() if mode == "graph" else torch.cuda.current_stream()
    assert (stream.cuda_stream != 0) == (mode == "graph")
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        m.execute(wf, outs, stream=stream)
        torch.cuda.synchronize()
        for i, (o, w) in enumerate(zip(outs, want)):
            assert np.array_equal(o.cpu().numpy(), w), (precision, rep, i)
        _ = (wf[0] * 2).sum().item()             # eager work between replays
    m.close()


def test_bundle_rejects_bad_arguments():
    torch, S = _setup()
    plan = S.precompute_geometry(synth.preset("C2"))
    with pytest.raises(S.SafrError):
        S.Multi([plan], [0])
    with pytest.raises(S.SafrError):
        S.Multi([plan], [4], precision=S.SAFR_BF16X3)      # no matrix-core path at M = 256


def test_mixed_size_workload_learned_filter():
    """64 instances drawn from three sizes, 16 frames each; learned filter at eta = 2%."""
    torch, S = _setup()
    count = collections.Counter(synth.c5_instances(64))
    params = synth.mlp_init(11)
    eta = 0.02
    names = [n for n in synth.C5_SIZES if count[n]]
    geos = [synth.preset(n) for n in names]
    frames = [16 * count[n] for n in names]
    plans = [S.precompute_geometry(g, filter=S.SAFR_FILTER_MLP, mlp=params, noise=eta) for g in geos]
    wf_host = [synth.random_wavefronts(g, f, seed=50 + i) for i, (g, f) in enumerate(zip(geos, frames))]
    wf = [torch.from_numpy(w).cuda() for w in wf_host]
    outs = [torch.empty((f, g.L, g.M, g.M), device="cuda") for g, f in zip(geos, frames)]
    m = S.Multi(plans, frames)
    m.autotune(wf, outs, iters=2)
    # a non-default stream: the first call captures the bundle's graph, the second replays it
    stream = torch.cuda.Stream()
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        m.execute(wf, outs, stream=stream)
        torch.cuda.synchronize()
        if rep == 0:
            first = [o.clone() for o in outs]
    for o, o1 in zip(outs, first):
        assert torch.equal(o, o1)
    for name, g, f, w, o in zip(names, geos, frames, wf_host, outs):
        ref = O.precompute_geometry(g, mlp_params=params.astype(np.float64), eta=np.float32(eta), mlp_bf16=True)
        got = o.cpu().numpy()
        assert np.isfinite(got).all(), name
        worst = 0.0
        for k in sorted({0, f // 2, f - 1}):
            e = _rel(got[k], O.reconstruct(ref, w[k].astype(np.float64)))
            worst = max(worst, e)
            assert e <= 1e-4, (name, k, e)
        print(f"{name}: {count[name]} instances, {f} frames, worst sampled rel-L2 {worst:.2e}")
    m.close()
