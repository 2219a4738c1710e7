"""Restoring B from an exported copy (safr_import_B) and the deadline monitor of the closed-loop step
(SAFR_OPT_DEADLINE_US), through the C ABI.

* Import: B is redone only when the parameters change (Alg. 2, soft real time); a plan that imports another
  plan's exported B must reconstruct exactly as that plan, in FP32 and on the matrix cores, including the
  natural-star basis images of a mixed asterism.
* Deadline: the loop runs at 500-1000 Hz (Sec. 1); with a period the loop step counts its steps and those
  longer than the period.  The condition is forced from the host: a period of one second is never missed,
  one microsecond always is (a step launches several kernels).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available()
    S.lib()
    return torch, S


def _run(S, torch, plan, x, prec):
    F = int(x.shape[0])
    d = plan.desc
    need = S.safr_workspace_size(plan, F, prec)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    S.safr_set_workspace(plan, (ws.data_ptr() + 255) & ~255, need)
    out = torch.full((F, d.L, d.M, d.M), float("nan"), device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out, prec)
    torch.cuda.synchronize()
    S.safr_set_workspace(plan, 0, 0)
    return out


@pytest.mark.parametrize("name", ["C2", "C1", "C5-Mid"])
def test_import_B_reconstructs_exactly_as_the_exporting_plan(name):
    torch, S = _mods()
    geo = synth.preset(name)
    src = S.precompute_geometry(geo)
    dst = S.precompute_geometry(geo, alpha=geo.alpha * 4.0, alpha_tt=geo.alpha_tt * 4.0)
    x = torch.from_numpy(synth.random_wavefronts(geo, 5, seed=3)).cuda()
    precs = [S.SAFR_FP32] + ([S.SAFR_BF16X3] if geo.M <= 128 else [])
    before = _run(S, torch, dst, x, S.SAFR_FP32)
    for g in range(src.desc.groups):
        S.safr_import_B(dst, g, S.safr_export_B(src, g))
        assert np.array_equal(S.safr_export_B(dst, g), S.safr_export_B(src, g))
    for prec in precs:
        a = _run(S, torch, src, x, prec)
        b = _run(S, torch, dst, x, prec)
        assert torch.equal(a, b), (name, prec)
    assert not torch.equal(before, _run(S, torch, dst, x, S.SAFR_FP32))      # the import did change B
    # a later refresh rebuilds B from the plan's own SVDs: back to the source plan's alpha gives its B again
    S.safr_update_alpha(dst, geo.alpha, geo.alpha_tt)
    for g in range(src.desc.groups):
        assert np.array_equal(S.safr_export_B(dst, g), S.safr_export_B(src, g))


def test_import_B_rejects_bad_input():
    torch, S = _mods()
    geo = synth.preset("C1")
    plan = S.precompute_geometry(geo)
    B = S.safr_export_B(plan, 0)
    with pytest.raises(S.SafrError) as e:
        S.safr_import_B(plan, 1, B)                 # one group only
    assert e.value.status == S.SAFR_ERR_ARG
    with pytest.raises(S.SafrError) as e:
        S.safr_import_B(plan, 0, B[:-1])            # wrong size
    assert e.value.status == S.SAFR_ERR_ARG
    bad = B.copy()
    bad[3, 4, 1, 2] = np.nan
    with pytest.raises(S.SafrError) as e:
        S.safr_import_B(plan, 0, bad)
    assert e.value.status == S.SAFR_ERR_NUMERIC
    assert np.array_equal(S.safr_export_B(plan, 0), B)   # a rejected import leaves B as it was


def _loop(S, torch, plan, geo, steps, stream=None):
    wf = torch.from_numpy(synth.random_wavefronts(geo, 1, seed=7)).cuda()
    a = torch.zeros((1, geo.L, geo.M, geo.M), device="cuda")
    for _ in range(steps):
        S.safr_loop_step(plan, 1, wf, a, 0.5, a, stream)
    torch.cuda.synchronize()


def test_deadline_monitor_counts_steps_and_misses():
    torch, S = _mods()
    geo = synth.preset("C1")
    plan = S.precompute_geometry(geo)
    off = S.safr_deadline_stats(plan)
    assert off["steps"] == 0 and off["period_us"] == 0.0          # off by default
    _loop(S, torch, plan, geo, 2)
    assert S.safr_deadline_stats(plan)["steps"] == 0
    S.safr_set_option(plan, S.SAFR_OPT_DEADLINE_US, 1_000_000)    # 1 s: never missed
    _loop(S, torch, plan, geo, 5)
    st = S.safr_deadline_stats(plan, reset=True)
    print("1 s period:", st)
    assert st["steps"] == 5 and st["misses"] == 0 and st["period_us"] == 1e6
    assert 0.0 < st["last_us"] <= st["max_us"] < 1e6
    S.safr_set_option(plan, S.SAFR_OPT_DEADLINE_US, 1)            # 1 us: every step misses
    _loop(S, torch, plan, geo, 4)
    st = S.safr_deadline_stats(plan, reset=True)
    print("1 us period:", st)
    assert st["steps"] == 4 and st["misses"] == 4 and st["last_us"] > 1.0
    # captured in the loop step's graph and replayed: the stamps run with every replay
    stream = torch.cuda.Stream()
    S.safr_set_option(plan, S.SAFR_OPT_GRAPH, 1)
    _loop(S, torch, plan, geo, 3, stream)
    st = S.safr_deadline_stats(plan, reset=True, stream=stream)
    assert st["steps"] == 3 and st["misses"] == 3
    S.safr_set_option(plan, S.SAFR_OPT_DEADLINE_US, 0)
    _loop(S, torch, plan, geo, 2, stream)
    assert S.safr_deadline_stats(plan, stream=stream)["steps"] == 0
    with pytest.raises(S.SafrError) as e:
        S.safr_set_option(plan, S.SAFR_OPT_DEADLINE_US, -5)
    assert e.value.status == S.SAFR_ERR_ARG


def test_deadline_monitor_leaves_the_step_unchanged():
    """The monitored step computes the same commands as the plain step."""
    torch, S = _mods()
    geo = synth.preset("C2")
    plan = S.precompute_geometry(geo)
    wf = torch.from_numpy(synth.random_wavefronts(geo, 1, seed=8)).cuda()
    rng = np.random.default_rng(9)
    a0 = torch.from_numpy((0.1 * rng.standard_normal((1, geo.L, geo.M, geo.M))).astype(np.float32)).cuda()
    a = a0.clone()
    S.safr_loop_step(plan, 1, wf, a, 0.5, a)
    S.safr_set_option(plan, S.SAFR_OPT_DEADLINE_US, 1000)
    b = a0.clone()
    S.safr_loop_step(plan, 1, wf, b, 0.5, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert S.safr_deadline_stats(plan)["steps"] == 1
