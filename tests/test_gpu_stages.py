"""Per-stage parity (white box): the intermediates a batched call leaves in the caller's workspace.

After safr_reconstruct_batched the workspace holds, at offset 0, the row spectra
R[f][slot][k][row] (complex64, group order, slots k = 0..M/2 of which k < M/2 are written: B
ignores the Nyquist column; the n pupil rows) of the transformed stars, and after them the layer spectra after the inverse column transforms,
C[f][l][p / 8][k][p % 8] (complex64, row tiles of 8, columns k < M/2; the 1/M^2
of IDFT2 is included).  Each is compared with what the oracle's steps give:
* R: the DFT along the second grid axis of the zero-extended, pupil-masked rows
  (numpy's FFT of the rows, a library primitive);
* C: the oracle's B applied to the oracle's DFT2 of the prepared data (tip/tilt
  removed for the laser stars of a mixed asterism), then the inverse DFT along the
  first axis scaled by 1/M^2.
Tolerance: relative L2 1e-5 per frame and star or layer (FP32 against FP64).

For mixed asterisms the workspace also holds, after C, the tip/tilt plane coefficients (b, c) of every
row chunk of every frame and star, part[f][slot][chunk] (the fit is linear in the data, so each row-pass
block forms its own rows' share), and, with more than 8 chunks, their sums planes[f][slot] after them: the
plane b x + c y that the summed parts define over the pupil must match the oracle's least-squares fit
(Sec. 3.3) within 1e-5 of the largest wavefront value.  The row-pass blocks take 2 x teams rows, so the
cases cover 1, 5 and 10 chunks at M = 32 and 5 and 9 at M = 256.
"""
import numpy as np
import pytest

import synth
from oracle import safr as O

pytestmark = pytest.mark.gpu


def _mods():
    import torch
    from paper_2510_19542_amd import safr as S
    assert torch.cuda.is_available()
    S.lib()
    return torch, S


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _small_mixed():
    rng = np.random.default_rng(77)
    M, n, pitch = 32, 19, 0.5
    stars = [(float(x), float(y), k) for (x, y), k in zip(rng.uniform(-3e-5, 3e-5, (5, 2)), (1, 1, 1, 0, 0))]
    h = np.array([0.0, 3000.0, 8000.0])
    return synth.Geometry(name="stage-mixed", n=n, M=M, pitch=pitch, diameter=(n - 1) * pitch, obstruction=0.2,
                          stars=stars, h_lgs=90e3, heights=h, weights=np.array([0.6, 0.3, 0.1]), alpha=1e-3,
                          alpha_tt=1e-3, beta=1.5, truth_heights=h, truth_fracs=np.array([0.6, 0.3, 0.1]),
                          r0=0.15, L0=25.0, eta=0.01, config_id=177)


CASES = {"C1": lambda: synth.preset("C1"), "C2": lambda: synth.preset("C2"), "m32-mixed": _small_mixed}


@pytest.mark.parametrize("case,teams", [("C1", None), ("C2", 8), ("C2", 4), ("m32-mixed", 10), ("m32-mixed", 2),
                                        ("m32-mixed", 1)])
def test_row_and_column_pass_intermediates(case, teams):
    torch, S = _mods()
    geo = CASES[case]()
    plan = S.precompute_geometry(geo)
    S.safr_set_option(plan, S.SAFR_OPT_FUSED, 0)     # the three passes, whose intermediates are inspected
    if teams is not None:
        S.safr_set_option(plan, S.SAFR_OPT_ROW_TEAMS, teams)
    ref = O.precompute_geometry(geo)
    F = 2
    wf = synth.frames(geo, F, first=4)
    x = torch.from_numpy(wf).cuda()
    need = S.safr_workspace_size(plan, F)
    ws = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    base = (int(ws.data_ptr()) + 255) & ~255
    off = base - int(ws.data_ptr())
    S.safr_set_workspace(plan, base, need)
    out = torch.empty((F, geo.L, geo.M, geo.M), device="cuda")
    S.safr_reconstruct_batched(plan, F, x, out)
    torch.cuda.synchronize()
    raw = ws[off:off + need].cpu().numpy()
    S.safr_set_workspace(plan, 0, 0)

    M, n, J, L = geo.M, geo.n, geo.J, geo.L
    Kh = M // 2 + 1
    p0 = (M - n + 1) // 2
    pupil = ref.pupil
    grp = ref.groups[0]                                     # the transformed group (laser stars when mixed)
    r_bytes = F * J * Kh * n * 8
    R = raw[:r_bytes].view(np.complex64).reshape(F, J, Kh, n)
    r_end = (r_bytes + 255) // 256 * 256
    C = raw[r_end:r_end + F * L * Kh * M * 8].view(np.complex64).reshape(F, L, M // 8, Kh, 8)
    for f in range(F):
        # R is stored in group order: the transformed group's stars first, slot i = its i-th star
        for slot, g in enumerate(grp.stars):
            ext = np.zeros((n, M))
            ext[:, p0:p0 + n] = np.where(pupil, wf[f, g].astype(np.float64), 0.0)
            want = np.fft.fft(ext, axis=1)[:, :Kh].T          # [k][row]
            e = rel(R[f, slot][: M // 2], want[: M // 2])
            assert e <= 1e-5, (case, f, g, e)
        psi = np.stack([O.prepare(wf[f, g].astype(np.float64), pupil, grp.tt_mode) for g in grp.stars])
        b = O.apply_B(grp.B, O.dft2(O.zero_extend(psi, M)))    # [l][j][k]
        want_c = np.fft.ifft(b, axis=1) / M                     # inverse along j, times 1/M^2 overall
        got_c = C[f].transpose(0, 1, 3, 2).reshape(L, M, Kh)      # [l][p][k]
        for l in range(L):
            e = rel(got_c[l][:, :M // 2], want_c[l][:, :M // 2])
            assert e <= 1e-5, (case, f, l, e)

    mixed = len(ref.groups) > 1
    if not mixed:
        return
    a256 = lambda b: (b + 255) // 256 * 256
    nchunk = -(-n // (2 * teams))
    m_off = a256(r_bytes) + a256(F * L * Kh * M * 8)
    part = raw[m_off:m_off + F * J * nchunk * 8].view(np.float32).reshape(F, J, nchunk, 2)
    planes = part.astype(np.float64).sum(axis=2)
    if nchunk > 8:                      # summed by one more launch: the passes read those sums
        p_off = m_off + a256(F * J * ((n + 1) // 2) * 8)
        sums = raw[p_off:p_off + F * J * 8].view(np.float32).reshape(F, J, 2)
        assert np.allclose(sums, planes, rtol=1e-5, atol=1e-6 * np.abs(planes).max())
    # stored in group order: the laser stars first, then the natural stars, each in star order
    slot = {g: i for i, g in enumerate([g for grp in ref.groups for g in grp.stars])}
    x = np.arange(n) - (n - 1) / 2.0
    X, Y = np.meshgrid(x, x, indexing="ij")
    for f in range(F):
        for g in range(J):
            psi = np.where(pupil, wf[f, g].astype(np.float64), 0.0)
            want_p = np.where(pupil, O.tt_plane(psi, pupil), 0.0)
            b, c = planes[f, slot[g]]
            got_p = np.where(pupil, b * X + c * Y, 0.0)
            err = np.max(np.abs(got_p - want_p))
            assert err <= 1e-5 * np.max(np.abs(psi)), (case, f, g, err, np.max(np.abs(psi)))
