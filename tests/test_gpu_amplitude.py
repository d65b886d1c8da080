"""Amplitude-modulating SLMs on the GPU against the FP64 oracle.

The binary and multi-level amplitude schemes (transmissions k / (L - 1),
nearest to Re g; the zero order keeps R and stays out of the NMSE) run
through every column-pass kernel: the single-launch small kernel (64^2),
the tile kernel (256^2, 512 x 1024, 1024^2) and the classic kernels
(2048 x 512).  hg_gs_step is compared with the oracle's step (R and g to
1e-4 relative L2, levels with the bounded distance exemption, both NMSE
values, weights), and whole batched calls, phase and amplitude problems
mixed in one size class, are held in lock-step for three iterations.
"""
import numpy as np
import pytest

import synth
from oracle import hologram, slm
from parity import FIELD_TOL, NMSE_TOL, level_check, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"
AMP = hg.HG_SLM_AMPLITUDE


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


# (ny, nx, L, weighted, Fresnel z or None)
CASES = [(64, 64, 2, False, None), (64, 64, 8, True, None), (256, 256, 2, False, None), (256, 256, 4, True, 0.2),
         (512, 1024, 16, False, 0.3), (1024, 1024, 2, True, None), (2048, 512, 3, False, None)]


@pytest.mark.parametrize("ny,nx,L,weighted,z", CASES)
def test_amplitude_step_matches_oracle_step(ny, nx, L, weighted, z):
    say("amplitude hg_gs_step", ny, nx, L, "wgs" if weighted else "gs", z)
    T_raw = synth.gaussian_target(nx, seed=31, ny=ny)
    T = hologram.prepare_target(T_raw, L, amplitude=True)
    rng = np.random.default_rng(ny + nx + L)
    lev = rng.integers(0, L, (ny, nx))
    f = slm.amplitude_value(lev, L) + 0j
    w = rng.uniform(0.5, 2.0, (ny, nx)) if weighted else None
    optics = (synth.WAVELENGTH_M, synth.PITCH_M, z) if z else (0.0, 0.0, 0.0)
    out = hg.hg_gs_step(dev(T_raw), L | AMP, levels_in=dev(lev.astype(np.uint8)),
                        weights=None if w is None else dev(w.astype(np.float32)), wavelength_m=optics[0],
                        pitch_m=optics[1], z_m=optics[2])
    gpu = {k: (None if v is None else host(v)) for k, v in out.items()}
    ref = hologram.gs_step(T, L, f, weighted=weighted, w_prev=w, optics=optics if z else None, amplitude=True)
    er, eg = rel_l2(gpu["replay"], ref["replay"]), rel_l2(gpu["g"], ref["g"])
    assert er < FIELD_TOL and eg < FIELD_TOL, (er, eg)
    bad, _ = level_check(gpu["levels"], ref["levels"], ref["g"], L, where="amplitude step", amplitude=True)
    assert bad == 0
    assert _rel(gpu["nmse"][0], ref["nmse"]) < NMSE_TOL, (gpu["nmse"][0], ref["nmse"])
    assert _rel(gpu["nmse"][1], ref["nmse_next"]) < NMSE_TOL, (gpu["nmse"][1], ref["nmse_next"])
    assert np.allclose(gpu["field"], slm.amplitude_value(gpu["levels"], L), rtol=0, atol=1e-6)
    if weighted:
        assert rel_l2(gpu["weights"], ref["weights"]) < FIELD_TOL
    say(f"  R rel L2 {er:.2e}, g rel L2 {eg:.2e}, nmse {gpu['nmse'][0]:.5f} -> {gpu['nmse'][1]:.5f}")


@pytest.mark.parametrize("n,weighted", [(64, False), (512, False), (1024, True)])
def test_amplitude_batched_lockstep_mixed_with_phase(n, weighted):
    """One size class holding amplitude (binary, 4 levels) and phase
    (8 levels) problems: three iterations of each checked problem in
    lock-step from the state the batched call reached."""
    say("amplitude batch lock-step", n, "wgs" if weighted else "gs")
    kinds = [(2, True), (8, False), (4, True), (2, True)]
    B = len(kinds)
    Ts = [synth.gaussian_target(n, seed=32, batch_item=b) for b in range(B)]
    seeds = [80 + b for b in range(B)]
    tg = [dev(t) for t in Ts]
    prev = {}
    for k in range(1, 4):
        wts = [torch.ones((n, n), dtype=torch.float32, device=DEV) for _ in range(B)] if weighted else None
        # one batched call per k; each problem its own slm_levels (phase or amplitude)
        levels, nmses = hg.hg_gs_batched(tg, k, [L | (AMP if amp else 0) for L, amp in kinds], seeds=seeds,
                                         weighted=weighted, weights=wts)
        for b, (L, amp) in enumerate(kinds):
            lev_k, nm_k = host(levels[b]).astype(np.int64), host(nmses[b])
            w_k = host(wts[b]).astype(np.float64) if weighted else None
            if k == 1:
                ref = hologram.gs(Ts[b], 1, L, seed=seeds[b], batch_item=b, weighted=weighted, amplitude=amp)
                r_lev, r_g, r_nm, r_w = ref["levels"], ref["g"], ref["nmse"][0], ref["weights"]
            else:
                lev_p, w_p = prev[b]
                T = hologram.prepare_target(Ts[b], L, amplitude=amp)
                f = slm.amplitude_value(lev_p, L) + 0j if amp else slm.level_phasor(lev_p, L)
                st = hologram.gs_step(T, L, f, weighted=weighted, w_prev=w_p, next_nmse=False, amplitude=amp)
                r_lev, r_g, r_nm, r_w = st["levels"], st["g"], st["nmse"], st["weights"]
            where = f"problem {b} ({'amplitude' if amp else 'phase'} L={L}) iteration {k}"
            bad, _ = level_check(lev_k, r_lev, r_g, L, where=where, amplitude=amp)
            assert bad == 0, where
            assert _rel(nm_k[k - 1], r_nm) < NMSE_TOL, (where, nm_k[k - 1], r_nm)
            if weighted:
                assert rel_l2(w_k, r_w) < FIELD_TOL, where
            prev[b] = (lev_k, w_k)
    say(f"  final nmse {[round(float(host(x)[-1]), 4) for x in nmses]}")
