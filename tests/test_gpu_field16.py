"""16-bit field storage on the GPU against the FP64 oracle's storage model.

With slm_levels | HG_FIELD_FP16 the field between the row and column passes
is held as two binary16 values per element; the oracle rounds at the same
points (hologram.forward16 / backward16).  The two sides still differ where
their values straddle a binary16 rounding boundary, which the replay
constraint amplifies, so fields are held to one binary16 step (2^-11
relative L2), the NMSE to 1e-4, and levels with a 50 times wider distance
band (parity.FIELD16_TOL, FIELD16_BAND, derived there).  Cases cover the three column lengths
the storage supports, staged 1024- and 2048-wide rows and unstaged ones,
Fresnel, weighted GS, Liu-Taghizadeh and an amplitude SLM, and a batched
call in lock-step.
"""
import numpy as np
import pytest

import synth
from oracle import hologram, slm
from parity import FIELD16_BAND, FIELD16_TOL, NMSE_TOL, level_check, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"
F16 = hg.HG_FIELD_FP16


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rel(a, b):
    return abs(float(a) - float(b)) / abs(float(b))


# (ny, nx, L, weighted, Fresnel z or None, LT radius or None, amplitude)
CASES = [(256, 256, 8, False, None, None, False), (512, 1024, 2, True, 0.3, None, False),
         (1024, 1024, 2, True, None, None, False), (256, 2048, 4, False, None, None, False),
         (1024, 512, 16, False, 0.2, None, False), (512, 512, 2, False, None, 60, False),
         (1024, 1024, 4, True, None, None, True)]


@pytest.mark.parametrize("ny,nx,L,weighted,z,lt,amp", CASES)
def test_field16_step_matches_oracle(ny, nx, L, weighted, z, lt, amp):
    say("16-bit storage hg_gs_step", ny, nx, L, "wgs" if weighted else "gs", z, lt, "amplitude" if amp else "")
    T_raw = synth.gaussian_target(nx, seed=41, ny=ny)
    T = hologram.prepare_target(T_raw, L, amplitude=amp)
    rng = np.random.default_rng(ny + nx + L)
    lev = rng.integers(0, L, (ny, nx))
    f = slm.amplitude_value(lev, L) + 0j if amp else slm.level_phasor(lev, L)
    w = rng.uniform(0.5, 2.0, (ny, nx)) if weighted else None
    optics = (synth.WAVELENGTH_M, synth.PITCH_M, z) if z else (0.0, 0.0, 0.0)
    flags = F16 | (hg.HG_SLM_AMPLITUDE if amp else 0)
    out = hg.hg_gs_step(dev(T_raw), L | flags, levels_in=dev(lev.astype(np.uint8)),
                        weights=None if w is None else dev(w.astype(np.float32)),
                        lt_radius=-1 if lt is None else lt, wavelength_m=optics[0], pitch_m=optics[1], z_m=optics[2])
    gpu = {k: (None if v is None else host(v)) for k, v in out.items()}
    ref = hologram.gs_step(T, L, f, weighted=weighted, w_prev=w, optics=optics if z else None, lt_r=lt,
                           amplitude=amp, field16=True)
    er, eg = rel_l2(gpu["replay"], ref["replay"]), rel_l2(gpu["g"], ref["g"])
    assert er < FIELD16_TOL and eg < FIELD16_TOL, (er, eg)
    bad, _ = level_check(gpu["levels"], ref["levels"], ref["g"], L, where="16-bit step", amplitude=amp,
                         band_scale=FIELD16_BAND)
    assert bad == 0
    assert _rel(gpu["nmse"][0], ref["nmse"]) < NMSE_TOL, (gpu["nmse"][0], ref["nmse"])
    assert _rel(gpu["nmse"][1], ref["nmse_next"]) < NMSE_TOL, (gpu["nmse"][1], ref["nmse_next"])
    if weighted:
        assert rel_l2(gpu["weights"], ref["weights"]) < FIELD16_TOL
    # the same step with complex64 storage differs from it by the storage
    # rounding only: about 2^-11 per stored element, amplified in g by the
    # constraint's division by |R| and by the weights (up to about 3e-3 here)
    out32 = hg.hg_gs_step(dev(T_raw), L | (hg.HG_SLM_AMPLITUDE if amp else 0), levels_in=dev(lev.astype(np.uint8)),
                          weights=None if w is None else dev(w.astype(np.float32)),
                          lt_radius=-1 if lt is None else lt, wavelength_m=optics[0], pitch_m=optics[1], z_m=optics[2])
    d16 = rel_l2(gpu["g"], host(out32["g"]))
    assert 0.0 < d16 < 2.0 ** -6, d16
    say(f"  R rel L2 {er:.2e}, g rel L2 {eg:.2e}, 16-bit vs complex64 storage {d16:.2e}, "
        f"nmse {gpu['nmse'][0]:.5f} -> {gpu['nmse'][1]:.5f}")


@pytest.mark.parametrize("n,B,L,weighted", [(1024, 32, 2, True), (512, 8, 8, False)])
def test_field16_batched_lockstep(n, B, L, weighted):
    """Iterations 1-3 of the first and last problem of a batched call with
    16-bit storage, each in lock-step with the oracle from the state the call
    reached."""
    say("16-bit storage batch lock-step", n, B, L, "wgs" if weighted else "gs")
    Ts = [synth.gaussian_target(n, seed=42, batch_item=b) for b in range(B)]
    seeds = [90 + b for b in range(B)]
    tg = [dev(t) for t in Ts]
    prev = {}
    for k in range(1, 4):
        wts = [torch.ones((n, n), dtype=torch.float32, device=DEV) for _ in range(B)] if weighted else None
        levels, nmses = hg.hg_gs_batched(tg, k, L | F16, seeds=seeds, weighted=weighted, weights=wts)
        for b in (0, B - 1):
            lev_k, nm_k = host(levels[b]).astype(np.int64), host(nmses[b])
            w_k = host(wts[b]).astype(np.float64) if weighted else None
            if k == 1:
                ref = hologram.gs(Ts[b], 1, L, seed=seeds[b], batch_item=b, weighted=weighted, field16=True)
                r_lev, r_g, r_nm, r_w = ref["levels"], ref["g"], ref["nmse"][0], ref["weights"]
            else:
                lev_p, w_p = prev[b]
                st = hologram.gs_step(hologram.prepare_target(Ts[b], L), L, slm.level_phasor(lev_p, L),
                                      weighted=weighted, w_prev=w_p, next_nmse=False, field16=True)
                r_lev, r_g, r_nm, r_w = st["levels"], st["g"], st["nmse"], st["weights"]
            where = f"problem {b} iteration {k}"
            bad, _ = level_check(lev_k, r_lev, r_g, L, where=where, band_scale=FIELD16_BAND)
            assert bad == 0, where
            assert _rel(nm_k[k - 1], r_nm) < NMSE_TOL, (where, nm_k[k - 1], r_nm)
            if weighted:
                assert rel_l2(w_k, r_w) < FIELD16_TOL, where
            prev[b] = (lev_k, w_k)
    say(f"  nmse after 3 iterations {float(host(nmses[0])[-1]):.5f}, {float(host(nmses[-1])[-1]):.5f}")


def test_field16_rejects_other_column_lengths():
    T = dev(synth.gaussian_target(2048, seed=1))
    with pytest.raises(hg.HologenError) as e:
        hg.hg_gs(T, 2, 2 | F16)
    assert e.value.status == hg.HG_ERR_UNSUPPORTED_SIZE
