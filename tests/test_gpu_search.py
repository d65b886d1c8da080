"""Holographic search on the GPU (hg_search) against the FP64 oracle.

Direct search and simulated annealing make sequential accept / reject
decisions from the sign of an error change (and, for annealing, Philox
draws that both sides compute bit for bit), so on small grids the GPU
follows the oracle's trajectory exactly: identical final levels and sweep
counts, errors to 1e-5.  On a batch of larger holograms, where the oracle's
own search would take minutes, each GPU result is checked for what is
unique about it: its error equals the oracle's FP64 error of its levels,
and no single-pixel change lowers that error (a direct-search optimum).
"""
import numpy as np
import pytest

import synth
from oracle import dft, hologram, search, slm
from parity import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2008_12214_amd as hg  # noqa: E402

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _error(levels, T, L):
    R = dft.centre(dft.dft2(slm.level_phasor(levels, L)))
    return float(np.sum((np.abs(R) - T) ** 2))


@pytest.mark.parametrize("ny,nx,L", [(8, 8, 2), (16, 16, 2), (16, 16, 4), (32, 16, 3), (8, 32, 8)])
def test_direct_search_follows_the_oracle(ny, nx, L):
    say("direct search", ny, nx, L)
    B = 2
    Ts = [synth.gaussian_target(nx, seed=51, batch_item=b, ny=ny) if ny >= 16 and nx >= 16
          else synth.uniform_target(ny, nx, seed=51 + b) for b in range(B)]
    init = np.random.default_rng(ny * nx + L).integers(0, L, (B, ny, nx))
    out = hg.hg_search(dev(np.stack(Ts)), L, hg.HG_SEARCH_DS, 60, dev(init.astype(np.uint8)))
    lev, err, sw = host(out["levels"]), host(out["error"]), host(out["sweeps"])
    for b in range(B):
        T = hologram.prepare_target(Ts[b], L)
        ref_lev, ref_err, ref_sw = search.direct_search(T, L, init[b], max_sweeps=60)
        assert np.array_equal(lev[b], ref_lev), (b, int(np.sum(lev[b] != ref_lev)))
        assert sw[b] == ref_sw, (sw[b], ref_sw)
        assert abs(err[b, sw[b]] - ref_err) <= 1e-5 * ref_err, (err[b, sw[b]], ref_err)
        assert abs(err[b, 0] - _error(init[b], T, L)) <= 1e-5 * err[b, 0]
        say(f"  problem {b}: {sw[b]} sweeps, error {err[b, 0]:.3f} -> {err[b, sw[b]]:.3f}")


@pytest.mark.parametrize("ny,nx,L,t0,alpha", [(16, 16, 2, 2.0, 0.7), (16, 32, 4, 1.0, 0.8), (32, 32, 2, 3.0, 0.85)])
def test_simulated_annealing_follows_the_oracle(ny, nx, L, t0, alpha):
    say("simulated annealing", ny, nx, L, t0, alpha)
    sweeps, seed = 8, 77
    B = 2
    Ts = [synth.gaussian_target(nx, seed=52, batch_item=b, ny=ny) for b in range(B)]
    init = np.random.default_rng(ny + nx + L).integers(0, L, (B, ny, nx))
    out = hg.hg_search(dev(np.stack(Ts)), L, hg.HG_SEARCH_SA, sweeps, dev(init.astype(np.uint8)), t0=t0,
                       alpha=alpha, seed=seed)
    lev, err = host(out["levels"]), host(out["error"])
    for b in range(B):
        T = hologram.prepare_target(Ts[b], L)
        ref_lev, ref_err, acc = search.simulated_annealing(T, L, init[b], sweeps, t0, alpha, seed=seed, batch_item=b)
        assert np.array_equal(lev[b], ref_lev), (b, int(np.sum(lev[b] != ref_lev)))
        assert np.max(np.abs(err[b] - ref_err) / ref_err) <= 1e-5, (err[b], ref_err)
        # the temperature mattered: at zero temperature the same draws lead elsewhere
        cold_lev, _, _ = search.simulated_annealing(T, L, init[b], sweeps, 0.0, alpha, seed=seed, batch_item=b)
        assert not np.array_equal(cold_lev, ref_lev)
        say(f"  problem {b}: {acc} accepted, error {err[b, 0]:.3f} -> {err[b, -1]:.3f}")


def test_direct_search_batch_results_are_local_optima():
    """64 holograms of 64 x 32 pixels, binary: the error of each result equals
    the oracle's error of its levels, and on three of them no single-pixel
    change lowers it."""
    B, ny, nx, L = 64, 64, 32, 2
    say("direct search batch", B, ny, nx)
    Ts = np.stack([synth.gaussian_target(nx, seed=53, batch_item=b, ny=ny) for b in range(B)])
    init = np.random.default_rng(5).integers(0, L, (B, ny, nx))
    out = hg.hg_search(dev(Ts), L, hg.HG_SEARCH_DS, 40, dev(init.astype(np.uint8)))
    lev, err, sw = host(out["levels"]), host(out["error"]), host(out["sweeps"])
    assert np.all(sw < 40)
    for b in range(B):
        T = hologram.prepare_target(Ts[b], L)
        e = _error(lev[b], T, L)
        assert abs(err[b, sw[b]] - e) <= 1e-5 * e, (b, err[b, sw[b]], e)
        assert err[b, sw[b]] < err[b, 0]
    for b in (0, 31, 63):
        T = hologram.prepare_target(Ts[b], L)
        R = dft.centre(dft.dft2(slm.level_phasor(lev[b], L)))
        e = float(np.sum((np.abs(R) - T) ** 2))
        f = slm.level_phasor(lev[b], L)  # binary: flipping pixel (y, x) changes it by -2 f
        worst = np.inf
        for y in range(ny):
            for x in range(nx):
                d = np.zeros((ny, nx), dtype=np.complex128)
                d[y, x] = 1.0
                kern = dft.centre(dft.dft2(d))
                Rn = R - 2.0 * f[y, x] * kern
                worst = min(worst, float(np.sum((np.abs(Rn) - T) ** 2)) - e)
        assert worst > -1e-6 * e, (b, worst)
        say(f"  problem {b}: {sw[b]} sweeps, error {err[b, 0]:.2f} -> {err[b, sw[b]]:.2f}, best single flip {worst:+.4f}")
