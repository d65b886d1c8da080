"""Pins for the oracle's amplitude-modulating SLM (binary and multi-level
amplitude schemes of the Background section).

Each check is fixed by something other than the oracle's own formula: the
projection is compared with an exhaustive search over every transmission
level, its decision margin with a brute-force minimum over every boundary
and with moves across it, the GS loop with the error-reduction property of
alternating nearest-point projections (which holds with the zero order left
free), the symmetrisation with the centro-symmetry of any real field's
replay, the zero-order freedom with the transform of g, and the GS result
with an exhaustive search over every binary amplitude pattern of a 4 x 4
grid.
"""
import itertools

import numpy as np
import pytest

from oracle import dft, hologram, slm
import synth


def _nonincreasing(e, rel=1e-10):
    e = np.asarray(e)
    return np.all(e[1:] <= e[:-1] * (1 + rel) + 1e-12)


def _random_g(n, seed, spread=1.5):
    rng = np.random.default_rng(seed)
    return rng.normal(0.4, spread, n) + 1j * rng.normal(0, spread, n)


@pytest.mark.parametrize("L", [2, 3, 4, 8, 16, 256])
def test_amplitude_projection_is_nearest_level(L):
    g = _random_g(20000, L)
    levels = np.arange(L) / (L - 1)
    d = np.abs(g[:, None] - levels[None, :])  # Euclidean distance to every transmission
    brute = np.argmin(d, axis=1)
    k = slm.amplitude_index(g, L)
    srt = np.sort(d, axis=1)
    clear = srt[:, 1] - srt[:, 0] > 1e-12  # ties are decided by the rounding rule
    assert np.array_equal(k[clear], brute[clear])
    f, k2 = slm.project_amplitude(g, L)
    assert np.array_equal(k2, k) and np.allclose(f, levels[k]) and np.all(np.imag(f) == 0)


@pytest.mark.parametrize("L", [2, 3, 4, 8, 16, 256])
def test_amplitude_margin_brute_force_and_crossing(L):
    g = _random_g(5000, 100 + L, spread=0.6)
    bounds = (np.arange(L - 1) + 0.5) / (L - 1)
    brute = np.min(np.abs(np.real(g)[:, None] - bounds[None, :]), axis=1)
    m = slm.amplitude_margin(g, L)
    assert np.allclose(m, brute, rtol=0, atol=1e-12)
    # moving Re g toward the nearest boundary by less than the margin keeps the
    # level, by more changes it
    x = np.real(g)
    nearest = bounds[np.argmin(np.abs(x[:, None] - bounds[None, :]), axis=1)]
    sgn = np.sign(nearest - x)
    ok = m > 1e-6
    k0 = slm.amplitude_index(g, L)
    inside = slm.amplitude_index(g + sgn * (m - 1e-9), L)
    across = slm.amplitude_index(g + sgn * (m + 1e-9), L)
    assert np.array_equal(inside[ok], k0[ok])
    assert np.all(across[ok] != k0[ok])


@pytest.mark.parametrize("L", [2, 4, 8])
@pytest.mark.parametrize("optics", [None, (532e-9, 8e-6, 0.01)])
def test_amplitude_gs_error_never_increases(L, optics):
    """Both steps are nearest-point maps (replay: amplitude T off the zero
    order, zero order free; SLM: nearest transmission) and the transform is
    unitary, so the replay error off the zero order never increases."""
    T = synth.gaussian_target(32, seed=5)
    out = hologram.gs(T, 25, L, seed=3, amplitude=True, optics=optics)
    assert _nonincreasing(out["fienup"]), out["fienup"]
    assert out["fienup"][-1] < 0.5 * out["fienup"][0]


def test_real_field_replay_is_centro_symmetric_and_target_symmetrised():
    rng = np.random.default_rng(4)
    a = slm.amplitude_value(rng.integers(0, 5, (16, 32)), 5)
    R = hologram.forward(a)
    A = np.abs(R)
    assert np.allclose(A, hologram.mirror(A), rtol=0, atol=1e-12)
    T = hologram.prepare_target(synth.gaussian_target(32, seed=6, ny=16), 5, amplitude=True)
    assert np.allclose(T, hologram.mirror(T), rtol=0, atol=1e-12)


def test_zero_order_is_free_and_the_rest_constrained():
    """After one amplitude GS step the transform of g is the replay at the
    zero order and has amplitude T everywhere else."""
    T = hologram.prepare_target(synth.gaussian_target(32, seed=7), 4, amplitude=True)
    rng = np.random.default_rng(8)
    f = slm.amplitude_value(rng.integers(0, 4, T.shape), 4) + 0j
    st = hologram.gs_step(T, 4, f, amplitude=True)
    Rg = hologram.forward(st["g"])
    dc = hologram.zero_order(*T.shape)
    assert abs(Rg[dc] - st["replay"][dc]) < 1e-9 * abs(st["replay"][dc])
    off = np.ones(T.shape, bool)
    off[dc] = False
    assert np.allclose(np.abs(Rg)[off], T[off], rtol=0, atol=1e-9)
    # the nmse leaves the zero order out: changing the target there changes nothing
    T2 = T.copy()
    T2[dc] = 123.0
    assert hologram.gs_step(T2, 4, f, amplitude=True)["nmse"] == pytest.approx(st["nmse"], rel=1e-12)


def test_binary_amplitude_gs_bounded_by_exhaustive_search():
    """4 x 4 binary amplitude: no pattern beats the exhaustive minimum of the
    replay error off the zero order, and GS reaches a pattern no better."""
    out = hologram.gs(synth.uniform_target(4, 4, seed=9), 20, 2, seed=1, amplitude=True)
    T = out["target"]
    dc = hologram.zero_order(4, 4)
    off = np.ones((4, 4), bool)
    off[dc] = False
    best = np.inf
    for bits in itertools.product((0.0, 1.0), repeat=16):
        A = np.abs(dft.centre(dft.dft2(np.array(bits).reshape(4, 4))))
        best = min(best, float(np.sum(((A - T) ** 2)[off])))
    assert out["fienup"][-1] >= best - 1e-9
    assert np.all(np.isin(out["levels"], (0, 1)))
