"""Pins for the oracle's GS, weighted GS, Fresnel and search loops.

Each check is fixed by the mathematics, not by re-typing the oracle:
alternating projections never increase the unscaled replay error (the DFT
is unitary and both constraint steps are nearest-point maps), a binary
replay is centro-symmetric, a consistent target is a fixed point, scale
freedom leaves the iterates unchanged, a lens phase focuses to a point, and
brute-force search bounds what GS can reach on tiny grids.
"""
import numpy as np
import pytest

from oracle import dft, hologram, philox, search, slm
import synth


def _nonincreasing(e, rel=1e-10):
    e = np.asarray(e)
    return np.all(e[1:] <= e[:-1] * (1 + rel) + 1e-12)


@pytest.mark.parametrize("L", [0, 2, 4, 8])
def test_gs_error_never_increases(L):
    T = synth.uniform_target(32, 32, seed=1)
    out = hologram.gs(T, 30, L, seed=1)
    assert _nonincreasing(out["fienup"]), out["fienup"]
    assert out["fienup"][-1] < out["fienup"][0]


def test_gs_error_never_increases_fresnel():
    T = synth.gaussian_target(32, seed=4)
    out = hologram.gs(T, 20, 8, seed=2, optics=(532e-9, 8e-6, 0.01))
    assert _nonincreasing(out["fienup"])


def test_gs_consistent_target_is_fixed_point():
    rng = np.random.default_rng(0)
    theta = rng.uniform(0, 2 * np.pi, (16, 32))
    f0 = np.exp(1j * theta)
    T = np.abs(hologram.forward(f0)).astype(np.float32)
    out = hologram.gs(T, 5, 0, init_field=f0)
    assert np.max(out["nmse"]) < 1e-6
    np.testing.assert_allclose(out["field"], f0, atol=1e-3)
    # weighted GS on a consistent target keeps ratio ~1, so it follows GS
    outw = hologram.gs(T, 5, 0, init_field=f0, weighted=True)
    assert np.max(outw["nmse"]) < 1e-6
    np.testing.assert_allclose(outw["weights"], 1.0, atol=1e-3)


@pytest.mark.parametrize("weighted", [False, True])
def test_scale_freedom(weighted):
    T = synth.gaussian_target(32, seed=5)
    a = hologram.gs(T, 10, 8, seed=3, weighted=weighted)
    b = hologram.gs(T * np.float32(8.0), 10, 8, seed=3, weighted=weighted)  # exact in float32
    np.testing.assert_array_equal(a["levels"], b["levels"])
    np.testing.assert_allclose(a["nmse"], b["nmse"], rtol=1e-12)
    c = hologram.gs(T.astype(np.float64) * 7.5, 10, 8, seed=3, weighted=weighted)
    np.testing.assert_array_equal(a["levels"], c["levels"])
    np.testing.assert_allclose(a["nmse"], c["nmse"], rtol=1e-10)


def test_prepare_target_energy_and_binary_symmetry():
    T = synth.gaussian_target(64, seed=2)
    Tp = hologram.prepare_target(T, 8)
    assert np.sum(Tp ** 2) == pytest.approx(64 * 64, rel=1e-12)
    Tb = hologram.prepare_target(T, 2)
    np.testing.assert_allclose(Tb, hologram.mirror(Tb), rtol=1e-14)
    assert np.sum(Tb ** 2) == pytest.approx(64 * 64, rel=1e-12)


def test_binary_replay_is_centrosymmetric():
    rng = np.random.default_rng(4)
    h = np.where(rng.random((16, 32)) < 0.5, 1.0, -1.0)
    A = np.abs(hologram.forward(h))
    np.testing.assert_allclose(A, hologram.mirror(A), atol=1e-12)


def test_weighted_binary_weights_stay_symmetric():
    T = synth.gaussian_target(32, seed=6)
    # from a binary start every replay is centro-symmetric, so are the weights
    init = (philox.u24(philox.line_words(3, 1, 32, 32, 1)) < 0.5).astype(np.int64)
    out = hologram.gs(T, 8, 2, init_levels=init, weighted=True)
    np.testing.assert_allclose(out["weights"], hologram.mirror(out["weights"]), rtol=1e-9)
    assert out["m"] > 0


def test_resume_equals_uninterrupted():
    T = synth.gaussian_target(32, seed=7)
    full = hologram.gs(T, 8, 4, seed=9, weighted=True)
    a = hologram.gs(T, 5, 4, seed=9, weighted=True)
    b = hologram.gs(T, 3, 4, init_levels=a["levels"], weighted=True, weights=a["weights"])
    np.testing.assert_array_equal(full["levels"], b["levels"])
    np.testing.assert_allclose(full["nmse"][5:], b["nmse"], rtol=1e-10)


def test_initial_phase_is_philox_draw():
    T = synth.uniform_target(8, 16, seed=1)
    out = hologram.gs(T, 1, 0, seed=77)
    f0 = np.exp(1j * philox.phase_field(77, philox.TAG_INIT, 8, 16))
    R0 = hologram.forward(f0)
    assert out["nmse"][0] == pytest.approx(
        1 - np.sum(hologram.prepare_target(T, 0) * abs(R0)) ** 2 / (128 * np.sum(abs(R0) ** 2)), rel=1e-12)


def test_lens_phase_focuses_to_centre():
    ny, nx = 32, 64
    lam, p, z = 532e-9, 8e-6, 0.05
    Q = hologram.fresnel_chirp(ny, nx, lam, p, z)
    R = hologram.fresnel_propagate(np.conj(Q), lam, p, z, +1)
    expect = np.zeros((ny, nx), complex)
    expect[ny // 2, nx // 2] = np.sqrt(nx * ny)
    np.testing.assert_allclose(R, expect, atol=1e-9)


def test_fresnel_round_trip_and_far_field_limit():
    rng = np.random.default_rng(8)
    f = rng.standard_normal((16, 32)) + 1j * rng.standard_normal((16, 32))
    R = hologram.fresnel_propagate(f, 532e-9, 8e-6, 0.2, +1)
    np.testing.assert_allclose(hologram.fresnel_propagate(R, 532e-9, 8e-6, 0.2, -1), f, atol=1e-12)
    far = hologram.fresnel_propagate(f, 532e-9, 8e-6, np.inf, +1)
    np.testing.assert_allclose(far, np.fft.fftshift(np.fft.fft2(f, norm="ortho")), atol=1e-12)
    # the chirp is separable in centred coordinates
    Q = hologram.fresnel_chirp(16, 32, 532e-9, 8e-6, 0.2)
    np.testing.assert_allclose(Q, np.outer(Q[:, 16], Q[8, :]), atol=1e-12)


def test_search_incremental_update_matches_recompute():
    T = hologram.prepare_target(synth.uniform_target(4, 4, seed=3), 2)
    lev = np.zeros((4, 4), np.int64)
    lev2 = lev.copy()
    lev2[1, 2] = 1
    kern = search._kernel(4, 4, 1, 2)
    R = dft.centre(dft.dft2(slm.level_phasor(lev, 2)))
    Rn = R + (slm.level_phasor(np.array(1), 2) - slm.level_phasor(np.array(0), 2)) * kern
    np.testing.assert_allclose(Rn, dft.centre(dft.dft2(slm.level_phasor(lev2, 2))), atol=1e-12)


@pytest.mark.parametrize("L", [2, 4])
def test_brute_force_bounds_gs_and_ds_on_4x4(L):
    T = hologram.prepare_target(synth.uniform_target(4, 4, seed=12), L)
    if L == 2:
        best, e_best = search.exhaustive(T, L)
    else:
        best, e_best = search.exhaustive(T, L, free=range(8))
    out = hologram.gs(T, 30, L, seed=4)
    T = out["target"]
    e_gs = out["fienup"][-1]
    lev, e_ds, _ = search.direct_search(T, L, out["levels"])
    if L == 2:
        assert e_best <= e_gs + 1e-9 and e_best <= e_ds + 1e-9
    assert e_ds <= e_gs + 1e-9  # DS from the GS result can only improve it
    # DS output is a local minimum under every single-pixel change
    for y in range(4):
        for x in range(4):
            for k in range(L):
                t = lev.copy()
                t[y, x] = k
                assert search.replay_error(t, T, L) >= e_ds - 1e-9


def test_direct_search_on_8x8_reaches_local_minimum():
    T = hologram.prepare_target(synth.gaussian_target(8, seed=3), 2)
    init = (philox.u24(philox.line_words(5, 1, 8, 8, 1)) < 0.5).astype(np.int64)
    lev, e, sweeps = search.direct_search(T, 2, init)
    assert e <= search.replay_error(init, T, 2)
    for p in range(64):
        t = lev.copy().ravel()
        t[p] ^= 1
        assert search.replay_error(t.reshape(8, 8), T, 2) >= e - 1e-9
    # exhaustive over 16 free pixels around the DS optimum cannot lose to it
    _, e16 = search.exhaustive(T, 2, free=range(16), base_levels=lev)
    assert e16 <= e + 1e-9


@pytest.mark.parametrize("L", [2, 8])
def test_weighting_improves_convergence(L):
    # Iterative Fourier Transform Algorithms section: weighting is a GS
    # variant that improves convergence; the weights stay bounded
    T = synth.gaussian_target(64, seed=2)
    plain = hologram.gs(T, 40, L, seed=1)
    wgs = hologram.gs(T, 40, L, seed=1, weighted=True)
    assert wgs["nmse"][-1] < plain["nmse"][-1]
    om = wgs["target"] > 0
    assert 1e-4 < wgs["weights"][om].min() and wgs["weights"][om].max() < 1e2


# ---------------------------------------------------------------------------
# Liu-Taghizadeh (growing target region, amplitude freedom outside it)
# ---------------------------------------------------------------------------
def test_lt_full_window_equals_gs():
    T = synth.gaussian_target(32, seed=4)
    a = hologram.gs(T, 4, 8, seed=3)
    b = hologram.gs(T, 4, 8, seed=3, lt=(16, 0))
    np.testing.assert_array_equal(a["levels"], b["levels"])
    np.testing.assert_array_equal(a["nmse"], b["nmse"])


def test_lt_amplitude_free_outside_and_constrained_inside():
    """One continuous-phase LT iteration: the field g that is projected has
    the replay R of the start field outside the window and amplitude T inside
    (the two parts of R' = where(window, T R/|R|, R))."""
    T = synth.gaussian_target(32, seed=5)
    rng = np.random.default_rng(2)
    f0 = np.exp(2j * np.pi * rng.random((32, 32)))
    out = hologram.gs(T, 1, 0, init_field=f0, lt=(6, 0))
    inside = hologram.lt_window(32, 32, 6)
    R0 = hologram.forward(f0)
    Rg = hologram.forward(out["g"])
    Tp = out["target"]
    np.testing.assert_allclose(Rg[~inside], R0[~inside], atol=1e-12)
    np.testing.assert_allclose(np.abs(Rg[inside]), Tp[inside], atol=1e-12)
    assert inside.sum() == 13 * 13


def test_lt_becomes_gs_once_the_window_covers_the_plane():
    """r0 = 8, dr = 4 on 32 x 32: iterations 1 and 2 use radii 8 and 12, the
    third and later cover the whole plane, so they are GS from the state after
    two iterations."""
    T = synth.gaussian_target(32, seed=6)
    full = hologram.gs(T, 5, 4, seed=9, lt=(8, 4))
    head = hologram.gs(T, 2, 4, seed=9, lt=(8, 4))
    tail = hologram.gs(T, 3, 4, init_levels=head["levels"])
    np.testing.assert_array_equal(full["levels"], tail["levels"])
    np.testing.assert_allclose(full["nmse"][2:], tail["nmse"], rtol=0, atol=0)
    # and the growing window differs from plain GS early on
    gs = hologram.gs(T, 5, 4, seed=9)
    assert gs["nmse"][1] != full["nmse"][1]


@pytest.mark.parametrize("L,weighted,lt_r,optics", [(2, True, None, None), (8, False, None, (532e-9, 8e-6, 0.1)),
                                                     (0, False, 5, None), (4, True, None, None)])
def test_gs_step_is_one_iteration_of_gs(L, weighted, lt_r, optics):
    """gs_step (one iteration from a caller's state, the lock-step interface)
    gives the iteration gs() takes from that state; its pre-constraint replay
    is the forward transform of the state."""
    T_raw = synth.gaussian_target(32, seed=4)
    T = hologram.prepare_target(T_raw, L)
    rng = np.random.default_rng(L)
    lev = rng.integers(0, max(L, 2), T.shape)
    f = np.exp(1j * rng.uniform(0, 2 * np.pi, T.shape)) if L == 0 else slm.level_phasor(lev, L)
    w = rng.uniform(0.5, 2.0, T.shape) if weighted else None
    st = hologram.gs_step(T, L, f, weighted=weighted, w_prev=w, optics=optics, lt_r=lt_r)
    ref = hologram.gs(T_raw, 1, L, init_field=f, weighted=weighted, weights=w, optics=optics,
                      lt=None if lt_r is None else (lt_r, 0))
    np.testing.assert_array_equal(st["g"], ref["g"])
    np.testing.assert_array_equal(st["field"], ref["field"])
    assert st["nmse"] == ref["nmse"][0] and st["nmse_next"] == ref["nmse"][1]
    if weighted:
        np.testing.assert_array_equal(st["weights"], ref["weights"])
    Q = hologram.fresnel_chirp(32, 32, *optics) if optics else None
    np.testing.assert_allclose(st["replay"], hologram.forward(f, Q), rtol=0, atol=1e-13)
