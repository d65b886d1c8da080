"""Pins for the oracle's OSPR / adaptive OSPR (Time-Averaged Algorithms section)."""
import numpy as np
import pytest

from oracle import hologram, philox
import synth


def test_ospr_energy_and_symmetry():
    T = synth.gaussian_target(32, seed=3)
    out = hologram.ospr(T, 6, adaptive=False, seed=11)
    n = 6
    # each binary subframe is unit modulus, so the mean replay intensity is 1 (Parseval)
    assert np.mean(out["accum"] / n) == pytest.approx(1.0, rel=1e-12)
    A = out["accum"]
    np.testing.assert_allclose(A, hologram.mirror(A), rtol=1e-9)
    assert out["levels"].shape == (6, 32, 32)
    assert set(np.unique(out["levels"])) <= {0, 1}


def test_ospr_subframe_phase_is_philox():
    T = synth.gaussian_target(16, seed=1)
    out = hologram.ospr(T, 1, adaptive=False, seed=5)
    Tp = hologram.prepare_target(T, 2)
    phi = philox.phase_field(5, philox.TAG_OSPR + 1, 16, 16)
    g = hologram.backward(Tp * np.exp(1j * phi))
    np.testing.assert_array_equal(out["levels"][0], (g.real < 0).astype(int))


def test_time_average_error_falls_reciprocally():
    # Eq. MSEdecline: the time-averaged error falls reciprocally with the
    # number of subframes.  The noise term of the averaged intensity falls
    # as 1/n for independent subframes; fit the log-log slope after
    # removing the n -> infinity floor estimated from many subframes.
    T = synth.gaussian_target(32, seed=8)
    out = hologram.ospr(T, 64, adaptive=False, seed=21)
    Tp = out["target"]
    # error of the averaged intensity against the infinite-average intensity
    big = hologram.ospr(T, 256, adaptive=False, seed=99)["accum"] / 256.0
    errs = []
    lv = out["levels"]
    ns = np.array([1, 2, 4, 8, 16, 32, 64])
    for n in ns:
        acc = np.zeros_like(Tp)
        for i in range(n):
            acc += np.abs(hologram.forward(np.where(lv[i] == 1, -1.0, 1.0))) ** 2
        errs.append(np.mean((acc / n - big) ** 2))
    slope = np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert -1.25 < slope < -0.75, slope
    # the reported NMSE falls with n
    assert out["nmse"][-1] < out["nmse"][0]


def test_adaptive_beats_plain_ospr():
    T = synth.gaussian_target(32, seed=9)
    plain = hologram.ospr(T, 24, adaptive=False, seed=3)
    adapt = hologram.ospr(T, 24, adaptive=True, seed=3)
    assert adapt["nmse"][-1] < plain["nmse"][-1]
    assert np.mean(adapt["accum"] / 24) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("n", [2, 3, 7, 24])
def test_adaptive_feedback_completes_the_target(n):
    """Adaptive OSPR's feedback (the reading of the Time-Averaged Algorithms
    section): subframe n asks for exactly the intensity that, added to the
    n - 1 subframes already accumulated, makes their average the target,
    (A_{n-1} + T_n^2) / n = T^2, wherever that is possible (deficit >= 0),
    and for nothing where the pixel is already too bright.  A_{n-1} is drawn
    independently of T; an off-by-one in n fails this."""
    rng = np.random.default_rng(n)
    T = rng.uniform(0.0, 2.0, (24, 24))
    A = rng.uniform(0.0, 2.0 * n, (24, 24))
    Tn = hologram.ospr_target(T, A, n, adaptive=True)
    deficit = n * T * T - A
    ok = deficit >= 0
    assert 0.2 < ok.mean() < 0.95
    np.testing.assert_allclose(((A + Tn ** 2) / n)[ok], (T * T)[ok], rtol=1e-12)
    assert np.all(Tn[~ok] == 0.0)
    np.testing.assert_array_equal(hologram.ospr_target(T, A, n, adaptive=False), T)
    np.testing.assert_array_equal(hologram.ospr_target(T, np.zeros_like(T), 1, adaptive=True), T)
