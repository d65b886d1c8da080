"""Pins for the oracle's 16-bit field storage model (Floating Points
section: 16-bit builds).

The staged transforms are checked against the plain unitary pair with the
rounding switched off; the rounding is checked against IEEE binary16
round-to-nearest-even values derived by hand (ties, overflow, subnormals);
the power-of-two scale is checked to change no mantissa; and one stored
plane is checked against the binary16 error bound.
"""
import numpy as np
import pytest

from oracle import hologram
import synth


def _identity(Z, scale):
    return np.asarray(Z, dtype=np.complex128)


@pytest.mark.parametrize("ny,nx,optics", [(16, 16, None), (16, 32, None), (32, 8, (532e-9, 8e-6, 0.01))])
def test_staged_transforms_equal_the_unitary_pair_without_rounding(ny, nx, optics):
    rng = np.random.default_rng(ny * nx)
    f = rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))
    Q = hologram.fresnel_chirp(ny, nx, *optics) if optics else None
    assert np.allclose(hologram.forward16(f, Q, store=_identity), hologram.forward(f, Q), rtol=0, atol=1e-12)
    assert np.allclose(hologram.backward16(f, Q, store=_identity), hologram.backward(f, Q), rtol=0, atol=1e-12)


def test_store16_is_ieee_binary16_round_to_nearest_even():
    u = 2.0 ** -10  # binary16 spacing just above 1
    cases = [
        (1.0 + u / 2, 1.0),            # a tie rounds to the even mantissa
        (1.0 + 1.5 * u, 1.0 + 2 * u),  # a tie above an odd mantissa rounds up
        (1.0 + 0.49 * u, 1.0),
        (1.0 + 0.51 * u, 1.0 + u),
        (65504.0, 65504.0),            # the largest finite value
        (65520.0, np.inf),             # half a spacing above it overflows
        (2.0 ** -24, 2.0 ** -24),      # the smallest subnormal
        (2.0 ** -26, 0.0),             # a quarter of it rounds to zero
        (-(1.0 + 1.5 * u), -(1.0 + 2 * u)),
    ]
    for x, want in cases:
        got = hologram.store16(np.array([x + 1j * x]), 1.0)[0]
        assert got.real == want and got.imag == want, (x, got, want)


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024, 2048, 4096])
def test_half_scale_is_a_power_of_two_that_changes_no_mantissa(n):
    s = hologram.half_scale(n)
    assert s == 2.0 ** -(int(np.log2(n)) // 2) and np.log2(s) == int(np.log2(s))
    Z = np.random.default_rng(n).normal(size=1000) * 30 + 1j * np.random.default_rng(n + 1).normal(size=1000) * 30
    assert np.array_equal(hologram.store16(Z, s), hologram.store16(Z, 1.0))


def test_one_stored_plane_is_within_the_binary16_bound():
    T = hologram.prepare_target(synth.gaussian_target(64, seed=3), 8)
    f = np.exp(2j * np.pi * np.random.default_rng(5).random(T.shape))
    R64, R16 = hologram.forward(f), hologram.forward16(f)
    # each stored component carries a relative error of at most 2^-11; the
    # unitary column transform preserves the L2 norm of the error
    assert np.linalg.norm(R16 - R64) / np.linalg.norm(R64) <= 2.0 ** -11
    assert np.linalg.norm(R16 - R64) / np.linalg.norm(R64) > 0.0
    g64 = hologram.backward(T * np.exp(1j * np.angle(R64)))
    g16 = hologram.backward16(T * np.exp(1j * np.angle(R64)))
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) <= 2.0 ** -11
    # a continuous-phase GS iteration: the NMSE moves by rounding only
    a = hologram.gs(synth.gaussian_target(64, seed=3), 2, 0, seed=1)
    b = hologram.gs(synth.gaussian_target(64, seed=3), 2, 0, seed=1, field16=True)
    assert np.max(np.abs(a["nmse"] - b["nmse"]) / a["nmse"]) < 1e-3
