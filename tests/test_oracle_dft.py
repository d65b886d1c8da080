"""Pins for the oracle's DFT (Background section, Eqs. fouriertrans2d5c/d)."""
import numpy as np
import pytest

from oracle import dft


@pytest.mark.parametrize("ny,nx", [(8, 16), (32, 64), (16, 16)])
def test_matches_numpy_fft_ortho(ny, nx):
    # independent library pin: numpy's pocketfft with unitary scaling
    rng = np.random.default_rng(1)
    f = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    np.testing.assert_allclose(dft.dft2(f), np.fft.fft2(f, norm="ortho"), rtol=0, atol=1e-12)
    np.testing.assert_allclose(dft.idft2(f), np.fft.ifft2(f, norm="ortho"), rtol=0, atol=1e-12)


def test_matches_literal_double_sum():
    rng = np.random.default_rng(2)
    f = rng.standard_normal((4, 8)) + 1j * rng.standard_normal((4, 8))
    np.testing.assert_allclose(dft.dft2(f), dft.dft2_direct(f), atol=1e-12)


def test_delta_gives_plane_wave():
    ny, nx, y0, x0 = 16, 32, 3, 5
    f = np.zeros((ny, nx), complex)
    f[y0, x0] = 1.0
    v, u = np.mgrid[0:ny, 0:nx]
    expect = np.exp(-2j * np.pi * (u * x0 / nx + v * y0 / ny)) / np.sqrt(nx * ny)
    np.testing.assert_allclose(dft.dft2(f), expect, atol=1e-13)


def test_plane_wave_gives_delta_at_its_frequency():
    # sign convention: e^{+2 pi i (u0 x/Nx + v0 y/Ny)} lands at (v0, u0), not (-v0, -u0)
    ny, nx, v0, u0 = 16, 32, 3, 7
    y, x = np.mgrid[0:ny, 0:nx]
    f = np.exp(2j * np.pi * (u0 * x / nx + v0 * y / ny))
    F = dft.dft2(f)
    expect = np.zeros((ny, nx), complex)
    expect[v0, u0] = np.sqrt(nx * ny)
    np.testing.assert_allclose(F, expect, atol=1e-10)


def test_parseval_and_inverse():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((32, 16)) + 1j * rng.standard_normal((32, 16))
    F = dft.dft2(f)
    assert abs(np.sum(abs(F) ** 2) - np.sum(abs(f) ** 2)) < 1e-9 * np.sum(abs(f) ** 2)
    np.testing.assert_allclose(dft.idft2(F), f, atol=1e-12)


def test_constant_field_centres_on_dc():
    f = np.ones((8, 16), complex)
    Fc = dft.centre(dft.dft2(f))
    assert abs(Fc[4, 8] - np.sqrt(128)) < 1e-12
    Fc[4, 8] = 0
    assert np.max(abs(Fc)) < 1e-12
    np.testing.assert_allclose(dft.uncentre(dft.centre(f)), f)
