"""Pins for the SLM projection (Listing 1) and the error metrics (Eq. mse)."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import slm, metrics
from conftest import golden


def test_listing1_worked_cases():
    rows = [l.split("#")[0].split() for l in open(golden("listing1_quantiser.txt"))]
    rows = [r for r in rows if r]
    assert len(rows) >= 10
    for L, arg, k in rows:
        L, arg, k = int(L), float(arg), int(k)
        g = 3.0 * np.exp(1j * arg)
        assert int(slm.level_index(np.array([g]), L)[0]) == k, (L, arg)


@pytest.mark.parametrize("L", [2, 3, 4, 8, 16, 256])
def test_listing1_formula_on_random_angles(L):
    # the listing's arithmetic (printed constants, roundf = half away from zero)
    pi2 = 6.28318530718
    spac = pi2 / L
    rng = np.random.default_rng(L)
    g = rng.standard_normal(20000) + 1j * rng.standard_normal(20000)
    arg = np.fmod(np.arctan2(g.imag, g.real), pi2)
    r = (arg - 0.0) / spac
    disc = np.sign(r) * np.floor(np.abs(r) + 0.5)
    k_listing = np.mod(disc.astype(np.int64), L)
    ok = slm.boundary_margin(g, L) > 1e-9
    assert ok.mean() > 0.99
    np.testing.assert_array_equal(slm.level_index(g, L)[ok], k_listing[ok])


@pytest.mark.parametrize("L", [2, 3, 5, 8, 64])
def test_projection_is_nearest_point_exhaustive(L):
    rng = np.random.default_rng(11 + L)
    g = rng.standard_normal(5000) + 1j * rng.standard_normal(5000)
    f, k = slm.project(g, L)
    cand = np.exp(2j * np.pi * np.arange(L) / L)
    d = np.abs(g[:, None] - cand[None, :])
    k_best = np.argmin(d, axis=1)
    ok = slm.boundary_margin(g, L) > 1e-9
    np.testing.assert_array_equal(k[ok], k_best[ok])
    np.testing.assert_allclose(np.abs(f), 1.0, atol=1e-15)


def test_projection_rotation_equivariance_and_binary_sign():
    L = 8
    rng = np.random.default_rng(5)
    g = rng.standard_normal(4000) + 1j * rng.standard_normal(4000)
    ok = slm.boundary_margin(g, L) > 1e-6
    k0 = slm.level_index(g, L)
    k1 = slm.level_index(g * np.exp(2j * np.pi / L), L)
    np.testing.assert_array_equal(k1[ok], (k0[ok] + 1) % L)
    kb = slm.level_index(g, 2)
    np.testing.assert_array_equal(kb, (g.real < 0).astype(int))


def test_continuous_projection():
    g = np.array([3 + 4j, 0j, -2.0 + 0j])
    f, k = slm.project(g, 0)
    assert k is None
    np.testing.assert_allclose(f, [0.6 + 0.8j, 1.0, -1.0])


def test_mse_worked_example():
    vals = {}
    for line in open(golden("mse_example.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, *nums = line.split()
        vals[name] = np.array([float(x) for x in nums])
    T = vals["T"].reshape(2, 2)
    R = vals["R"].reshape(2, 2)
    assert metrics.mse(T, R) == pytest.approx(float(vals["E"][0]), abs=1e-15)


def test_nmse_is_scale_optimal_mse():
    rng = np.random.default_rng(3)
    T = rng.random((16, 16))
    A = T * 1.7 + 0.3 * rng.random((16, 16))
    stt = np.sum(T * T)
    # brute-force the best scale of Eq. mse, normalised by the target energy
    res = minimize_scalar(lambda s: metrics.mse(T, s * A) * T.size / stt, bounds=(0, 10),
                          method="bounded", options={"xatol": 1e-12})
    assert metrics.nmse(T, A) == pytest.approx(res.fun, rel=1e-7)
    assert metrics.nmse(T, 3.0 * T) == pytest.approx(0.0, abs=1e-14)
    assert 0.0 <= metrics.nmse(T, rng.random((16, 16))) <= 1.0


@pytest.mark.parametrize("L", [2, 3, 4, 8, 16, 256])
def test_boundary_margin_against_brute_force(L):
    """The parity exemption's margin: the angular distance from arg g to the
    nearest decision boundary (2m + 1) pi / L of the nearest-level rule,
    found here by brute force over all L boundaries on the circle."""
    rng = np.random.default_rng(100 + L)
    g = (rng.standard_normal(3000) + 1j * rng.standard_normal(3000)) * rng.uniform(0.01, 10.0, 3000)
    theta = np.arctan2(g.imag, g.real)
    b = (2 * np.arange(L) + 1) * np.pi / L
    d = np.abs(theta[:, None] - b[None, :]) % (2 * np.pi)
    brute = np.min(np.minimum(d, 2 * np.pi - d), axis=1)
    np.testing.assert_allclose(slm.boundary_margin(g, L), brute, rtol=0, atol=1e-12)
    assert np.all(slm.boundary_margin(np.zeros(3, complex), L) == 0.0)


@pytest.mark.parametrize("L", [2, 3, 4, 8, 16, 256])
def test_boundary_margin_is_the_distance_to_a_level_change(L):
    """Rotating g towards its nearest boundary by just less than the margin
    keeps its level; by just more, it changes the level."""
    rng = np.random.default_rng(200 + L)
    g = rng.standard_normal(2000) + 1j * rng.standard_normal(2000)
    m = slm.boundary_margin(g, L)
    keep = m > 1e-6
    g, m = g[keep], m[keep]
    theta = np.arctan2(g.imag, g.real)
    b = (2 * np.arange(L) + 1) * np.pi / L
    d = (b[None, :] - theta[:, None] + np.pi) % (2 * np.pi) - np.pi  # signed, in [-pi, pi)
    sgn = np.sign(d[np.arange(len(g)), np.argmin(np.abs(d), axis=1)])
    k0 = slm.level_index(g, L)
    inside = slm.level_index(g * np.exp(1j * sgn * (m - 1e-9)), L)
    across = slm.level_index(g * np.exp(1j * sgn * (m + 1e-9)), L)
    np.testing.assert_array_equal(inside, k0)
    assert np.all(across != k0)
