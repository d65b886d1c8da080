"""Pins for the oracle's region-of-interest GS (Background section: an
application may care about part of the replay field only, and the error
metric may count that part alone; Algorithms section: amplitude freedom
where the replay is not controlled).

Each check is fixed by something other than the oracle's own formula:
  * a region covering the plane is plain GS;
  * a centred square region on a target that is zero outside it is
    Liu-Taghizadeh at a fixed radius (same constraint, same prepared target),
    whose own pins are in test_oracle_gs;
  * the region NMSE is the scale-optimal error over the region, found here by
    a numerical minimisation over the scale;
  * for binary phase a mask and its mirror image control the same pixels
    (the replay is centro-symmetric), so on a symmetric target they give the
    same run -- which fails if the region is not symmetrised;
  * continuous-phase GS with free pixels is still an alternating projection,
    so the unscaled error over the region never increases.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import hologram
import synth


def _nonincreasing(e, rel=1e-10):
    e = np.asarray(e)
    return np.all(e[1:] <= e[:-1] * (1 + rel) + 1e-12)


@pytest.mark.parametrize("L", [0, 2, 8])
def test_roi_covering_the_plane_is_gs(L):
    T = synth.gaussian_target(32, seed=4)
    a = hologram.gs(T, 4, L, seed=3)
    b = hologram.gs(T, 4, L, seed=3, roi=np.ones((32, 32), np.uint8))
    if L >= 2:
        np.testing.assert_array_equal(a["levels"], b["levels"])
    np.testing.assert_allclose(a["nmse"], b["nmse"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("L,r", [(8, 9), (0, 6), (2, 10)])
def test_centred_square_roi_is_fixed_radius_lt(L, r):
    """The constraint inside the square and the free amplitude outside are
    LT's at radius r (dr = 0); the prepared target is the same because the
    target is zero outside the square.  Only the NMSE differs: the region run
    counts the square alone."""
    n = 32
    T = synth.gaussian_target(n, seed=7).astype(np.float64)
    sq = hologram.lt_window(n, n, r)
    T = np.where(sq, T, 0.0)
    if L == 2:  # a centro-symmetric target, so symmetrisation keeps it inside the square
        T = np.sqrt(0.5 * (T * T + hologram.mirror(T) ** 2))
        assert np.all(T[~sq] == 0)
    a = hologram.gs(T, 5, L, seed=2, lt=(r, 0))
    b = hologram.gs(T, 5, L, seed=2, roi=sq.astype(np.uint8))
    if L >= 2:
        np.testing.assert_array_equal(a["levels"], b["levels"])
    np.testing.assert_allclose(b["field"], a["field"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(b["replay"], a["replay"], rtol=0, atol=1e-12)
    assert np.all(b["nmse"] != a["nmse"])


def test_region_nmse_is_the_scale_optimal_error_over_the_region():
    ny, nx = 32, 64
    T = synth.gaussian_target(nx, seed=3, ny=ny)
    M = synth.roi_mask(ny, nx, seed=5)
    out = hologram.gs(T, 3, 4, seed=1, roi=M)
    region = M != 0
    Tp = out["target"][region]
    A = np.abs(out["replay"])[region]

    def err(s):
        return np.sum((s * A - Tp) ** 2) / np.sum(Tp ** 2)

    best = minimize_scalar(err, bounds=(0.0, 10.0), method="bounded", options={"xatol": 1e-12})
    assert abs(best.fun - out["nmse"][-1]) < 1e-9
    # the target outside the region was dropped before the energy scaling
    assert np.all(out["target"][~region] == 0)
    assert abs(np.sum(out["target"] ** 2) - ny * nx) < 1e-8 * ny * nx


def test_binary_region_is_symmetrised():
    n = 32
    T = synth.gaussian_target(n, seed=8).astype(np.float64)
    T = np.sqrt(0.5 * (T * T + hologram.mirror(T) ** 2))  # symmetric, so masking commutes with the mirror
    M = synth.roi_mask(n, n, seed=2)
    assert np.any(M != hologram.mirror(M))
    a = hologram.gs(T, 4, 2, seed=6, roi=M)
    b = hologram.gs(T, 4, 2, seed=6, roi=hologram.mirror(M))
    np.testing.assert_array_equal(a["levels"], b["levels"])
    np.testing.assert_allclose(a["nmse"], b["nmse"], rtol=0, atol=1e-13)
    assert np.array_equal(a["region"], (M != 0) | (hologram.mirror(M) != 0))
    # phase levels other than two take the mask as given
    c = hologram.gs(T, 2, 8, seed=6, roi=M)
    assert np.array_equal(c["region"], M != 0)


@pytest.mark.parametrize("kind", ["shapes", "pixels"])
def test_region_error_never_increases(kind):
    ny, nx = 32, 32
    T = synth.uniform_target(ny, nx, seed=3)
    M = synth.roi_mask(ny, nx, seed=4, kind=kind)
    out = hologram.gs(T, 25, 0, seed=1, roi=M)
    assert _nonincreasing(out["fienup"]), out["fienup"]
    assert out["fienup"][-1] < out["fienup"][0]


def test_roi_rejects_weighted_and_lt():
    T = synth.uniform_target(16, 16, seed=1)
    M = np.ones((16, 16), np.uint8)
    with pytest.raises(ValueError):
        hologram.gs(T, 1, 2, roi=M, weighted=True)
    with pytest.raises(ValueError):
        hologram.gs(T, 1, 2, roi=M, lt=(4, 0))
