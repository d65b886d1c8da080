"""Shared parity checks of the GPU tests (helpers, no tests here).

Tolerances (the parity protocol): complex fields and NMSE within 1e-4
relative (L2 for fields).  Quantised levels must match the FP64 oracle
exactly, except at pixels within 1e-5 rad of a decision boundary.  The
angle is taken two ways, and either exempts: at the pixel's own magnitude
(its angular margin) and at the field's rms magnitude (a Euclidean distance
|g| sin(margin) below 1e-5 of the rms of g).  The second matters because
the FP32 error of g is absolute, about the same at every pixel (7e-7 of the
rms, measured at 1024^2), so a small |g| turns it into a large angle: a
pixel at |g| = 1e-3 rms and 7e-5 rad from the boundary is 7e-8 rms away from
it and its level is not decided by FP32 arithmetic; a zero field is the
extreme case.  Those exempt mismatches are counted separately, printed, and
bounded per comparison (exempt_bounds).
"""
import numpy as np

from oracle import slm

FIELD_TOL = 1e-4
NMSE_TOL = 1e-4
BAND = 1e-5
DIST = 1e-5
# 16-bit field storage: both sides round the stored field to binary16 at the
# same points, so they differ only where an FP32 and an FP64 value straddle a
# binary16 rounding boundary: one binary16 step (2^-11 relative) on a small
# fraction of the stored elements.  That leaves R within about 1e-5 relative
# L2, but the replay constraint divides by |R| (and weighted GS multiplies by
# the weights), so g differs by up to about 1.3e-4 (measured on the GPU and
# reproduced on the CPU by perturbing the oracle's values by FP32-sized
# errors before each store).  Fields are therefore held to one binary16 step,
# 2^-11 relative L2, and the distance band and its bound widen 50-fold
# (5e-4 rms: about four times the per-pixel error of g).
FIELD16_TOL = 2.0 ** -11
FIELD16_BAND = 50.0


def say(*a):
    print("[gpu]", *a, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rel_max(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def exempt_bounds(npx, L, scale=1.0):
    """Most exempt level mismatches one comparison of npx pixels at L levels
    may have: (in either band, in the distance band alone).

    A pixel flips when the FP32 error of g across the nearest boundary
    exceeds its distance to it.  A circular Gaussian g has a density of
    about 0.56 L / rms per unit distance from its L boundary rays (a real g,
    binary phase: 0.8 / rms), and the error across a boundary is about 5e-7
    rms, so about 2.3e-7 L flips per pixel are expected (0.5 per million
    pixels at L = 2, 2 at L = 8, 60 at L = 256).  The angular band adds
    pixels of small |g| that the distance band mostly holds already.  The
    bounds leave a four-fold headroom, plus a count of 2 for small planes."""
    dist = 2 + int(np.ceil(scale * 1e-6 * max(L, 2) * npx))
    return dist + int(np.ceil(1e-5 * npx)), dist


def level_check(gpu_lev, ref_lev, g_ref, L, where="", amplitude=False, band_scale=1.0):
    """(non-exempt mismatches, exempt mismatches) of GPU levels against the
    oracle's; prints each non-exempt mismatch and asserts the exempt counts
    are within exempt_bounds.  amplitude: levels of an amplitude SLM, whose
    decision boundaries are values of Re g (only the distance band applies).
    band_scale widens the distance band and its bound together (16-bit field
    storage: 10, see FIELD16_BAND)."""
    mism = np.asarray(gpu_lev, np.int64) != np.asarray(ref_lev, np.int64)
    rms = np.sqrt(np.mean(np.abs(g_ref) ** 2))
    if amplitude:
        margin = slm.amplitude_margin(g_ref, L)  # a distance in field units
        zero = mism & (margin < band_scale * DIST * rms)
        band = np.zeros_like(mism)
    else:
        margin = slm.boundary_margin(g_ref, L)
        # Euclidean distance to the nearest boundary ray (margin <= pi/L <= pi/2)
        zero = mism & (np.abs(g_ref) * np.sin(margin) < band_scale * DIST * rms)
        band = mism & (margin < BAND) & ~zero
    bad = mism & ~(band | zero)
    if bad.any():
        for y, x in list(zip(*np.nonzero(bad)))[:20]:
            a = abs(g_ref[y, x])
            say(f"  mismatch at ({y},{x}): margin {margin[y, x]:.3e} rad, |g|/rms {a / rms:.3e}, "
                f"distance/rms {a * np.sin(margin[y, x]) / rms:.3e}")
    nb, nz = int(band.sum()), int(zero.sum())
    if nb or nz:
        say(f"  {where} exempt level mismatches: {nb} in the angular band, {nz} in the distance band")
    max_all, max_zero = exempt_bounds(mism.size, L, band_scale)
    assert nb + nz <= max_all, f"{where}: {nb + nz} exempt mismatches exceed the bound {max_all}"
    assert nz <= max_zero, f"{where}: {nz} distance-band mismatches exceed the bound {max_zero}"
    return int(bad.sum()), nb + nz
