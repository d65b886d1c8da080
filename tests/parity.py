"""Shared parity checks of the GPU tests (helpers, no tests here).

Tolerances (the parity protocol): complex fields and NMSE within 1e-4
relative (L2 for fields).  Quantised levels must match the FP64 oracle
exactly, except at pixels whose oracle phase lies within 1e-5 rad of a
decision boundary, or whose field lies closer to a decision boundary than
FP32 transform precision resolves: a Euclidean distance |g| sin(margin)
below 1e-6 of the rms of g (about 16 FP32 ulps, the absolute error of a
1024-point transform; the field being zero is the special case |g| below
that).  The FP32 error of g is absolute, about the same at every pixel, so
a small |g| turns it into a large angle: a pixel at |g| = 1e-3 rms and
7e-5 rad from the boundary is 7e-8 rms away from it and its level is not
decided by FP32 arithmetic.  Those exempt mismatches are counted
separately, printed, and bounded per comparison (exempt_bounds).
"""
import numpy as np

from oracle import slm

FIELD_TOL = 1e-4
NMSE_TOL = 1e-4
BAND = 1e-5
ZERO = 1e-6


def say(*a):
    print("[gpu]", *a, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def rel_max(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def exempt_bounds(npx):
    """Most exempt level mismatches one comparison of npx pixels may have:
    (in the angular band or within FP32 distance of a boundary, within FP32
    distance alone).

    A fraction L 2e-5 / (2 pi) of uniformly spread phases lies in the band
    (2.5e-5 at L = 8), and only the part of it where the FP32 angle error
    (about 1e-6 rad at |g| = rms) exceeds the margin can flip, about a tenth
    of it; a real-valued g (binary phase, symmetrised target) lies within
    1e-6 of its rms of the boundary on about 8e-7 of the pixels, and flips
    only well inside that.  The bounds leave a few-fold headroom over those
    rates, plus a count of 2 for small planes."""
    return 2 + int(np.ceil(1e-5 * npx)), 2 + int(np.ceil(2e-6 * npx))


def level_check(gpu_lev, ref_lev, g_ref, L, where=""):
    """(non-exempt mismatches, exempt mismatches) of GPU levels against the
    oracle's; prints each non-exempt mismatch and asserts the exempt counts
    are within exempt_bounds."""
    mism = np.asarray(gpu_lev, np.int64) != np.asarray(ref_lev, np.int64)
    margin = slm.boundary_margin(g_ref, L)
    rms = np.sqrt(np.mean(np.abs(g_ref) ** 2))
    # Euclidean distance to the nearest boundary ray (margin <= pi/L <= pi/2)
    zero = mism & (np.abs(g_ref) * np.sin(margin) < ZERO * rms)
    band = mism & (margin < BAND) & ~zero
    bad = mism & ~(band | zero)
    if bad.any():
        for y, x in list(zip(*np.nonzero(bad)))[:20]:
            a = abs(g_ref[y, x])
            say(f"  mismatch at ({y},{x}): margin {margin[y, x]:.3e} rad, |g|/rms {a / rms:.3e}, "
                f"distance/rms {a * np.sin(margin[y, x]) / rms:.3e}")
    nb, nz = int(band.sum()), int(zero.sum())
    if nb or nz:
        say(f"  {where} exempt level mismatches: {nb} in the angular band, {nz} within FP32 distance")
    max_all, max_zero = exempt_bounds(mism.size)
    assert nb + nz <= max_all, f"{where}: {nb + nz} exempt mismatches exceed the bound {max_all}"
    assert nz <= max_zero, f"{where}: {nz} FP32-distance mismatches exceed the bound {max_zero}"
    return int(bad.sum()), nb + nz
