"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds input generators only: no step of the hologram method
(no transform, projection, constraint or metric).  It draws with numpy's
Philox bit generator; none of these draws is one of the method's own random
phases (those are computed by each side from the counter-based definition).

Workloads (seeded stand-ins for the paper's test images, which are not
available; the paper uses no public dataset):

  uniform_target   sqrt of a uniform[0, 1) intensity (64x64 GS case)
  gaussian_target  sqrt of a sum of 32 isotropic Gaussians (sigma 5-60 px,
                   peak amplitudes uniform in [0.2, 1]) whose centres lie in
                   the central N/2 x N/2 window, clipped to that window and
                   zero outside; lengths scale by N/1024 for other grids
  fresnel_z        per-problem propagation distance, uniform in [0.1, 0.5] m
  batch_mix        the uneven 256-problem Fresnel batch (64x256^2,
                   96x512^2, 64x1024^2, 32x2048^2)
  roi_mask         a region-of-interest mask: the union of a few discs and
                   rectangles placed off centre (kind "shapes"), or
                   independent pixels with probability 1/2 (kind "pixels")
"""
import numpy as np

TAG_TARGET = 2
TAG_GAUSS = 3
TAG_ZDRAW = 4
TAG_ROI = 5

WAVELENGTH_M = 532e-9
PITCH_M = 8e-6


def _rng(seed, tag, batch_item=0):
    return np.random.Generator(np.random.Philox(key=[seed & (2**64 - 1), (batch_item << 32) | tag]))


def uniform_target(ny, nx, seed):
    """Amplitude sqrt(U[0, 1)) per pixel, float32 [ny][nx]."""
    rng = _rng(seed, TAG_TARGET)
    return np.sqrt(rng.random((ny, nx))).astype(np.float32)


def gaussian_target(n, seed, batch_item=0, count=32, ny=None):
    """Gaussian-sum intensity target on an n x n grid (or ny x n), amplitude float32."""
    ny = n if ny is None else ny
    nx = n
    rng = _rng(seed, TAG_GAUSS, batch_item)
    scale = nx / 1024.0
    wy, wx = ny // 2, nx // 2
    y0, x0 = ny // 4, nx // 4
    cy = y0 + wy * rng.random(count)
    cx = x0 + wx * rng.random(count)
    sig = (5.0 + 55.0 * rng.random(count)) * scale
    amp = 0.2 + 0.8 * rng.random(count)
    # each isotropic Gaussian is the outer product of two 1-D profiles, so the
    # sum over Gaussians is one (ny x count) (count x nx) product
    yy = np.arange(ny, dtype=np.float64)[:, None]
    xx = np.arange(nx, dtype=np.float64)[:, None]
    gy = np.exp(-((yy - cy[None, :]) ** 2) / (2.0 * sig[None, :] ** 2))
    gx = np.exp(-((xx - cx[None, :]) ** 2) / (2.0 * sig[None, :] ** 2))
    inten = (gy * amp[None, :]) @ gx.T
    win = np.zeros((ny, nx), bool)
    win[y0:y0 + wy, x0:x0 + wx] = True
    inten = np.where(win, inten, 0.0)
    return np.sqrt(inten).astype(np.float32)


def fresnel_z(seed, batch_item):
    """Propagation distance uniform in [0.1, 0.5] m for one batch item."""
    return 0.1 + 0.4 * float(_rng(seed, TAG_ZDRAW, batch_item).random())


def batch_mix(scale=1):
    """Sizes of the uneven Fresnel batch; scale divides every count (>= 1 each)."""
    mix = [(256, 64), (512, 96), (1024, 64), (2048, 32)]
    out = []
    for n, c in mix:
        out += [n] * max(1, c // scale)
    return out


def roi_mask(ny, nx, seed, kind="shapes"):
    """Region-of-interest mask, uint8 [ny][nx] (1 = controlled replay pixel).

    shapes: 2 discs (radius ny/16 - ny/6) and 2 rectangles (sides nx/8 -
    nx/3), centres uniform over the plane, so the mask is neither centred
    nor centro-symmetric; pixels: each pixel in with probability 1/2."""
    rng = _rng(seed, TAG_ROI)
    if kind == "pixels":
        return (rng.random((ny, nx)) < 0.5).astype(np.uint8)
    yy = np.arange(ny)[:, None]
    xx = np.arange(nx)[None, :]
    m = np.zeros((ny, nx), bool)
    for _ in range(2):
        cy, cx = rng.random() * ny, rng.random() * nx
        r = (1.0 / 16 + (1.0 / 6 - 1.0 / 16) * rng.random()) * ny
        m |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    for _ in range(2):
        h = int((1.0 / 8 + (1.0 / 3 - 1.0 / 8) * rng.random()) * ny)
        w = int((1.0 / 8 + (1.0 / 3 - 1.0 / 8) * rng.random()) * nx)
        y0, x0 = int(rng.random() * (ny - h)), int(rng.random() * (nx - w))
        m[y0:y0 + h, x0:x0 + w] = True
    return m.astype(np.uint8)
