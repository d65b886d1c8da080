"""Holographic search on tiny grids (oracle; test infrastructure).

Holographic Search Algorithms section: direct search (DS) greedily trials
changes to single SLM pixels and keeps a change only if the error falls.
Here it serves as a brute-force reference for the iterative algorithms:

  * ``exhaustive``: every L^(Ny Nx) pattern (feasible for 4x4 binary) or
    every pattern of a chosen subset of free pixels; returns the global
    minimum of the unscaled replay error sum (|R| - T)^2.
  * ``direct_search``: raster sweeps over all pixels, trying every other
    level, accepting strict decreases, until a sweep changes nothing.  The
    result is a local minimum under every single-pixel change.

The replay change from one pixel change is formed incrementally,
dR = dh * w / sqrt(Nx Ny) with w the centred DFT kernel of that pixel;
tests check it against a full recomputation.
"""
import itertools

import numpy as np

from . import dft as _dft
from . import slm as _slm


def _kernel(ny, nx, y, x):
    """Centred replay of a unit impulse at SLM pixel (y, x)."""
    d = np.zeros((ny, nx), dtype=np.complex128)
    d[y, x] = 1.0
    return _dft.centre(_dft.dft2(d))


def replay_error(levels, T, L):
    R = _dft.centre(_dft.dft2(_slm.level_phasor(levels, L)))
    return float(np.sum((np.abs(R) - T) ** 2))


def exhaustive(T, L, free=None, base_levels=None):
    """Global minimum of the replay error over all patterns of the free pixels."""
    T = np.asarray(T, dtype=np.float64)
    ny, nx = T.shape
    npx = ny * nx
    free = list(range(npx)) if free is None else list(free)
    base = np.zeros(npx, np.int64) if base_levels is None else np.asarray(base_levels, np.int64).ravel().copy()
    # replay = fixed part + sum over free pixels of phasor * kernel
    fixed = base.copy()
    fixed_mask = np.ones(npx, bool)
    fixed_mask[free] = False
    h0 = np.where(fixed_mask, _slm.level_phasor(fixed, L), 0.0)
    R0 = _dft.centre(_dft.dft2(h0.reshape(ny, nx))).ravel()
    K = np.stack([_kernel(ny, nx, p // nx, p % nx).ravel() for p in free], axis=0)  # (F, npx)
    best_e, best = np.inf, None
    combos = np.array(list(itertools.product(range(L), repeat=len(free))), dtype=np.int64)
    for start in range(0, len(combos), 4096):
        c = combos[start:start + 4096]
        R = R0[None, :] + _slm.level_phasor(c, L) @ K
        e = np.sum((np.abs(R) - T.ravel()[None, :]) ** 2, axis=1)
        i = int(np.argmin(e))
        if e[i] < best_e:
            best_e = float(e[i])
            best = base.copy()
            best[free] = c[i]
    return best.reshape(ny, nx), best_e


def direct_search(T, L, init_levels, max_sweeps=1000):
    """Greedy single-pixel search from init_levels; returns (levels, error, sweeps)."""
    T = np.asarray(T, dtype=np.float64)
    ny, nx = T.shape
    lev = np.asarray(init_levels, np.int64).copy()
    R = _dft.centre(_dft.dft2(_slm.level_phasor(lev, L)))
    err = float(np.sum((np.abs(R) - T) ** 2))
    kernels = {}
    for sweep in range(1, max_sweeps + 1):
        changed = False
        for y in range(ny):
            for x in range(nx):
                if (y, x) not in kernels:
                    kernels[(y, x)] = _kernel(ny, nx, y, x)
                kern = kernels[(y, x)]
                cur = _slm.level_phasor(np.array(lev[y, x]), L)
                for k in range(L):
                    if k == lev[y, x]:
                        continue
                    Rn = R + (_slm.level_phasor(np.array(k), L) - cur) * kern
                    en = float(np.sum((np.abs(Rn) - T) ** 2))
                    if en < err - 1e-12:
                        lev[y, x] = k
                        R, err, cur = Rn, en, _slm.level_phasor(np.array(k), L)
                        changed = True
        if not changed:
            return lev, err, sweep
    return lev, err, max_sweeps
