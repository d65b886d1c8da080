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
  * ``simulated_annealing``: the same trial, one proposed level per pixel
    per sweep, accepted when the error falls or, with probability
    exp(-dE / tau), when it rises (the temperature-based acceptance of the
    Holographic Search Algorithms section; Metropolis rule), with a
    geometric temperature schedule tau_s = t0 alpha^(s - 1).  Proposals and
    acceptance draws come from Philox4x64-10 (see sa_words).

The replay change from one pixel change is formed incrementally,
dR = dh * w / sqrt(Nx Ny) with w the centred DFT kernel of that pixel;
tests check it against a full recomputation.
"""
import itertools

import numpy as np

from . import dft as _dft
from . import philox as _ph
from . import slm as _slm

TAG_SA = 0x5A  # Philox tag of the simulated-annealing draws


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


def sa_words(seed, sweep, ny, nx, batch_item=0):
    """The two random words of every simulated-annealing trial of a sweep:
    trial (sweep s, pixel p = y nx + x) takes words 0 and 1 of the
    Philox4x64-10 block at counter (p, s, 0, 0) under key
    (seed, (item << 32) | TAG_SA).  Returns two (ny, nx) uint64 arrays."""
    p = np.arange(ny * nx, dtype=np.uint64)
    s = np.full_like(p, np.uint64(sweep))
    z = np.zeros_like(p)
    key = (np.uint64(seed), np.uint64(((batch_item & 0xFFFFFFFF) << 32) | TAG_SA))
    w = _ph.philox4x64_10((p, s, z, z), key)
    return w[0].reshape(ny, nx), w[1].reshape(ny, nx)


def sa_proposal(k, L, word):
    """Proposed level of a trial: another level than k, uniformly
    (k + 1 + floor(u (L - 1))) mod L with u = u24(word); binary: the flip."""
    return int((k + 1 + int(np.floor(float(_ph.u24(word)) * (L - 1)))) % L)


def simulated_annealing(T, L, init_levels, sweeps, t0, alpha, seed=0, batch_item=0, history=False):
    """Simulated annealing from init_levels over `sweeps` raster sweeps.

    Trial at pixel (y, x): propose sa_proposal(k, L, word 0); dE = change of
    the replay error sum (|R| - T)^2; accept when dE < 0, or when tau > 0
    and u24(word 1) < exp(-dE / tau), tau = t0 alpha^(s - 1) in the units of
    the error.  Returns (levels, errors: the error before sweep 1 and after
    each sweep, accepted trial count[, the levels after each sweep when
    history]).  Parity unpinned as a quality
    statement (the schedule is a reading); the acceptance rule is pinned by
    its stationary distribution.
    """
    T = np.asarray(T, dtype=np.float64)
    ny, nx = T.shape
    lev = np.asarray(init_levels, np.int64).copy()
    R = _dft.centre(_dft.dft2(_slm.level_phasor(lev, L)))
    err = float(np.sum((np.abs(R) - T) ** 2))
    errors, accepted, hist = [err], 0, []
    kernels = {}
    for sweep in range(1, sweeps + 1):
        tau = t0 * alpha ** (sweep - 1)
        w0, w1 = sa_words(seed, sweep, ny, nx, batch_item)
        for y in range(ny):
            for x in range(nx):
                if (y, x) not in kernels:
                    kernels[(y, x)] = _kernel(ny, nx, y, x)
                k = int(lev[y, x])
                kn = sa_proposal(k, L, w0[y, x])
                Rn = R + (_slm.level_phasor(np.array(kn), L) - _slm.level_phasor(np.array(k), L)) * kernels[(y, x)]
                en = float(np.sum((np.abs(Rn) - T) ** 2))
                de = en - err
                ok = de < 0.0 or (tau > 0.0 and float(_ph.u24(w1[y, x])) < np.exp(-de / tau))
                if ok:
                    lev[y, x], R, err = kn, Rn, en
                    accepted += 1
        errors.append(err)
        if history:
            hist.append(lev.copy())
    if history:
        return lev, np.array(errors), accepted, hist
    return lev, np.array(errors), accepted
