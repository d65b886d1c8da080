"""Pins for the oracle's simulated annealing (Holographic Search Algorithms
section): at zero temperature on a binary SLM it is direct search, sweep for
sweep; at infinite temperature it accepts every proposal; and at a fixed
temperature its chain visits the states of a 2 x 2 binary hologram with the
Boltzmann probabilities exp(-E / tau) / Z computed by enumerating all 16
states (the defining property of the Metropolis acceptance rule, which a
wrong sign, a missing factor or a swapped draw would break).
"""
import itertools

import numpy as np

from oracle import dft, hologram, search, slm
import synth


def test_zero_temperature_binary_is_direct_search():
    T = hologram.prepare_target(synth.uniform_target(8, 8, seed=3), 2)
    init = np.random.default_rng(4).integers(0, 2, (8, 8))
    lev_ds, e_ds, sweeps = search.direct_search(T, 2, init)
    lev_sa, errs, _ = search.simulated_annealing(T, 2, init, sweeps + 1, 0.0, 0.9, seed=5)
    assert np.array_equal(lev_sa, lev_ds)
    assert abs(errs[-1] - e_ds) <= 1e-9 * e_ds
    assert np.all(np.diff(errs) <= 1e-12)  # greedy: the error never rises


def test_infinite_temperature_accepts_every_proposal():
    T = hologram.prepare_target(synth.uniform_target(4, 8, seed=6), 2)
    init = np.random.default_rng(7).integers(0, 2, (4, 8))
    lev, _, acc = search.simulated_annealing(T, 2, init, 1, 1e300, 1.0, seed=8)
    assert acc == 32 and np.array_equal(lev, 1 - init)


def test_proposals_are_other_levels_uniformly():
    w0, _ = search.sa_words(11, 1, 64, 64)
    for L in (3, 4, 8):
        for k in range(L):
            props = np.array([search.sa_proposal(k, L, w) for w in w0.ravel()[:3000]])
            assert np.all(props != k) and np.all((props >= 0) & (props < L))
            counts = np.bincount(props, minlength=L)[np.arange(L) != k]
            assert counts.min() > 0.8 * counts.mean()


def test_fixed_temperature_chain_has_the_boltzmann_distribution():
    T = hologram.prepare_target(np.array([[1.0, 0.2], [0.5, 0.9]]), 2)
    states = list(itertools.product((0, 1), repeat=4))
    E = np.array([float(np.sum((np.abs(dft.centre(dft.dft2(slm.level_phasor(np.array(s).reshape(2, 2), 2)))) - T) ** 2))
                  for s in states])
    tau = 0.5 * np.std(E)
    p = np.exp(-(E - E.min()) / tau)
    p /= p.sum()
    n = 6000
    _, _, _, hist = search.simulated_annealing(T, 2, np.zeros((2, 2), np.int64), n, tau, 1.0, seed=13, history=True)
    counts = np.zeros(16)
    for lev in hist:
        counts[int("".join(str(int(b)) for b in lev.ravel()), 2)] += 1
    emp = counts / n
    assert 0.5 * np.abs(emp - p).sum() < 0.04, (emp, p)
