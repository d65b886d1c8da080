"""Pins for the oracle's Philox4x64-10 (published generator, Salmon et al. SC'11)."""
import numpy as np
import pytest

from oracle import philox
from conftest import golden

M64 = (1 << 64) - 1


def _np_words(counter, key, n=4):
    # numpy's Philox increments its 256-bit counter before each block
    c = (sum(int(w) << (64 * i) for i, w in enumerate(counter)) - 1) % (1 << 256)
    g = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                         counter=np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64))
    return [int(v) for v in g.random_raw(n)]


def test_known_answer_vectors():
    rows = [l.split() for l in open(golden("philox_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 2
    for r in rows:
        v = [int(h, 16) for h in r]
        ctr, key, out = v[0:4], v[4:6], v[6:10]
        got = philox.philox4x64_10([np.array([c], np.uint64) for c in ctr], key)
        assert [int(g[0]) for g in got] == out


def test_matches_numpy_philox_random_blocks():
    rng = np.random.default_rng(7)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        got = philox.philox4x64_10([np.array([c], np.uint64) for c in ctr], key)
        assert [int(g[0]) for g in got] == _np_words(ctr, key)


@pytest.mark.parametrize("axis", [0, 1])
def test_line_word_mapping_against_numpy(axis):
    seed, tag, b, ny, nx = 0x1234ABCD5678, 0x105, 3, 8, 16
    words = philox.line_words(seed, tag, ny, nx, axis, batch_item=b)
    key = [seed, (b << 32) | tag]
    n = nx if axis == 1 else ny
    for y in range(ny):
        for x in range(nx):
            i, l = (x, y) if axis == 1 else (y, x)
            blk = _np_words([i % (n // 4), l, 0, 0], key)
            assert int(words[y, x]) == blk[i // (n // 4)]


def test_u24_exact_and_in_range():
    w = np.array([0, 1 << 40, M64, 0xFFFFFF0000000000], dtype=np.uint64)
    u = philox.u24(w)
    assert u[0] == 0.0 and u[1] == 2.0 ** -24
    assert u[2] == 1.0 - 2.0 ** -24 and u[3] == u[2]
    ph = philox.phase_field(5, philox.TAG_INIT, 16, 16)
    assert ph.min() >= 0 and ph.max() < 2 * np.pi
    # uniformity sanity on a larger draw
    big = philox.u24(philox.line_words(9, 1, 256, 256, 1))
    assert abs(big.mean() - 0.5) < 0.01 and abs(big.var() - 1 / 12) < 0.005
