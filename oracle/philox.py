"""Philox4x64-10 counter-based generator (oracle; test infrastructure).

Written from the published definition (J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11): a 4-word, 64-bit-lane Philox network of 10 rounds.  Each round
multiplies counter words 0 and 2 by the constants M0 and M1 (full 128-bit
products), and permutes/mixes:

    out0 = hi(M1 * c2) ^ c1 ^ k0      out1 = lo(M1 * c2)
    out2 = hi(M0 * c0) ^ c3 ^ k1      out3 = lo(M0 * c0)

and the key is bumped by the Weyl constants between rounds.

How the hologram method draws its random numbers (a reading; the paper
does not specify a generator).  A plane is split into lines of length n
(rows, n = Nx, for the SLM-plane initial phase; columns, n = Ny, for the
replay-plane OSPR phases); element i of line l uses

    key     = (seed, (b << 32) | tag)     b = batch item (0 unbatched)
    counter = (i mod n/4, l, 0, 0)        one block serves i, i + n/4, i + n/2, i + 3n/4
    word    = i div (n/4)                 output word 0..3 of the block
    u24     = (word >> 40) * 2^-24        exact in float32 and float64
    phase   = 2 pi u24

Tags: INIT = 1 (initial SLM phase, row lines), OSPR subframe n uses
0x100 + n (replay phase, column lines).
Vectorised with numpy uint64 arithmetic; 64x64->128 products are formed
from 32-bit halves.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
MASK32 = np.uint64(0xFFFFFFFF)

TAG_INIT = 1
TAG_OSPR = 0x100


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays a * b -> (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    s32 = np.uint64(32)
    a_lo, a_hi = a & MASK32, a >> s32
    b_lo, b_hi = b & MASK32, b >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    # middle column with carries (each term < 2^32, sum < 2^34)
    mid = (ll >> s32) + (lh & MASK32) + (hl & MASK32)
    lo = (ll & MASK32) | ((mid & MASK32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.  ctr: 4 uint64 arrays; key: 2 uint64 values."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64).copy() for c in ctr)
    k0 = np.uint64(key[0])
    k1 = np.uint64(key[1])
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = np.uint64((int(k0) + int(W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def line_words(seed, tag, ny, nx, axis, batch_item=0):
    """One 64-bit word per element of an ny x nx plane, mapping above.

    axis = 1: lines are rows (i = x, l = y); axis = 0: lines are columns
    (i = y, l = x).  Returns an (ny, nx) uint64 array.
    """
    n, nl = (nx, ny) if axis == 1 else (ny, nx)
    q = n // 4
    i = np.arange(q, dtype=np.uint64)
    l = np.arange(nl, dtype=np.uint64)
    ctr0 = np.repeat(i[None, :], nl, axis=0).ravel()
    ctr1 = np.repeat(l[:, None], q, axis=1).ravel()
    z = np.zeros_like(ctr0)
    key = (np.uint64(seed), np.uint64(((batch_item & 0xFFFFFFFF) << 32) | (tag & 0xFFFFFFFF)))
    blocks = np.stack(philox4x64_10((ctr0, ctr1, z, z), key), axis=0).reshape(4, nl, q)
    lines = np.concatenate([blocks[w] for w in range(4)], axis=1)  # (nl, n): word w covers i in [w q, (w+1) q)
    return lines if axis == 1 else lines.T.copy()


def u24(words):
    """Top 24 bits of each word as a float in [0, 1) (exact)."""
    return (np.asarray(words, dtype=np.uint64) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24


def phase_field(seed, tag, ny, nx, batch_item=0):
    """Uniform random phases 2 pi u24 on an Ny x Nx grid (float64).

    The initial SLM phase (tag INIT) uses row lines, OSPR phases column lines.
    """
    axis = 1 if tag == TAG_INIT else 0
    return 2.0 * np.pi * u24(line_words(seed, tag, ny, nx, axis, batch_item))
