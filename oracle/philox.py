"""Philox4x32-10 and Box-Muller, FP64 oracle side (test infrastructure only).

The Gaussian test matrix Omega of Sec 3 (entries i.i.d. N(0,1)) is drawn from a
counter-based generator so that any element can be recomputed from its index.
Philox4x32-10 is taken from its published definition (J. Salmon, M. Moraes,
R. Dror, D. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11):

* state: four 32-bit counter words c0..c3 and a two-word key k0, k1;
* one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 as 64-bit products,
  new counter = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* ten rounds; between rounds the key advances by the Weyl constants W0, W1.

Element layout used for a rows x cols matrix drawn on stream ``stream`` with a
64-bit ``seed`` (row-major flat index e):
  block = e // 4, word = e % 4,
  counter = (block mod 2^32, block div 2^32, stream, 0), key = (seed lo, seed hi).
Normals: words (0,1) and (2,3) of a block form Box-Muller pairs with
u = (x + 0.5) * 2^-32 in (0, 1); z_even = sqrt(-2 ln u_a) cos(2 pi u_b),
z_odd = sqrt(-2 ln u_a) sin(2 pi u_b), evaluated in FP64.
Uniforms in [0, 1): (x >> 8) * 2^-24.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10: arrays of uint32 counters and keys -> 4 uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint32).copy() for c in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint32).copy()
    k1 = np.asarray(k1, dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def _blocks(count, stream, seed, start=0):
    """Raw Philox words for the ``count`` flat elements from index ``start``
    (a multiple of 4), shape (nblocks, 4)."""
    assert start % 4 == 0
    nblk = (count + 3) // 4
    blk = np.arange(start // 4, start // 4 + nblk, dtype=np.uint64)
    c0 = (blk & MASK32).astype(np.uint32)
    c1 = (blk >> np.uint64(32)).astype(np.uint32)
    c2 = np.full(nblk, stream & 0xFFFFFFFF, dtype=np.uint32)
    c3 = np.zeros(nblk, dtype=np.uint32)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    return np.stack(philox4x32_10(c0, c1, c2, c3, k0, k1), axis=1)


def raw_words(count, stream, seed):
    """uint32 word for each flat element index 0..count-1."""
    return _blocks(count, stream, seed).reshape(-1)[:count]


def normal(rows, cols, stream, seed, row0=0):
    """N(0,1) matrix (rows x cols) in FP64 by Box-Muller on Philox words; with
    row0, rows row0 .. row0 + rows - 1 of a matrix of `cols` columns (flat
    indices from row0 * cols, which must be a multiple of 4)."""
    count = rows * cols
    w = _blocks(count, stream, seed, row0 * cols).astype(np.float64)
    u = (w + 0.5) * 2.0 ** -32
    out = np.empty_like(u)
    for a, b in ((0, 1), (2, 3)):
        rad = np.sqrt(-2.0 * np.log(u[:, a]))
        ang = 2.0 * np.pi * u[:, b]
        out[:, a] = rad * np.cos(ang)
        out[:, b] = rad * np.sin(ang)
    return out.reshape(-1)[:count].reshape(rows, cols)


def uniform(rows, cols, stream, seed):
    """U[0,1) matrix with 24-bit resolution (exact in FP32)."""
    count = rows * cols
    w = raw_words(count, stream, seed)
    return ((w >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).reshape(rows, cols)
