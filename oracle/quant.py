"""Low-precision number formats used by the compression extension (test
infrastructure only).  Values are returned as FP64 arrays holding exactly the
representable numbers, so every oracle product on them is exact before
accumulation.

BF16: 1 sign, 8 exponent, 7 fraction bits (FP32's exponent range); conversion
from FP32 rounds to nearest, ties to even.

FP8 e4m3 (OCP 8-bit floating point specification, E4M3 "FN" variant): 1 sign,
4 exponent bits with bias 7, 3 fraction bits, subnormals, largest finite 448, no
infinities.  Conversion rounds to nearest even and saturates to +-448.

Block scaling: every 128 x 128 tile of X gets a power-of-two scale 2^e with e the
smallest integer such that amax(tile) <= 448 * 2^e (e = 0 for an all-zero tile),
and stores code = e4m3(x * 2^-e).  Power-of-two scales make x * 2^-e exact, so
the only rounding is the e4m3 conversion itself.
"""
import numpy as np


def _round_to_grid(x, mant_bits, emin, maxval=None, inf_at=None):
    """Round FP64 values to a binary format with `mant_bits` fraction bits and
    minimum normal exponent `emin` (so subnormal spacing 2^(emin - mant_bits)),
    ties to even (np.rint).  Saturates to +-maxval when given; magnitudes that
    round to `inf_at` or beyond become inf."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # guard against log2 rounding at exact powers of two
    e = np.where(2.0 ** e > ax, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= ax, e + 1, e)
    e = np.maximum(e, emin)
    spacing = 2.0 ** (e - mant_bits)
    q = np.rint(ax / spacing) * spacing
    if maxval is not None:
        q = np.minimum(q, maxval)
    if inf_at is not None:
        q = np.where(q >= inf_at, np.inf, q)
    out[nz] = np.sign(x[nz]) * q
    return out


def bf16_round(x32):
    """FP32 -> BF16 round-to-nearest-even, returned as FP64 values."""
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    return _round_to_grid(x, 7, -126, inf_at=2.0 ** 128)


def bf16_round_bits(x32):
    """The same rounding as bf16_round on the FP32 bit patterns (finite values):
    add 0x7FFF plus the lowest kept bit, clear the low 16 bits.  For large arrays."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32)


def e4m3_round(x):
    """Real -> e4m3 (FN) round-to-nearest-even with saturation to +-448."""
    return _round_to_grid(x, 3, -6, maxval=448.0)


def block_exponents(X, tile=128):
    """Power-of-two exponent e per tile x tile block: smallest e with
    amax <= 448 * 2^e (0 for an all-zero block).  Shape (ceil(m/tile), ceil(n/tile))."""
    X = np.asarray(X, dtype=np.float64)
    m, n = X.shape
    bm, bn = -(-m // tile), -(-n // tile)
    E = np.zeros((bm, bn), dtype=np.int64)
    for a in range(bm):
        for b in range(bn):
            amax = float(np.max(np.abs(X[a * tile:(a + 1) * tile, b * tile:(b + 1) * tile])))
            if amax > 0:
                e = int(np.ceil(np.log2(amax / 448.0)))
                while amax > 448.0 * 2.0 ** e:
                    e += 1
                while amax <= 448.0 * 2.0 ** (e - 1):
                    e -= 1
                E[a, b] = e
    return E


def e4m3_block_quantise(X, tile=128):
    """Returns (dequantised FP64 values, exponents, codes as FP64 values)."""
    X = np.asarray(X, dtype=np.float64)
    E = block_exponents(X, tile)
    scale = np.repeat(np.repeat(2.0 ** E, tile, axis=0), tile, axis=1)[:X.shape[0], :X.shape[1]]
    codes = e4m3_round(X / scale)
    return codes * scale, E, codes
