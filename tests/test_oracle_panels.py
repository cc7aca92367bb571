"""Pins of the pieces the largest workload (262144 x 16384, held in FP32 with
FP64 products over row panels) adds to the oracle and the input generator:
the panel products equal the whole FP64 products, the row-range Philox draws
equal the rows of the whole draw, and the dyadic factors make W0 H0 exact in
FP32 in any summation order (CPU)."""
import numpy as np
import pytest

import datagen
from oracle import nmf, philox


def _proj(Q):
    return Q @ Q.T


def test_row_panel_compression_equals_whole_fp64_compression():
    g = np.random.default_rng(7)
    m, n, r, kp, q = 1000, 300, 6, 12, 2
    X = (g.random((m, r)) @ g.random((r, n)) + 0.01 * g.random((m, n))).astype(np.float32)
    OL = g.standard_normal((n, kp)).astype(np.float32)
    OR = g.standard_normal((m, kp)).astype(np.float32)
    ref = nmf.compress(X, OL, OR, q)
    got = nmf.compress(nmf.RowPanels(X, panel=128), OL, OR, q)
    for a, b in ((ref[0], got[0]), (ref[1], got[1])):
        assert np.abs(_proj(a) - _proj(b)).max() < 1e-12
    # projected data: X^T Q_L and X Q_R depend on the basis only through Q Q^T
    X64 = X.astype(np.float64)
    assert np.abs(got[0] @ got[2].T - _proj(ref[0]) @ X64).max() < 1e-10
    assert np.abs(got[3] @ got[1].T - X64 @ _proj(ref[1])).max() < 1e-10
    # the panel products themselves against the whole products (a plausible
    # slip, a missing panel or a transposed operand, breaks these)
    B_n = g.standard_normal((n, 5))
    B_m = g.standard_normal((m, 5))
    P = nmf.RowPanels(X, panel=96)
    assert np.abs(P.matmul(B_n) - X64 @ B_n).max() < 1e-11
    assert np.abs(P.tmatmul(B_m) - X64.T @ B_m).max() < 1e-10
    W = g.random((m, r))
    Ht = g.random((n, r))
    assert abs(nmf.rel_error(P, W, Ht) - nmf.rel_error(X, W, Ht)) < 1e-14


def test_philox_row_range_equals_rows_of_whole_draw():
    full = philox.normal(40, 12, 2, 99)
    for row0 in (0, 1, 7, 33):
        part = philox.normal(5 if row0 < 35 else 40 - row0, 12, 2, 99, row0=row0)
        assert np.array_equal(part, full[row0:row0 + part.shape[0]])


def test_dyadic_factors_make_the_planted_product_exact_in_fp32():
    m, n, r = 2048, 512, 128
    W0, H0 = datagen.dyadic_parts_factors(m, n, r, 5)
    for A in (W0, H0):
        assert A.dtype == np.float32
        assert np.array_equal(A * 256.0, np.floor(A * 256.0)) and A.min() >= 0 and A.max() < 1
    assert 0.15 < float(np.mean(W0 > 0)) < 0.25
    exact = W0.astype(np.float64) @ H0.astype(np.float64)
    # FP32 sums in three different orders all give the exact product
    assert np.array_equal((W0 @ H0).astype(np.float64), exact)
    rev = np.zeros((m, n), dtype=np.float32)
    for k in reversed(range(r)):
        rev += np.outer(W0[:, k], H0[k])
    assert np.array_equal(rev.astype(np.float64), exact)
    halves = (W0[:, :64] @ H0[:64]) + (W0[:, 64:] @ H0[64:])
    assert np.array_equal(halves.astype(np.float64), exact)


def test_bf16_bit_rounding_equals_the_grid_rounding():
    """The bit-level BF16 rounding used for large panels equals the pinned
    grid rounding on ties, subnormals, both signs and the whole FP32 range."""
    from oracle import quant
    g = np.random.default_rng(3)
    x = (g.standard_normal(200000) * 10.0 ** g.integers(-40, 37, 200000)).astype(np.float32)
    ties = (g.integers(1, 2 ** 16, 5000).astype(np.uint32) << np.uint32(16)) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32), -ties.view(np.float32),
                        np.array([0.0, -0.0, 1e-45, 1e-40, 3.4e38], dtype=np.float32)])
    x = x[np.isfinite(quant.bf16_round(x))]
    assert np.array_equal(quant.bf16_round_bits(x).astype(np.float64), quant.bf16_round(x))


@pytest.mark.parametrize("fmt,refine,lps", [("fp8", 2, 2), ("fp8", 1, 0), ("bf16", 0, 1), ("bf16", 2, 2)])
def test_row_panel_low_precision_model_equals_whole_model(fmt, refine, lps):
    """The low-precision compression model over row panels (quantised copy per
    panel, split products per panel) equals the model on the whole matrix."""
    g = np.random.default_rng(8)
    m, n, r, kp, q = 700, 260, 5, 12, 1
    # full rank (low rank plus noise), so that every basis direction is determined
    X = ((g.random((m, r)) @ g.random((r, n)) + 0.05 * g.random((m, n))) * 10.0 ** g.integers(-2, 2, (m, 1)))
    X = X.astype(np.float32)
    OL = g.standard_normal((n, kp)).astype(np.float32)
    OR = g.standard_normal((m, kp)).astype(np.float32)
    ref = nmf.compress_lowp(X, OL, OR, q, fmt, refine=refine, lowp_sketches=lps)
    got = nmf.compress_lowp(nmf.RowPanels(X, panel=256), OL, OR, q, fmt, refine=refine, lowp_sketches=lps)
    for a, b in zip(ref[:2], got[:2]):
        assert np.abs(_proj(a) - _proj(b)).max() < 1e-10
    scale = np.abs(X).max()
    assert np.abs(got[0] @ got[2].T - ref[0] @ ref[2].T).max() < 1e-9 * scale
    assert np.abs(got[3] @ got[1].T - ref[3] @ ref[1].T).max() < 1e-9 * scale
