"""Pins of the oracle's low-precision compression model and of its Adam
recursion beyond the first step (CPU only).

The model of the low-precision range finder (`nmf.compress_lowp`) is pinned by
facts that do not restate its code:
  * on inputs whose values the formats represent exactly, the model without
    power iterations is the exact compression (Sec 3.1, eq 3.5 with w = 0);
  * the chain of products of eq 3.5 (subspace iteration) built here from
    torch's BF16 / float8_e4m3fn casts and LAPACK's QR gives the same bases;
  * one power iteration on the exact X after the low-precision chain captures
    range(X) exactly when rank(X) <= k' (the refinement extension), while the
    chain alone does not;
  * the FP8 thin-operand rounding equals the 128 x 128 tile model of the data
    when the operand is at most 128 columns wide, and torch's e4m3 cast with
    power-of-two block scales otherwise, including an amax of exactly 448 2^e.
"""
import numpy as np
import torch

from oracle import mlp, nmf, quant


def proj(Q):
    return Q @ Q.T


def pow2_block_exp(amax):
    """Smallest integer e with amax <= 448 2^e, from frexp (0 for amax == 0)."""
    if amax == 0:
        return 0
    mant, ex = np.frexp(amax / 448.0)        # amax / 448 = mant 2^ex, mant in [0.5, 1)
    return int(ex) - (1 if mant == 0.5 else 0)


def torch_bf16(a):
    """FP64 -> FP32 -> BF16 (nearest even at both steps) with torch's casts."""
    t = torch.from_numpy(np.asarray(a, dtype=np.float64).astype(np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def torch_e4m3_rowblocks(B):
    """FP32 values of B rounded to e4m3 with one power-of-two scale per block of
    128 rows (all columns), by torch's float8_e4m3fn cast."""
    B = np.asarray(B, dtype=np.float64).astype(np.float32).astype(np.float64)
    out = np.empty_like(B)
    for k0 in range(0, B.shape[0], 128):
        blk = B[k0:k0 + 128]
        e = pow2_block_exp(float(np.max(np.abs(blk))) if blk.size else 0.0)
        codes = torch.from_numpy(blk * 2.0 ** -e).to(torch.float8_e4m3fn).to(torch.float64).numpy()
        out[k0:k0 + 128] = codes * 2.0 ** e
    return out


def torch_e4m3_tiles(X, tile=128):
    """X rounded to e4m3 with one power-of-two scale per tile x tile block."""
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    out = np.empty_like(X)
    for a in range(0, X.shape[0], tile):
        for b in range(0, X.shape[1], tile):
            blk = X[a:a + tile, b:b + tile]
            e = pow2_block_exp(float(np.max(np.abs(blk))))
            codes = torch.from_numpy(blk * 2.0 ** -e).to(torch.float8_e4m3fn).to(torch.float64).numpy()
            out[a:a + tile, b:b + tile] = codes * 2.0 ** e
    return out


def small_int_problem(m, n, kp, seed):
    g = np.random.default_rng(seed)
    X = g.integers(0, 16, (m, n)).astype(np.float32)        # <= 4 significant bits: BF16 and e4m3 exact
    OL = g.integers(-3, 4, (n, kp)).astype(np.float32)
    OR = g.integers(-3, 4, (m, kp)).astype(np.float32)
    return X, OL, OR


def test_lowp_model_without_power_iterations_is_exact_on_representable_inputs():
    """With w = 0 the range finder is one product and one QR (eq 3.5).  When the
    formats represent X and Omega exactly, the low-precision model must give the
    exact compression: same projectors and the same basis-free products."""
    X, OL, OR = small_int_problem(300, 260, 12, 5)
    QL, QR, Xh, Xc = nmf.compress(X, OL, OR, 0)
    for fmt in ("bf16", "fp8"):
        assert np.array_equal(nmf.quantize_data(X, fmt), X.astype(np.float64))
        qL, qR, xh, xc = nmf.compress_lowp(X, OL, OR, 0, fmt)
        assert np.max(np.abs(proj(qL) - proj(QL))) < 1e-12
        assert np.max(np.abs(proj(qR) - proj(QR))) < 1e-12
        assert np.max(np.abs(xh @ qL.T - Xh @ QL.T)) < 1e-9 * np.abs(X).max()
        assert np.max(np.abs(xc @ qR.T - Xc @ QR.T)) < 1e-9 * np.abs(X).max()


def _chain(Xq, Omega, q, rnd):
    """eq 3.5 as subspace iteration with every product on the rounded data and
    a rounded thin operand; QR by LAPACK."""
    Q = np.linalg.qr(Xq @ rnd(Omega))[0]
    for _ in range(q):
        Z = np.linalg.qr(Xq.T @ rnd(Q))[0]
        Q = np.linalg.qr(Xq @ rnd(Z))[0]
    return Q


def test_lowp_chain_matches_products_built_from_torch_casts():
    g = np.random.default_rng(7)
    m, n, kp = 384, 300, 10
    W0 = g.random((m, 6))
    X = (W0 @ g.random((6, n)) + 0.05 * g.random((m, n))).astype(np.float32)
    OL = g.standard_normal((n, kp)).astype(np.float32)
    OR = g.standard_normal((m, kp)).astype(np.float32)
    for fmt, data, thin in (("bf16", torch_bf16(X), torch_bf16), ("fp8", torch_e4m3_tiles(X), torch_e4m3_rowblocks)):
        for q in (1, 2):
            QL, QR, Xh, Xc = nmf.compress_lowp(X, OL, OR, q, fmt)
            assert np.max(np.abs(proj(QL) - proj(_chain(data, OL, q, thin)))) < 1e-10, (fmt, q)
            assert np.max(np.abs(proj(QR) - proj(_chain(data.T, OR, q, thin)))) < 1e-10, (fmt, q)
            # projected data on the exact X (lowp_sketches 0)
            assert np.allclose(Xh, X.astype(np.float64).T @ QL, rtol=0, atol=1e-12 * np.abs(X).max() * m)
            assert np.allclose(Xc, X.astype(np.float64) @ QR, rtol=0, atol=1e-12 * np.abs(X).max() * n)
            # lowp_sketches 1: the projected data are products on the rounded copies too
            _, _, xh1, xc1 = nmf.compress_lowp(X, OL, OR, q, fmt, lowp_sketches=1)
            assert np.max(np.abs(xh1 - data.T @ thin(QL))) < 1e-10 * np.abs(X).max()
            assert np.max(np.abs(xc1 - data @ thin(QR))) < 1e-10 * np.abs(X).max()
            # and they are not the exact products: the rounding shows
            assert np.max(np.abs(xh1 - Xh)) > 1e-4 * np.abs(Xh).max()


def test_refinement_pass_captures_exact_range():
    """rank(X) = k': after the low-precision chain, one power iteration on the
    exact X (refinement) spans range(X) to rounding; the chain alone leaves a
    residual of the order of the format's precision."""
    g = np.random.default_rng(11)
    m, n, kp = 400, 260, 8
    # 9-bit factors: every entry of X is exact in FP32, so rank(X) = k' exactly
    A = g.integers(1, 512, (m, kp)) / 512.0
    B = g.integers(1, 512, (kp, n)) / 512.0
    X = (A @ B).astype(np.float32)
    Xd = X.astype(np.float64)
    assert np.array_equal(Xd, A @ B)
    OL = g.standard_normal((n, kp)).astype(np.float32)
    OR = g.standard_normal((m, kp)).astype(np.float32)
    nx = np.linalg.norm(Xd)
    for fmt in ("bf16", "fp8"):
        QL, QR, _, _ = nmf.compress_lowp(X, OL, OR, 1, fmt)
        assert np.linalg.norm(Xd - QL @ (QL.T @ Xd)) / nx > 1e-6
        assert np.linalg.norm(Xd - (Xd @ QR) @ QR.T) / nx > 1e-6
        QL, QR, _, _ = nmf.compress_lowp(X, OL, OR, 1, fmt, refine=True)
        assert np.linalg.norm(Xd - QL @ (QL.T @ Xd)) / nx < 1e-12
        assert np.linalg.norm(Xd - (Xd @ QR) @ QR.T) / nx < 1e-12
        # the refinement on split-BF16 products: the products carry about 16
        # significant bits, so the captured range is good to about 2^-16 relative
        # (a pass on the rounded copy of X would stay at the chain's level above)
        QL, QR, _, _ = nmf.compress_lowp(X, OL, OR, 1, fmt, refine=2)
        for res in (np.linalg.norm(Xd - QL @ (QL.T @ Xd)) / nx, np.linalg.norm(Xd - (Xd @ QR) @ QR.T) / nx):
            assert 1e-12 < res < 2.0 ** -16


def test_split_sketches_within_bound_of_exact_products():
    """lowp_sketches 2: X-hat^T = X^T Q_L and X-check = X Q_R as split-BF16
    products, within 3.1 2^-16 (|X| |Q|) of the exact products and not equal to them."""
    g = np.random.default_rng(13)
    m, n, kp = 300, 200, 9
    X = (g.random((m, 5)) @ g.random((5, n)) + 0.01 * g.random((m, n))).astype(np.float32)
    Xd = X.astype(np.float64)
    OL = g.standard_normal((n, kp)).astype(np.float32)
    OR = g.standard_normal((m, kp)).astype(np.float32)
    QL, QR, Xh, Xc = nmf.compress_lowp(X, OL, OR, 1, "bf16", refine=True, lowp_sketches=2)
    QL32, QR32 = QL.astype(np.float32).astype(np.float64), QR.astype(np.float32).astype(np.float64)
    bh = 3.1 * 2.0 ** -16 * (np.abs(Xd).T @ np.abs(QL32))
    bc = 3.1 * 2.0 ** -16 * (np.abs(Xd) @ np.abs(QR32))
    assert np.all(np.abs(Xh - Xd.T @ QL32) <= bh)
    assert np.all(np.abs(Xc - Xd @ QR32) <= bc)
    assert np.max(np.abs(Xh - Xd.T @ QL32)) > 0


def test_fp8_thin_operand_rounding():
    g = np.random.default_rng(17)
    # <= 128 columns: one block per 128 rows, the same as the 128 x 128 tiles of the data model
    B = g.standard_normal((300, 100)) * 10.0 ** g.integers(-3, 3)
    B[5, 7] = 448.0 * 2.0 ** -3 * 1.5      # block 0: amax 84
    B[130:256] = np.clip(B[130:256], -55.0, 55.0)
    B[140, 3] = 56.0                        # block 1: amax exactly 448 2^-3
    B[256:] = 0.0                           # block 2: all zero
    Bq = nmf.quantize_thin(B, "fp8")
    want, E, _ = quant.e4m3_block_quantise(B.astype(np.float32).astype(np.float64))
    assert np.array_equal(Bq, want)
    assert E[1, 0] == -3 and E[2, 0] == 0 and E[0, 0] == -2
    assert np.array_equal(Bq, torch_e4m3_rowblocks(B))
    assert np.all(Bq[256:] == 0)
    # 256 columns: still one scale per 128 rows over all columns
    C = g.standard_normal((260, 256))
    C[:128, 200] = 300.0
    Cq = nmf.quantize_thin(C, "fp8")
    assert np.array_equal(Cq, torch_e4m3_rowblocks(C))
    # the large entry in columns 128..255 sets the scale of columns 0..127 too
    assert not np.array_equal(Cq[:128, :128], quant.e4m3_block_quantise(C[:128, :128].astype(np.float32)
                                                                       .astype(np.float64))[0])


def test_adam_second_and_third_steps_closed_form():
    """Adam (Kingma & Ba) on a scalar with gradients 1, -2, 1/2, lr 0.01:
    t = 1: m = 0.1, v = 0.001, bias corrections 0.1 and 0.001;
    t = 2: m = -0.11, v = 0.004999, corrections 0.19 and 0.001999;
    t = 3: m = -0.049, v = 0.005244001, corrections 0.271 and 0.002997001."""
    lr, eps = 0.01, 1e-8
    p = [np.array([0.5])]
    mm = [np.zeros(1)]
    vv = [np.zeros(1)]
    want = 0.5
    steps = [(1.0, 0.1, 0.001, 0.1, 0.001), (-2.0, -0.11, 0.004999, 0.19, 0.001999),
             (0.5, -0.049, 0.005244001, 0.271, 0.002997001)]
    for t, (gr, m_t, v_t, c1, c2) in enumerate(steps, start=1):
        p, mm, vv = mlp.adam_step(p, [np.array([gr])], mm, vv, t, lr)
        want = want - lr * (m_t / c1) / (np.sqrt(v_t / c2) + eps)
        assert abs(mm[0][0] - m_t) < 1e-15 and abs(vv[0][0] - v_t) < 1e-15
        assert abs(p[0][0] - want) < 1e-13, (t, p[0][0], want)
