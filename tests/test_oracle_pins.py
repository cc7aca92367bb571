"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(not against the oracle itself).  CPU only."""
import os

import numpy as np
import pytest
import scipy.stats
import torch

from oracle import mlp, nmf, philox, quant

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def proj(Q):
    return Q @ Q.T


# ---------------------------------------------------------------- Philox / Box-Muller

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [np.array([int(x, 16)], dtype=np.uint32) for x in row]
        out = philox.philox4x32_10(v[0], v[1], v[2], v[3], v[4][0], v[5][0])
        assert [int(o[0]) for o in out] == [int(x, 16) for x in row[6:10]]


def test_philox_layout_counter_mapping():
    # element e of stream s uses counter (e//4, 0, s, 0) and word e%4
    w = philox.raw_words(12, stream=7, seed=(5 << 32) | 9)
    for e in range(12):
        out = philox.philox4x32_10(np.array([e // 4], np.uint32), np.array([0], np.uint32),
                                   np.array([7], np.uint32), np.array([0], np.uint32),
                                   np.uint32(9), np.uint32(5))
        assert int(w[e]) == int(out[e % 4][0])


def test_normal_and_uniform_distribution():
    z = philox.normal(400, 250, stream=3, seed=12345).reshape(-1)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1) < 0.01
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # the two members of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 0.01
    u = philox.uniform(300, 300, stream=4, seed=99).reshape(-1)
    assert u.min() >= 0 and u.max() < 1
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    # different streams / seeds give different numbers
    assert not np.allclose(philox.normal(4, 4, 3, 12345), philox.normal(4, 4, 4, 12345))


# ---------------------------------------------------------------- quantisers

def test_bf16_matches_torch_cast():
    g = np.random.default_rng(0)
    x = (g.standard_normal(100000) * 10.0 ** g.integers(-30, 30, 100000)).astype(np.float32)
    x[:7] = [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, 1e-40]  # ties, subnormal
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(quant.bf16_round(x), want)


def test_e4m3_matches_torch_cast():
    g = np.random.default_rng(1)
    y = np.clip(g.standard_normal(100000) * 10.0 ** g.integers(-4, 3, 100000), -448, 448)
    y[:6] = [0.0, 448.0, 2.0 ** -9, 2.0 ** -10, 1.0625, 17.0]
    want = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(quant.e4m3_round(y), want)


def test_block_exponents():
    g = np.random.default_rng(2)
    X = g.random((300, 200)) * 10.0 ** g.integers(-3, 4)
    X[128:256, 128:200] = 0.0
    E = quant.block_exponents(X)
    assert E.shape == (3, 2) and E[1, 1] == 0
    for a in range(3):
        for b in range(2):
            amax = np.abs(X[a * 128:(a + 1) * 128, b * 128:(b + 1) * 128]).max()
            if amax > 0:
                assert 224.0 * 2.0 ** E[a, b] < amax <= 448.0 * 2.0 ** E[a, b]
    deq, _, codes = quant.e4m3_block_quantise(X)
    assert np.abs(codes).max() <= 448
    # relative error of normal-range values is at most half an e4m3 ulp (2^-4)
    big = np.abs(codes) >= 2.0 ** -6
    assert np.max(np.abs(deq - X)[big] / np.abs(X)[big]) <= 2.0 ** -4 * (1 + 1e-12)


# ---------------------------------------------------------------- range finder (Sec 3)

def _lowrank(m, n, rank, seed, noise=0.0):
    g = np.random.default_rng(seed)
    X = g.random((m, rank)) @ g.random((rank, n))
    return X + noise * g.standard_normal((m, n))


def test_range_finder_orthonormal_and_exact_capture():
    X = _lowrank(120, 80, 5, 0)
    Om = np.random.default_rng(1).standard_normal((80, 8))
    Q = nmf.range_finder(X, Om, q=2)
    assert np.abs(Q.T @ Q - np.eye(8)).max() < 1e-14
    assert np.linalg.norm(X - Q @ (Q.T @ X)) / np.linalg.norm(X) < 1e-13


def test_range_finder_span_equals_eq35():
    """Re-orthonormalised subspace iteration spans (X X^T)^w X Omega (eq 3.5)."""
    g = np.random.default_rng(3)
    U, _ = np.linalg.qr(g.standard_normal((60, 60)))
    V, _ = np.linalg.qr(g.standard_normal((40, 40)))
    s = np.linspace(2.0, 1.0, 40)               # mild spectrum: eq 3.5 stays well conditioned
    X = U[:, :40] @ np.diag(s) @ V.T
    Om = g.standard_normal((40, 6))
    for w in (0, 1, 2):
        P = np.linalg.matrix_power(X @ X.T, w) @ X @ Om
        Qe, _ = np.linalg.qr(P)
        Q = nmf.range_finder(X, Om, q=w)
        assert np.abs(proj(Q) - proj(Qe)).max() < 1e-10


def test_power_spectrum_identity():
    """sigma_j((X X^T)^w X) = sigma_j(X)^(2w+1) (Sec 3)."""
    X = np.random.default_rng(4).random((12, 9))
    s = np.linalg.svd(X, compute_uv=False)
    for w in (1, 2):
        sw = np.linalg.svd(np.linalg.matrix_power(X @ X.T, w) @ X, compute_uv=False)
        assert np.allclose(sw, s ** (2 * w + 1), rtol=1e-10)


def test_power_iterations_converge_to_top_singular_subspace():
    g = np.random.default_rng(5)
    U, _ = np.linalg.qr(g.standard_normal((100, 50)))
    V, _ = np.linalg.qr(g.standard_normal((50, 50)))
    s = 2.0 ** -np.arange(50.0)
    X = U @ np.diag(s) @ V.T
    Q = nmf.range_finder(X, g.standard_normal((50, 6)), q=30)   # (1/2)^61 leakage
    ang = scipy.linalg.subspace_angles(Q, U[:, :6])
    assert ang.max() < 1e-8


def test_cholesky_qr2_matches_householder_projector():
    g = np.random.default_rng(6)
    Y = g.standard_normal((500, 20)) @ np.diag(10.0 ** np.linspace(0, 4, 20))
    Q, shifted = nmf.cholesky_qr2(Y)
    assert not shifted
    assert np.abs(Q.T @ Q - np.eye(20)).max() < 1e-13
    assert np.abs(proj(Q) - proj(nmf.householder_q(Y))).max() < 1e-12


def test_shifted_cholesky_qr3_on_breakdown():
    """kappa(Y) = 1e12: plain CholeskyQR2 breaks down or loses orthogonality;
    shifted CholeskyQR3 stays orthonormal and spans range(Y)."""
    g = np.random.default_rng(7)
    U, _ = np.linalg.qr(g.standard_normal((400, 12)))
    V, _ = np.linalg.qr(g.standard_normal((12, 12)))
    Y = U @ np.diag(10.0 ** np.linspace(0, -12, 12)) @ V.T
    try:
        Q1, _ = nmf.cholesky_qr(Y)
        Q2, _ = nmf.cholesky_qr(Q1)
        plain_ok = np.abs(Q2.T @ Q2 - np.eye(12)).max() < 1e-10
    except nmf.CholeskyBreakdown:
        plain_ok = False
    assert not plain_ok
    Q, shifted = nmf.cholesky_qr2(Y, force_shift=True)
    assert shifted
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-12
    assert np.abs(proj(Q) - proj(U)).max() < 1e-3
    Q, shifted = nmf.cholesky_qr2(Y)
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-12


def test_sketch_preserves_distances_in_range():
    """Columns in range(Q_L): ||x_i - x_j|| = ||Q_L^T (x_i - x_j)||; rows of X vs
    rows of X Q_R likewise (Sec 3: distance preservation)."""
    X = _lowrank(50, 30, 4, 8)
    g = np.random.default_rng(9)
    QL, QR, Xh, Xc = nmf.compress(X, g.standard_normal((30, 6)), g.standard_normal((50, 6)), q=1)
    for i, j in [(0, 1), (3, 17), (5, 29)]:
        assert np.isclose(np.linalg.norm(X[:, i] - X[:, j]), np.linalg.norm(Xh[i] - Xh[j]), rtol=1e-12)
    for i, j in [(0, 1), (10, 40)]:
        assert np.isclose(np.linalg.norm(X[i] - X[j]), np.linalg.norm(Xc[i] - Xc[j]), rtol=1e-12)
    # Pythagoras for a generic (noisy) pair
    Xn = X + 0.1 * g.standard_normal(X.shape)
    QL = nmf.range_finder(Xn, g.standard_normal((30, 6)), 1)
    d = Xn[:, 2] - Xn[:, 7]
    assert np.isclose(d @ d, np.sum((QL.T @ d) ** 2) + np.sum((d - QL @ (QL.T @ d)) ** 2), rtol=1e-12)


# ---------------------------------------------------------------- update rules (Sec 4)

def _problem(m=40, n=30, r=3, kp=7, seed=11, noise=0.05, q=1):
    g = np.random.default_rng(seed)
    X = np.abs(g.random((m, r)) @ g.random((r, n)) + noise * g.standard_normal((m, n)))
    QL, QR, Xh, Xc = nmf.compress(X, g.standard_normal((n, kp)), g.standard_normal((m, kp)), q)
    W = g.random((m, r))
    Ht = g.random((n, r))
    return X, QL, QR, Xh, Xc, W, Ht


def test_fast_rule_equals_naive_hals_rp():
    """eq fastHALS_a is algebraically eq hals_update with eq 4_6 substituted."""
    X, QL, QR, Xh, Xc, W, Ht = _problem()
    for normalize in (0, 1, 2):
        Wf, Hf = W, Ht
        Wn, Hn = W, Ht
        for _ in range(5):
            Wf, Hf = nmf.fasthals_rp_iteration(Wf, Hf, Xh, Xc, QL, QR, normalize)
            Wn, Hn = nmf.hals_rp_naive_iteration(Wn, Hn, Xh, Xc, QL, QR, normalize)
        assert np.abs(Wf - Wn).max() < 1e-12 * max(1, np.abs(Wn).max())
        assert np.abs(Hf - Hn).max() < 1e-12 * max(1, np.abs(Hn).max())


def test_square_orthogonal_sketch_reduces_to_fasthals():
    """k' = m = n: the projectors are identities and FastHALS-RP is FastHALS (Sec 2.2)."""
    g = np.random.default_rng(12)
    m = n = 16
    X = g.random((m, 3)) @ g.random((3, n)) + 0.01 * g.random((m, n))
    QL, QR, Xh, Xc = nmf.compress(X, g.standard_normal((n, 16)), g.standard_normal((m, 16)), 1)
    W = g.random((m, 3))
    Ht = g.random((n, 3))
    Wa, Ha = W, Ht
    Wb, Hb = W, Ht
    for _ in range(4):
        Wa, Ha = nmf.fasthals_rp_iteration(Wa, Ha, Xh, Xc, QL, QR)
        Wb, Hb = nmf.fasthals_iteration(X, Wb, Hb)
    assert np.abs(Wa - Wb).max() < 1e-12 and np.abs(Ha - Hb).max() < 1e-11


def test_single_component_is_exact_nnls():
    """r = 1: each update is the closed-form non-negative minimiser."""
    X, QL, QR, Xh, Xc, W, Ht = _problem(r=1)
    W1, H1 = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=0)
    b = QR.T @ Ht[:, 0]
    a = np.maximum(Xc @ b / (b @ b), 0)
    assert np.allclose(W1[:, 0], a, rtol=1e-12, atol=1e-14)
    ah = QL.T @ a
    assert np.allclose(H1[:, 0], np.maximum(Xh @ ah / (ah @ ah), 0), rtol=1e-12, atol=1e-14)


def test_kkt_monotone_and_nonnegative_per_column():
    """Each column update minimises its compressed sub-problem: KKT holds for the
    updated column, J_R (A side) and J_L (B side) never increase, values >= 0."""
    X, QL, QR, Xh, Xc, W, Ht = _problem(r=4, kp=9)
    Hc = QR.T @ Ht
    GH = Hc.T @ Hc
    XcHc = Xc @ Hc
    Wc = W.copy()
    JR = 0.5 * np.sum((Xc - Wc @ Hc.T) ** 2)
    for j in range(4):
        Wc[:, j] = np.maximum(Wc[:, j] + (XcHc[:, j] - Wc @ GH[:, j]) / GH[j, j], 0)
        grad = Wc @ GH[:, j] - XcHc[:, j]          # dJ_R / d a_j (eq hals_a)
        a = Wc[:, j]
        assert np.all(a >= 0)
        assert np.all(np.abs(grad[a > 0]) < 1e-10 * max(1, np.abs(XcHc).max()))
        assert np.all(grad[a == 0] > -1e-10 * max(1, np.abs(XcHc).max()))
        JR_new = 0.5 * np.sum((Xc - Wc @ Hc.T) ** 2)
        assert JR_new <= JR * (1 + 1e-13)
        JR = JR_new
    # the sweep helper agrees with the column-by-column construction above
    assert np.allclose(nmf.w_sweep(W, XcHc, GH), Wc, rtol=1e-12, atol=1e-14)
    Wh = QL.T @ Wc
    GW = Wh.T @ Wh
    P = Xh @ Wh
    Hs = Ht.copy()
    JL = 0.5 * np.sum((Xh.T - Wh @ Hs.T) ** 2)
    for j in range(4):
        Hs[:, j] = np.maximum(Hs[:, j] + (P[:, j] - Hs @ GW[:, j]) / GW[j, j], 0)
        grad = Hs @ GW[:, j] - P[:, j]               # dJ_L / d b_j (eq hals_b)
        b = Hs[:, j]
        assert np.all(np.abs(grad[b > 0]) < 1e-10 * max(1, np.abs(P).max()))
        assert np.all(grad[b == 0] > -1e-10 * max(1, np.abs(P).max()))
        JL_new = 0.5 * np.sum((Xh.T - Wh @ Hs.T) ** 2)
        assert JL_new <= JL * (1 + 1e-13)
        JL = JL_new
    assert np.allclose(nmf.h_sweep(Ht, P, GW), Hs, rtol=1e-12, atol=1e-14)


def test_plain_fasthals_monotone():
    g = np.random.default_rng(13)
    X = g.random((30, 20))
    W = g.random((30, 4))
    Ht = g.random((20, 4))
    J = nmf.objective(X, W, Ht)
    for _ in range(20):
        W, Ht = nmf.fasthals_iteration(X, W, Ht)
        Jn = nmf.objective(X, W, Ht)
        assert Jn <= J * (1 + 1e-13)
        J = Jn


def test_normalisation_modes():
    X, QL, QR, Xh, Xc, W, Ht = _problem()
    W1, H1 = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=1)
    assert np.allclose(np.linalg.norm(W1, axis=0), 1.0)
    W0_, H0_ = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=0)
    # compensated normalisation leaves the product unchanged (exact arithmetic)
    assert np.allclose(W1 @ H1.T, W0_ @ H0_.T, rtol=1e-10)
    W2, _ = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=2)
    assert np.allclose(np.linalg.norm(W2, axis=0), 1.0)


def test_scale_and_permutation_equivariance():
    g = np.random.default_rng(14)
    m, n, r, kp = 36, 28, 3, 7
    X = g.random((m, r)) @ g.random((r, n)) + 0.02 * g.random((m, n))
    OL, OR = g.standard_normal((n, kp)), g.standard_normal((m, kp))
    W, Ht = g.random((m, r)), g.random((n, r))
    a = nmf.fasthals_rp(X, OL, OR, 1, W, Ht, 6)
    b = nmf.fasthals_rp(3.0 * X, OL, OR, 1, W, 3.0 * Ht, 6)
    assert np.allclose(b["W"], a["W"], rtol=1e-9) and np.allclose(b["Ht"], 3.0 * a["Ht"], rtol=1e-9)
    p = g.permutation(m)
    c = nmf.fasthals_rp(X[p], OL, OR[p], 1, W[p], Ht, 6)
    assert np.allclose(c["W"], a["W"][p], rtol=1e-8, atol=1e-12)
    assert np.allclose(c["Ht"], a["Ht"], rtol=1e-8, atol=1e-12)


def test_planted_fixed_point_and_rank_one():
    g = np.random.default_rng(15)
    m, n, r, kp = 50, 40, 4, 8
    W0, H0 = g.random((m, r)), g.random((n, r))
    s = np.linalg.norm(W0, axis=0)
    W0, H0 = W0 / s, H0 * s
    X = W0 @ H0.T
    QL, QR, Xh, Xc = nmf.compress(X, g.standard_normal((n, kp)), g.standard_normal((m, kp)), 1)
    W, Ht = W0, H0
    for _ in range(10):
        W, Ht = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR)
    assert nmf.rel_error(X, W, Ht) < 1e-14
    assert nmf.rel_error(X, W0, H0) == 0.0
    # rank one: one iteration recovers the factors up to scale
    a, b = g.random(m), g.random(n)
    X1 = np.outer(a, b)
    QL, QR, Xh, Xc = nmf.compress(X1, g.standard_normal((n, 3)), g.standard_normal((m, 3)), 1)
    W1, H1 = nmf.fasthals_rp_iteration(g.random((m, 1)), g.random((n, 1)), Xh, Xc, QL, QR)
    assert nmf.rel_error(X1, W1, H1) < 1e-14


def test_planted_separable_converges_to_1e10():
    g = np.random.default_rng(5)
    m, n, r, kp = 60, 40, 3, 6
    W0 = g.random((m, r)); W0[:r] = np.eye(r)
    H0 = g.random((n, r)); H0[:r] = np.eye(r)
    X = W0 @ H0.T
    out = nmf.fasthals_rp(X, g.standard_normal((n, kp)), g.standard_normal((m, kp)), 2,
                          g.random((m, r)), g.random((n, r)), 1500)
    assert out["e"] < 1e-10


def test_residual_direct_vs_expansion_and_proxy():
    g = np.random.default_rng(16)
    X = g.random((70, 50))
    W, Ht = g.random((70, 4)), g.random((50, 4))
    res, nx = nmf.frob_sq_diff(X, W, Ht, block=16)
    exp = np.sum(X * X) - 2 * np.sum((W.T @ X) * Ht.T) + np.sum((W.T @ W) * (Ht.T @ Ht))
    assert np.isclose(res, exp, rtol=1e-10) and np.isclose(nx, np.sum(X * X))
    # proxy is exact when Q_L = I
    QL = np.eye(70)
    assert np.isclose(nmf.proxy_rel_error(nx, X.T @ QL, QL.T @ W, Ht), nmf.rel_error(X, W, Ht), rtol=1e-10)
    # ... and when the columns of W lie in range(Q_L)
    QL = nmf.householder_q(g.standard_normal((70, 9)))
    Wp = QL @ (QL.T @ W)
    assert np.isclose(nmf.proxy_rel_error(nx, X.T @ QL, QL.T @ Wp, Ht), nmf.rel_error(X, Wp, Ht), rtol=1e-10)


def test_gini_closed_forms_and_pairwise_definition():
    assert abs(nmf.gini(np.ones((5, 4)))) < 1e-15
    v = np.zeros(20); v[3] = 2.5
    assert np.isclose(nmf.gini(v), 19 / 20)
    x = np.random.default_rng(17).random(37)
    pair = np.sum(np.abs(x[:, None] - x[None, :])) / (2 * x.size * x.sum())
    assert np.isclose(nmf.gini(x), pair, rtol=1e-12)


def test_constrained_rule_reduces_and_sparsifies():
    X, QL, QR, Xh, Xc, W, Ht = _problem()
    a = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=0)
    b = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=0, alpha=0.0, beta=0.0)
    Wh = QL.T @ a[0]
    Hz = nmf.h_sweep_constrained(Ht, Xh @ Wh, Wh.T @ Wh, 0.0, 0.0)
    assert np.allclose(Hz, a[1]) and np.allclose(b[1], a[1])
    # the HALS-RP form of the sparse rule (eq hals_constr) for one component
    Wh1 = Wh[:, :1]
    P = Xh @ Wh1
    h = nmf.h_sweep_constrained(Ht[:, :1], P, Wh1.T @ Wh1, 0.3, 0.7)
    want = np.maximum(P[:, 0] - 0.3, 0) / (Wh1[:, 0] @ Wh1[:, 0] + 0.7)
    assert np.allclose(h[:, 0], want, rtol=1e-12)
    # larger alpha gives a sparser B (Gini grows)
    out = [nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, alpha=al)[1] for al in (0.0, 1.0)]
    assert nmf.gini(out[1]) >= nmf.gini(out[0])


def test_table_memory_formulas():
    """Table 4.1's memory formulas reproduce the printed memory columns (the
    tables print two significant digits, truncated)."""
    def two_digits(v):
        p = 10.0 ** (np.floor(np.log10(v)) - 1)
        return np.floor(v / p) * p

    rows = [l.split() for l in open(os.path.join(GOLDEN, "table_memory.txt"))
            if l.strip() and not l.startswith("#")]
    for d, n, k, kp, nonrp, rp, unit in rows:
        a, b = nmf.complexity_memory(int(d), int(n), int(k), int(kp))
        assert round(two_digits(a) / float(unit)) == int(nonrp)
        assert round(two_digits(b) / float(unit)) == int(rp)


# ---------------------------------------------------------------- MLP (extension)

def _small_net(seed=0, k=8, hdim=16, r=4):
    g = np.random.default_rng(seed)
    return [g.standard_normal(s) * 0.5 for s in mlp.shapes(k, hdim, r)]


def test_mlp_gradients_vs_finite_differences():
    g = np.random.default_rng(1)
    P = _small_net()
    X = g.random((5, 8)) + 0.1
    T = g.random((5, 4))
    _, grads = mlp.loss_grad(P, X, T)
    flat = mlp.flatten(P)
    gflat = mlp.flatten(grads)
    h = 1e-6
    idx = g.choice(flat.size, 60, replace=False)
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        Lp, _ = mlp.loss_grad(mlp.unflatten(fp, 8, 16, 4), X, T)
        Lm, _ = mlp.loss_grad(mlp.unflatten(fm, 8, 16, 4), X, T)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_mlp_closed_forms():
    z = np.array([-30.0, -1.0, 0.0, 2.0, 40.0])
    assert np.allclose(mlp.softplus(z), np.log1p(np.exp(z)))
    assert np.allclose(mlp.sigmoid(z), 1 / (1 + np.exp(-z)))
    # positive homogeneity of the scaled net
    P = _small_net(2)
    x = np.random.default_rng(3).random((3, 8))
    assert np.allclose(mlp.infer(P, 5.0 * x), 5.0 * mlp.infer(P, x))
    assert np.all(mlp.infer(P, np.zeros((2, 8))) == 0)
    # first Adam step from zero moments moves every parameter by lr * g/(|g|+eps)
    gr = [np.full(p.shape, 0.3) for p in P]
    z0 = [np.zeros_like(p) for p in P]
    P1, _, _ = mlp.adam_step(P, gr, z0, z0, 1, lr=1e-2)
    for p, p1 in zip(P, P1):
        assert np.allclose(p - p1, 1e-2 * 0.3 / (0.3 + 1e-8))


def test_warm_selection_never_worse_than_cold():
    g = np.random.default_rng(4)
    Xh = g.random((50, 6))
    Wh = g.random((6, 3))
    Hn, Hc = g.random((50, 3)), g.random((50, 3))
    Hsel, rej = mlp.select_warm(Xh, Wh, Hn, Hc)
    rs = np.sum((Xh - Hsel @ Wh.T) ** 2, 1)
    assert np.all(rs <= np.sum((Xh - Hc @ Wh.T) ** 2, 1))
    assert np.all(rs <= np.sum((Xh - Hn @ Wh.T) ** 2, 1) + 0 * rej)
    assert 0 < rej.sum() < 50


def test_column_nnls_matches_active_set_nnls():
    """The training targets (column NNLS by repeated H sweeps) converge to the
    unique non-negative least-squares solution (Lawson-Hanson active set)."""
    from scipy.optimize import nnls
    g = np.random.default_rng(9)
    Wh = g.random((12, 5))
    H_true = np.maximum(g.standard_normal((40, 5)), 0)
    Xr = H_true @ Wh.T + 0.05 * g.standard_normal((40, 12))
    Ht = nmf.column_nnls(Xr, Wh, sweeps=3000)
    for j in range(40):
        ref, _ = nnls(Wh, Xr[j])
        assert np.allclose(Ht[j], ref, atol=1e-9)
    assert np.all(Ht >= 0)


def test_split_bf16_representation():
    """Two-term BF16 split: hi and lo agree with torch's round-to-nearest-even
    BF16 cast, |a - hi - lo| <= 2^-16 |a|, and values with at most 16
    significant bits are represented exactly."""
    g = np.random.default_rng(17)
    a = (g.standard_normal(20000) * 10.0 ** g.integers(-20, 20, 20000)).astype(np.float32)
    hi, lo = nmf.split_bf16(a)
    t_hi = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(hi, t_hi)
    r32 = (a.astype(np.float64) - hi).astype(np.float32)
    assert np.array_equal(r32.astype(np.float64), a.astype(np.float64) - hi)      # a - hi is exact in FP32
    assert np.array_equal(lo, torch.from_numpy(r32).to(torch.bfloat16).to(torch.float64).numpy())
    assert np.all(np.abs(a.astype(np.float64) - hi - lo) <= 2.0 ** -16 * np.abs(a.astype(np.float64)))
    # 16 significant bits: integers below 2^16, scaled by powers of two
    b = (g.integers(1, 2 ** 16, 5000) * 2.0 ** g.integers(-30, 30, 5000)).astype(np.float32)
    bh, bl = nmf.split_bf16(b)
    assert np.array_equal(bh + bl, b.astype(np.float64))


def test_split_product_bound_and_exact_case():
    """Split-BF16 product (lo*lo dropped) within 3.1 * 2^-16 (|A| |B|) of the
    exact product, and exact when both operands are BF16 values."""
    g = np.random.default_rng(23)
    A = g.random((300, 500)).astype(np.float32)
    B = g.standard_normal((500, 40)).astype(np.float32)
    P = nmf.split_product(A, B)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    bound = 3.1 * 2.0 ** -16 * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)))
    assert np.all(np.abs(P - exact) <= bound)
    # a dropped cross term would be visible: the bound is far below |Ah Bl|
    Ah, Al = nmf.split_bf16(A)
    Bh, Bl = nmf.split_bf16(B)
    assert np.max(np.abs(Ah @ Bl) - bound) > 0
    Ab = torch.from_numpy(A).to(torch.bfloat16).to(torch.float32).numpy()
    Bb = torch.from_numpy(B).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(nmf.split_product(Ab, Bb), Ab.astype(np.float64) @ Bb.astype(np.float64))
