"""Parity of the wide-factor paths (r up to 128, k' up to 256: the largest
workload's shape) against the FP64 oracle on small seeded inputs that span
several tiles with ragged edges (GPU, through the C ABI): the half-step
launches of eq fastHALS_a in all normalisation modes and with the sparsity /
smoothness rule of Sec 4.1, the 2 x 2 block CholeskyQR for 128 < k' <= 256,
column NNLS, the uncompressed FastHALS sweep, the FP8 thin operand of 256
columns, the BF16 range finder on the copy of X^T, and the warm-start network
at 256 -> 512 -> 512 -> 128."""
import numpy as np
import pytest
import torch

import datagen
from oracle import mlp as omlp
from oracle import nmf as onmf
from oracle import quant

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300))


def proj(Q):
    return Q @ Q.T


def parts_case(m, n, r_true, r, kp, seed):
    X = datagen.planted_parts(m, n, r_true, seed)[0]
    OL = datagen.gaussian(n, kp, seed, datagen.S_OMEGA_L)
    OR = datagen.gaussian(m, kp, seed, datagen.S_OMEGA_R)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    return X, OL, OR, W0, H0


# (m, n, r, k'): r = 128 with k' = 256 (the largest workload's widths), r and k'
# between the paths' limits, and P2-like widths (k' <= 128, r > 64); ragged in
# every dimension but n (a multiple of 4, as the library requires)
WIDE = [(2100, 1028, 128, 256, 1), (3001, 776, 100, 140, 1), (1500, 600, 70, 82, 2), (1000, 520, 40, 180, 1)]
# tall enough for the 128-row tiles of the gradient product (N >= 65536)
TALL = (70001, 520, 128, 256, 1)


@pytest.mark.parametrize("m,n,r,kp,q,normalize,up", [w + (nm, 0) for w in WIDE for nm in (1, 0, 2)] +
                         [w + (nm, 1) for w in WIDE for nm in (1, 2)] + [TALL + (1, 0), TALL + (1, 1)])
def test_wide_iterations_match_oracle(lib, m, n, r, kp, q, normalize, up):
    """Iterations 1, 2 and 5 against the oracle's FP64 iterations on its own
    compression, with the update products on FP32 MFMA (up 0) or split-BF16
    MFMA (up 1)."""
    print(f"wide iterations m={m} n={n} r={r} k'={kp} normalize={normalize} update_prec={up}", flush=True)
    seed = 9000 + r + kp
    X, OL, OR, W0, H0 = parts_case(m, n, r, r, kp, seed)
    rQL, rQR, rXh, rXc = onmf.compress(X, OL, OR, q)
    ctx = lib.NMF(m, n, r, kp, q, seed=7, normalize=normalize, update_prec=up)
    Xd = dev(X)
    ctx.compress(Xd, dev(OL), dev(OR))
    assert ctx.sync() == 0
    QL, QR, Xh, Xc = (t.cpu().numpy().astype(np.float64) for t in ctx.state())
    assert np.abs(QL.T @ QL - np.eye(kp)).max() < 5e-6
    assert np.abs(QR.T @ QR - np.eye(kp)).max() < 5e-6
    # same range: the oracle's basis lies in range(Q_L) (O(m k'^2), no m x m projector)
    assert np.abs(QL @ (QL.T @ rQL) - rQL).max() < 1e-4
    W, Ht = W0.astype(np.float64), H0.astype(np.float64)
    ctx.init(dev(W0), dev(H0))
    done = 0
    for iters in (1, 2, 5):
        ctx.step(iters - done)
        for _ in range(iters - done):
            W, Ht = onmf.fasthals_rp_iteration(W, Ht, rXh, rXc, rQL, rQR, normalize)
        done = iters
        Wg, Hg = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
        dw, dh = rel_norm(Wg, W), rel_norm(Hg, Ht)
        print(f"  it={iters} |dW|/|W|={dw:.2e} |dH|/|H|={dh:.2e}", flush=True)
        assert (Wg >= 0).all() and (Hg >= 0).all()
        # the literal rule (normalize = 2) rescales W's columns without moving H,
        # so every later sweep starts away from the fitted scale; there the FP32
        # differences of the first iteration grow fast (measured at r = 128,
        # k' = 256: 6e-5 after one iteration, 2.7e-3 after two)
        # the same for both product precisions (the split gradient carries three
        # BF16 parts, FP32 accuracy): measured at most 7.7e-5 with up = 1
        tol = 1e-4 * iters if (normalize != 2 or iters == 1) else 5e-3 * iters
        assert dw <= tol and dh <= tol, iters
    e, e_ref = ctx.residual(Xd), onmf.rel_error(X, W, Ht)
    assert abs(e - e_ref) <= 1e-5


def test_wide_sparsity_smoothness_rule(lib):
    """The H sweep with alpha, beta (Sec 4.1) on the wide path."""
    print("wide alpha/beta", flush=True)
    m, n, r, kp, q = 2100, 1028, 100, 160, 1
    X, OL, OR, W0, H0 = parts_case(m, n, r, r, kp, 77)
    alpha, beta = 0.3, 2.0
    ctx = lib.NMF(m, n, r, kp, q, seed=7, alpha=alpha, beta=beta)
    ctx.compress(dev(X), dev(OL), dev(OR))
    ctx.init(dev(W0), dev(H0))
    ctx.step(2)
    rQL, rQR, rXh, rXc = onmf.compress(X, OL, OR, q)
    W, Ht = W0.astype(np.float64), H0.astype(np.float64)
    for _ in range(2):
        W, Ht = onmf.fasthals_rp_iteration(W, Ht, rXh, rXc, rQL, rQR, 1, alpha, beta)
    Wg, Hg = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    print(f"  |dW|/|W|={rel_norm(Wg, W):.2e} |dH|/|H|={rel_norm(Hg, Ht):.2e}", flush=True)
    assert rel_norm(Wg, W) <= 2e-4 and rel_norm(Hg, Ht) <= 2e-4


@pytest.mark.parametrize("rows,k,cond", [(5000, 256, 1e4), (3001, 129, 1e3), (4000, 200, 1e5), (256, 256, 10.0)])
def test_orth_wide_cholesky_qr2(lib, rows, k, cond):
    print(f"orth rows={rows} k={k}", flush=True)
    g = np.random.default_rng(rows + k)
    U, _ = np.linalg.qr(g.standard_normal((rows, k)))
    V, _ = np.linalg.qr(g.standard_normal((k, k)))
    Y = (U @ np.diag(np.logspace(0, -np.log10(cond), k)) @ V.T).astype(np.float32)
    ld = (k + 3) // 4 * 4                      # rows of a multiple of 4 floats
    full = np.zeros((rows, ld), dtype=np.float32)
    full[:, :k] = Y
    Yd = dev(full)[:, :k]
    shifted = lib.orth(Yd)
    Q = Yd.cpu().numpy().astype(np.float64)
    assert shifted == 0
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 5e-6
    Qr = onmf.householder_q(Y.astype(np.float64))
    assert np.abs(Q @ Q.T - Qr @ Qr.T).max() < 5e-6


@pytest.mark.parametrize("k", [160, 256])
def test_orth_wide_shifted_fallback(lib, k):
    """A 1e12-conditioned input: the Schur-complement pivots break down, the whole
    factorisation restarts shifted (shifted CholeskyQR3)."""
    print(f"orth shifted k={k}", flush=True)
    g = np.random.default_rng(3)
    rows = 6000
    U, _ = np.linalg.qr(g.standard_normal((rows, k)))
    V, _ = np.linalg.qr(g.standard_normal((k, k)))
    Y = (U @ np.diag(np.logspace(0, -12, k)) @ V.T).astype(np.float32)
    Yd = dev(Y)
    shifted = lib.orth(Yd)
    Q = Yd.cpu().numpy().astype(np.float64)
    assert shifted == 1
    assert np.all(np.isfinite(Q))
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-4
    Y64 = Y.astype(np.float64)
    assert np.linalg.norm(Y64 - Q @ (Q.T @ Y64)) / np.linalg.norm(Y64) < 1e-5


@pytest.mark.parametrize("k,r,rows,sweeps", [(256, 128, 3000, 30), (200, 100, 1001, 50), (90, 70, 500, 20)])
def test_wide_nnls_rows_match_oracle(lib, k, r, rows, sweeps):
    print(f"wide nnls k={k} r={r} rows={rows}", flush=True)
    g = np.random.default_rng(43 + r)
    Wh = g.random((k, r)).astype(np.float32)
    H = np.maximum(g.standard_normal((rows, r)), 0)
    Xr = (H @ Wh.T.astype(np.float64) + 0.05 * g.standard_normal((rows, k))).astype(np.float32)
    out = lib.nnls_rows(dev(Xr), dev(Wh), sweeps).cpu().numpy()
    ref = onmf.column_nnls(Xr.astype(np.float64), Wh.astype(np.float64), sweeps)
    assert np.all(out >= 0)
    d = np.abs(out - ref).max() / (np.abs(ref).max() + 1e-30)
    print(f"  max|d|/max|ref| = {d:.2e}", flush=True)
    assert d <= 1e-4
    H0 = np.maximum(g.standard_normal((rows, r)), 0).astype(np.float32)
    out2 = lib.nnls_rows(dev(Xr), dev(Wh), sweeps, out=dev(H0), warm=True).cpu().numpy()
    ref2 = onmf.column_nnls(Xr.astype(np.float64), Wh.astype(np.float64), sweeps, Ht0=H0)
    assert np.abs(out2 - ref2).max() <= 1e-4 * (np.abs(ref2).max() + 1e-30)


@pytest.mark.parametrize("normalize", [1, 2])
def test_wide_uncompressed_fasthals(lib, normalize):
    print(f"wide uncompressed fasthals normalize={normalize}", flush=True)
    m, n, r, kp = 1500, 600, 90, 102
    X, OL, OR, W0, H0 = parts_case(m, n, 20, r, kp, 31)
    ctx = lib.NMF(m, n, r, kp, 1, seed=7, normalize=normalize)
    Xd = dev(X)
    ctx.init(dev(W0), dev(H0))
    ctx.fasthals_step(Xd, 3)
    W, Ht = onmf.fasthals(X, W0, H0, 3, normalize)
    Wg, Hg = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    print(f"  |dW|/|W|={rel_norm(Wg, W):.2e} |dH|/|H|={rel_norm(Hg, Ht):.2e}", flush=True)
    assert rel_norm(Wg, W) <= 3e-4 and rel_norm(Hg, Ht) <= 3e-4


@pytest.mark.parametrize("rows,k", [(2048, 256), (1000, 200)])
def test_fp8_thin_operand_256_columns(lib, rows, k):
    """The e4m3 copy of a thin operand of up to 256 columns (one launch, the
    exponent of each 128-row block from all columns) against the oracle's
    rounding, through the product it feeds."""
    print(f"fp8 thin K={rows} k={k}", flush=True)
    g = np.random.default_rng(rows + k)
    B = (g.standard_normal((rows, k)) * 10.0 ** g.integers(-3, 3, (rows // 128 + 1, 1)).repeat(128, 0)[:rows])
    B = B.astype(np.float32)
    X = np.abs(g.standard_normal((300, rows))).astype(np.float32)
    Xq, _, E = lib.quantize_x(dev(X), lib.NMF_FP8_E4M3)
    C = lib.gemm_lowp(lib.NMF_FP8_E4M3, Xq, rows, dev(B), E, (E.shape[1], 1)).cpu().numpy().astype(np.float64)
    Xdq = quant.e4m3_block_quantise(X.astype(np.float64))[0]
    ref = Xdq @ onmf.quantize_thin(B, "fp8")
    bound = 2.0 * rows * 2.0 ** -24 * (np.abs(Xdq) @ np.abs(onmf.quantize_thin(B, "fp8"))) + 1e-30
    assert np.all(np.abs(C - ref) <= bound)


def test_bf16_range_finder_on_the_copy_of_x_transposed(lib):
    """BF16 with k' > 128 keeps a BF16 copy of X^T: the whole compression against
    the oracle's low-precision model (projectors) and a few iterations."""
    print("bf16 k'=256 compression", flush=True)
    m, n, r, kp, q = 2100, 1028, 100, 256, 1
    X, OL, OR, W0, H0 = parts_case(m, n, 100, r, kp, 5)
    ctx = lib.NMF(m, n, r, kp, q, seed=7, prec=lib.NMF_BF16)
    ctx.compress(dev(X), dev(OL), dev(OR))
    assert ctx.sync() == 0
    QL, QR, _, _ = (t.cpu().numpy().astype(np.float64) for t in ctx.state())
    mQL, mQR, _, _ = onmf.compress_lowp(X, OL, OR, q, "bf16")
    dl, dr = np.abs(proj(QL) - proj(mQL)).max(), np.abs(proj(QR) - proj(mQR)).max()
    print(f"  projector gaps {dl:.2e} {dr:.2e}", flush=True)
    assert dl < 1e-3 and dr < 1e-3
    ctx.init(dev(W0), dev(H0))
    ctx.step(20)
    e = ctx.residual(dev(X))
    ref = onmf.fasthals_rp(X, OL, OR, q, W0, H0, 20, fmt="bf16")["e"]
    print(f"  e_gpu={e:.6e} R_q={ref:.6e}", flush=True)
    assert abs(e - ref) <= 1e-4


def test_wide_network_gradients_and_inference(lib):
    """The 256 -> 512 -> 512 -> 128 network: loss and gradients against the FP64
    oracle on the same weights and batch, and inference.  A ReLU whose input lies
    within FP32 rounding of zero may switch on one side only (the decision
    belongs to each side's precision), so the batch keeps only the samples whose
    hidden pre-activations are all at least 1e-6 away from zero in the oracle."""
    print("mlp 256-512-512-128", flush=True)
    k, hdim, r, B = 256, 512, 128, 1024
    g = np.random.default_rng(17)
    p0 = datagen.mlp_he_init(k, hdim, r, 3)
    Xb = g.standard_normal((B, k)).astype(np.float32)
    T = np.abs(g.standard_normal((B, r))).astype(np.float32)
    P = omlp.unflatten(p0.astype(np.float64), k, hdim, r)
    _, inv = omlp.scale_rows(Xb.astype(np.float64))
    Xs = Xb.astype(np.float64) * inv[:, None]
    _, (_, z1, _, z2, _, _) = omlp.forward(P, Xs)
    keep = (np.abs(z1).min(axis=1) > 1e-6) & (np.abs(z2).min(axis=1) > 1e-6)
    assert keep.sum() > 0.9 * B
    Xb, T = Xb[keep], T[keep]
    net = lib.Mlp(k, hdim, r, dev(p0), max_batch=B)
    loss, grads = net.loss_grad(dev(Xb), dev(T))
    lref, gref = omlp.loss_grad(P, Xb.astype(np.float64), T.astype(np.float64))
    print(f"  {keep.sum()} samples: loss {loss:.8e} ref {lref:.8e}", flush=True)
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    gg = omlp.unflatten(grads.cpu().numpy(), k, hdim, r)
    for name, a, b in zip(omlp.LAYER_NAMES, gg, gref):
        d = rel_norm(np.asarray(a, dtype=np.float64), b)
        print(f"  {name}: {d:.2e}", flush=True)
        assert d <= 1e-4, name
    out = net.infer(dev(Xb)).cpu().numpy().astype(np.float64)
    ref = omlp.infer(P, Xb.astype(np.float64))
    assert rel_norm(out, ref) <= 1e-5


def test_adaptive_fit_on_a_sampled_residual(lib):
    """nmf_fit's adaptive schedule on a tall problem, where the schedule's residual
    estimates sample every s-th row strip in column parts: the run never stops
    before the exact error reaches eps, stops within a few chunks after it, and
    the reported error is the stopping test's (within its bound of the exact)."""
    m, n, r, kp, q = TALL
    print(f"adaptive fit m={m} n={n} r={r} k'={kp}", flush=True)
    seed = 9000 + r + kp
    X, OL, OR, W0, H0 = parts_case(m, n, r, r, kp, seed)
    Xd = dev(X)
    ref = lib.NMF(m, n, r, kp, q, seed=7)
    ref.compress(Xd, dev(OL), dev(OR))
    ref.init(dev(W0), dev(H0))
    curve = [ref.residual(Xd)]
    for _ in range(60):
        ref.step(1)
        curve.append(ref.residual(Xd))
    eps = 1.0005 * curve[40]
    first = next(i for i, e in enumerate(curve) if e <= eps)
    ctx = lib.NMF(m, n, r, kp, q, seed=7)
    ctx.compress(Xd, dev(OL), dev(OR))
    ctx.init(dev(W0), dev(H0))
    it, e = ctx.fit(Xd, 200, eps, check_every=0)
    e_exact = ctx.residual(Xd)
    _, b, _ = ctx.residual_check(Xd, 10.0)
    print(f"  eps {eps:.6e}: first iteration at eps {first}, fit stopped at {it} with e {e:.6e} "
          f"(exact {e_exact:.6e})", flush=True)
    assert e_exact <= eps and it >= first
    assert it <= first + 25
    assert abs(e - e_exact) <= b
