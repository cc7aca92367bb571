"""Kernel-level parity of the HIP path against the FP64 oracle (GPU)."""
import numpy as np
import pytest
import torch

import datagen
from oracle import nmf as onmf
from oracle import philox as ophilox

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


def f32_ulp(x):
    return np.spacing(np.abs(x).astype(np.float32)).astype(np.float64)


@pytest.mark.parametrize("rows,cols,sid,seed", [(1000, 37, 3, 12345), (7, 5, 4, (0xDEADBEEF << 32) | 77),
                                                (4096, 64, 0xFFFFFFF0, 2 ** 64 - 1)])
def test_philox_normal_and_uniform(lib, rows, cols, sid, seed):
    print(f"philox rows={rows} cols={cols} sid={sid} seed={seed}", flush=True)
    z = lib.gaussian(rows, cols, sid, seed).cpu().numpy().astype(np.float64)
    want = ophilox.normal(rows, cols, sid, seed).astype(np.float32).astype(np.float64)
    diff = np.abs(z - want)
    assert np.all(diff <= f32_ulp(want) * 1.0001 + 1e-37)
    assert np.mean(diff == 0) > 0.999
    u = lib.uniform(rows, cols, sid, seed, scale=1.0).cpu().numpy().astype(np.float64)
    assert np.array_equal(u, ophilox.uniform(rows, cols, sid, seed))
    u3 = lib.uniform(rows, cols, sid, seed, scale=3.0).cpu().numpy().astype(np.float64)
    assert np.array_equal(u3, (ophilox.uniform(rows, cols, sid, seed) * 3.0).astype(np.float32))


GEMM_CASES = [
    (1000, 20, 1004, False), (1000, 20, 1004, True), (4096, 64, 4096, False), (4096, 64, 8192, True),
    (300, 128, 512, False), (512, 256, 1000, True), (130, 100, 36, False), (64, 32, 65536, True),
    (257, 256, 260, False), (4, 4, 4, True), (0, 8, 16, False),
    # N <= 32 on 256-row tiles: several tiles with a ragged tail, split-K
    (1300, 32, 5000, False), (780, 20, 70000, True), (4100, 28, 4096, True),
    # 33 <= N <= 64: ragged tails and split-K on 128-row tiles (too few workgroups
    # for 256-row ones) and on 256-row tiles (the last two)
    (3000, 64, 2000, False), (1000, 60, 4100, True), (300, 36, 70000, True),
    (4200, 48, 16384, False), (2100, 64, 20000, True),
]


@pytest.mark.parametrize("M,N,K,at", GEMM_CASES)
def test_gemm_f32(lib, M, N, K, at):
    print(f"gemm M={M} N={N} K={K} at={at}", flush=True)
    g = np.random.default_rng(M * 7 + N + K)
    A = (g.random((K, M)) if at else g.random((M, K))).astype(np.float32) - 0.3
    B = g.standard_normal((K, N)).astype(np.float32)
    C = lib.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), a_trans=at).cpu().numpy()
    A64 = A.astype(np.float64).T if at else A.astype(np.float64)
    ref = A64 @ B.astype(np.float64)
    bound = 2.0 * max(K, 1) * 2.0 ** -24 * (np.abs(A64) @ np.abs(B.astype(np.float64))) + 1e-30
    assert C.shape == (M, N)
    assert np.all(np.abs(C - ref) <= bound)


# k = 1, 16, 17, 48, 63, 64: the 16-column panels of the blocked factorisation
# (one panel, a full panel plus one column, ragged last panels)
@pytest.mark.parametrize("rows,k,cond", [(5000, 64, 1e3), (3001, 20, 1e2), (20000, 128, 1e4), (64, 64, 10.0),
                                         (2000, 1, 1.0), (2000, 16, 1e3), (2000, 17, 1e3), (4000, 48, 1e4),
                                         (4000, 63, 1e4)])
def test_orth_cholesky_qr2(lib, rows, k, cond):
    print(f"orth rows={rows} k={k}", flush=True)
    g = np.random.default_rng(rows + k)
    U, _ = np.linalg.qr(g.standard_normal((rows, k)))
    V, _ = np.linalg.qr(g.standard_normal((k, k)))
    Y = (U @ np.diag(np.logspace(0, -np.log10(cond), k)) @ V.T).astype(np.float32)
    ld = (k + 3) // 4 * 4                      # rows of a multiple of 4 floats
    full = np.zeros((rows, ld), dtype=np.float32)
    full[:, :k] = Y
    Yd = torch.from_numpy(full).cuda()[:, :k]
    shifted = lib.orth(Yd)
    Q = Yd.cpu().numpy().astype(np.float64)
    assert shifted == 0
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 2e-6
    Qr = onmf.householder_q(Y.astype(np.float64))
    assert np.abs(Q @ Q.T - Qr @ Qr.T).max() < 2e-6


@pytest.mark.parametrize("k", [32, 64])
def test_orth_shifted_fallback(lib, k):
    print(f"orth shifted k={k}", flush=True)
    g = np.random.default_rng(3)
    rows = 4000
    U, _ = np.linalg.qr(g.standard_normal((rows, k)))
    V, _ = np.linalg.qr(g.standard_normal((k, k)))
    Y = (U @ np.diag(np.logspace(0, -12, k)) @ V.T).astype(np.float32)
    Yd = torch.from_numpy(Y.copy()).cuda()
    shifted = lib.orth(Yd)
    Q = Yd.cpu().numpy().astype(np.float64)
    assert shifted == 1
    assert np.all(np.isfinite(Q))
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-4
    Y64 = Y.astype(np.float64)
    assert np.linalg.norm(Y64 - Q @ (Q.T @ Y64)) / np.linalg.norm(Y64) < 1e-5


def test_orth_partial_column_group_ignores_padding(lib):
    """k = 37 inside rows of 40 floats: the padding columns hold NaN and must be
    neither read into the result nor written."""
    print("orth k=37 ld=40", flush=True)
    rows, k, ld = 3000, 37, 40
    g = np.random.default_rng(5)
    Y = g.standard_normal((rows, k)) @ np.diag(np.logspace(0, 2, k))
    full = np.full((rows, ld), np.nan, dtype=np.float32)
    full[:, :k] = Y
    Fd = torch.from_numpy(full).cuda()
    Yd = Fd[:, :k]
    assert lib.orth(Yd) == 0
    F = Fd.cpu().numpy()
    assert np.isnan(F[:, k:]).all()
    Q = F[:, :k].astype(np.float64)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 2e-6
    Qr = onmf.householder_q(Y)
    assert np.abs(Q @ Q.T - Qr @ Qr.T).max() < 1e-4
