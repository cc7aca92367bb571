"""Parity of the HIP spectrum path (symmetric Jacobi eigenvalues, singular values
of the compressed data) and of the parameter-study runs against the FP64 oracle
(GPU, through the C ABI)."""
import numpy as np
import pytest
import torch

import datagen
from oracle import nmf as onmf
from oracle import spectrum as ospec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


def sym_case(k, seed, kind):
    g = np.random.default_rng(seed)
    if kind == "gauss":
        B = g.standard_normal((k, k))
        return B + B.T
    if kind == "repeated":   # eigenvalues 3 (half) and -1 (half) in a random basis
        Q = np.linalg.qr(g.standard_normal((k, k)))[0]
        lam = np.where(np.arange(k) < k // 2, 3.0, -1.0)
        return Q @ np.diag(lam) @ Q.T
    if kind == "graded":     # a Gram with singular values over 8 decades
        Y = g.standard_normal((3 * k, k)) @ np.diag(np.logspace(0, -4, k))
        return Y.T @ Y
    raise ValueError(kind)


@pytest.mark.parametrize("k,kind", [(1, "gauss"), (2, "gauss"), (3, "gauss"), (17, "gauss"), (20, "graded"),
                                    (64, "gauss"), (64, "repeated"), (64, "graded"), (127, "gauss"),
                                    (128, "gauss"), (128, "graded")])
def test_sym_eigvals_matches_oracle(lib, k, kind):
    """Within 1e-12 of ||A||_F (the stopping bound is 1e-13 of it, plus rounding)."""
    print(f"sym_eigvals k={k} {kind}", flush=True)
    A = sym_case(k, 10 + k, kind)
    # the upper triangle holds NaN: only the lower one may be read
    Ah = np.tril(A) + np.triu(np.full((k, k), np.nan), 1)
    w, sweeps = lib.sym_eigvals(torch.from_numpy(Ah).cuda())
    ref = ospec.sym_eigvals(A)
    got = w.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.abs(got - ref).max() <= 1e-12 * np.linalg.norm(A)
    assert np.all(np.diff(got) <= 0)
    # quadratic convergence: 8-12 sweeps; a cluster of equal eigenvalues converges
    # linearly (the 64 "repeated" case: 22 sweeps in a CPU emulation of the kernel)
    assert 0 <= sweeps <= (30 if kind == "repeated" else 16)


def test_sym_eigvals_diagonal_and_padded_lda(lib):
    print("sym_eigvals diagonal, lda 70", flush=True)
    k, lda = 50, 70
    d = np.random.default_rng(1).standard_normal(k)
    full = np.full((k, lda), np.nan)
    full[:, :k] = np.diag(d)
    Fd = torch.from_numpy(full).cuda()
    w, sweeps = lib.sym_eigvals(Fd[:, :k])
    assert sweeps == 0
    assert np.array_equal(w.cpu().numpy(), np.sort(d)[::-1])


def test_sym_eigvals_rejects_non_finite(lib):
    print("sym_eigvals non-finite", flush=True)
    A = np.eye(8)
    A[5, 2] = np.inf
    with pytest.raises(lib.NmfError) as ei:
        lib.sym_eigvals(torch.from_numpy(A).cuda())
    assert "non-finite" in str(ei.value)
    with pytest.raises(ValueError):
        lib.sym_eigvals(torch.zeros(4, 5, dtype=torch.float64, device="cuda"))


def spectrum_case(m, n, r, kp, q, seed, family):
    X = (datagen.planted_c1(m, n, r, seed)[0] if family == "c1"
         else datagen.planted_parts(m, n, r, seed)[0])
    OL = datagen.gaussian(n, kp, seed, datagen.S_OMEGA_L)
    OR = datagen.gaussian(m, kp, seed, datagen.S_OMEGA_R)
    return X, OL, OR


@pytest.mark.parametrize("m,n,r,kp,q,family", [(512, 256, 10, 20, 2, "c1"), (1000, 300, 5, 9, 1, "parts"),
                                               (400, 4096, 20, 25, 4, "parts"), (1500, 200, 60, 100, 1, "parts")])
def test_sketch_spectrum_matches_oracle(lib, m, n, r, kp, q, family):
    """sigma_j(Q_L^T X) from the GPU compression against the oracle's compression
    of the same X and Omega: within 1e-5 of sigma_1 (the FP32 sketches' rounding,
    far below the 1e-4 the projected data are held to)."""
    print(f"sketch spectrum m={m} n={n} kp={kp} q={q}", flush=True)
    X, OL, OR = spectrum_case(m, n, r, kp, q, 500 + m, family)
    ctx = lib.NMF(m, n, r, kp, q, seed=7)
    with pytest.raises(lib.NmfError):
        ctx.sketch_spectrum()        # no compressed data yet
    ctx.compress(torch.from_numpy(X).cuda(), torch.from_numpy(OL).cuda(), torch.from_numpy(OR).cuda())
    sig = ctx.sketch_spectrum().numpy()
    QL = onmf.compress(X, OL, OR, q)[0]
    ref = ospec.sketch_singular_values(X, QL)
    assert sig.shape == (kp,)
    assert np.abs(sig - ref).max() <= 1e-5 * ref[0]
    assert np.all(np.diff(sig) <= 0) and sig[-1] >= 0
    # repeatable, and unchanged by factor updates
    ctx.init(*(torch.from_numpy(a).cuda() for a in datagen.init_factors(X.mean(), m, n, r, 3)))
    ctx.step(3)
    assert np.array_equal(ctx.sketch_spectrum().numpy(), sig)


@pytest.mark.parametrize("r,q", [(10, 1), (10, 5), (50, 1), (50, 5)])
def test_sweep_points_match_oracle(lib, r, q):
    """Corners of the P1 parameter grid (400 x 4096, k' = r + 5): FastHALS-RP and
    FastHALS errors after 50 iterations against the oracle's, within the 1e-4 gate."""
    print(f"sweep point P1 r={r} q={q}", flush=True)
    name = "P1"
    cfg = datagen.CONFIGS[name]
    m, n, kp, seed = cfg["m"], cfg["n"], r + 5, datagen.cfg_seed(name)
    X = datagen.make_x(name)
    OL = datagen.gaussian(n, kp, seed, datagen.S_OMEGA_L)
    OR = datagen.gaussian(m, kp, seed, datagen.S_OMEGA_R)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    Xd = torch.from_numpy(X).cuda()
    ctx = lib.NMF(m, n, r, kp, q, seed=seed)
    ctx.compress(Xd, torch.from_numpy(OL).cuda(), torch.from_numpy(OR).cuda())
    ctx.init(torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda())
    ctx.step(50)
    ref = onmf.fasthals_rp(X, OL, OR, q, W0, H0, 50)
    assert abs(ctx.residual(Xd) - ref["e"]) <= 1e-4
    if q == 1:
        ctx.init(torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda())
        ctx.fasthals_step(Xd, 50)
        Wu, Hu = onmf.fasthals(X, W0, H0, 50)
        assert abs(ctx.residual(Xd) - onmf.rel_error(X, Wu, Hu)) <= 1e-4


def test_sym_eigvals_degenerate_inputs(lib):
    """A zero matrix (no sweep), and off-diagonal entries so small that the
    rotation's tau overflows the plain formula (its guarded branch)."""
    print("sym_eigvals degenerate", flush=True)
    w, sweeps = lib.sym_eigvals(torch.zeros(5, 5, dtype=torch.float64, device="cuda"))
    assert sweeps == 0 and np.array_equal(w.cpu().numpy(), np.zeros(5))
    # the (1, 3) entry keeps the sweeps running; the (0, 2) pair then has
    # tau ~ 5e159, where t = 1 / (2 tau) replaces the formula that would overflow
    A = np.diag([3.0, 1.0, 2.0, -1.0])
    A[2, 0] = A[0, 2] = 1e-160
    A[3, 1] = A[1, 3] = 0.5
    w, sweeps = lib.sym_eigvals(torch.from_numpy(A).cuda())
    got = w.cpu().numpy()
    assert sweeps >= 1 and np.all(np.isfinite(got))
    assert np.abs(got - ospec.sym_eigvals(A)).max() <= 1e-12 * np.linalg.norm(A)
    # only a pair of tiny entries: below the stopping bound from the start
    B = np.diag([3.0, 1.0, 2.0, -1.0])
    B[3, 1] = B[1, 3] = 1e-300
    w, sweeps = lib.sym_eigvals(torch.from_numpy(B).cuda())
    assert sweeps == 0 and np.array_equal(w.cpu().numpy(), np.array([3.0, 2.0, 1.0, -1.0]))
