"""Parity at the largest single-GPU size: X 262144 x 16384 (16 GiB, the dyadic
parts family formed on the device), r = 128, k' = 256, q = 1, 300 iterations,
against the FP64 oracle's stored errors (tests/golden/oracle_errors.json,
written by make_oracle_errors.py from the oracle alone); the device-formed X
against the oracle's own construction of the same rows; and the split-BF16
products at the full sizes of both parts workloads on sampled outputs (GPU)."""
import json
import os

import numpy as np
import pytest
import torch

import datagen
from datagen import device as ddev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_errors.json")
NAME = "c5"


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


@pytest.fixture(scope="module")
def c5(lib):
    print("c5: forming X 262144 x 16384 on the device", flush=True)
    Xd, _, mean = ddev.dyadic_parts_x(torch, lib.gaussian, NAME)
    c = datagen.CONFIGS[NAME]
    W0, H0 = datagen.init_factors(mean, c["m"], c["n"], c["r"], datagen.cfg_seed(NAME))
    yield Xd, torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda(), mean
    del Xd
    torch.cuda.empty_cache()


def test_c5_device_rows_match_the_oracle_construction(lib, c5):
    """Sampled rows (head, middle, tail) of the device X equal the oracle's
    host construction bit for bit, but for the rare noise value whose FP64
    Box-Muller result rounds to the other side of an FP32 boundary on one side
    (then the entry differs by at most one FP32 ulp); the FP64 means agree."""
    from oracle import inputs
    Xd, _, _, mean = c5
    ref = json.load(open(GOLDEN))[NAME]
    assert abs(mean - ref["x_mean"]) <= 1e-12 * ref["x_mean"]
    for row0 in (0, 131072 + 4096, 262144 - 8):
        host = inputs.dyadic_parts_rows(NAME, row0, 8)
        got = Xd[row0:row0 + 8].cpu().numpy()
        diff = got != host
        print(f"  rows {row0}..{row0 + 7}: {int(diff.sum())} of {diff.size} differ", flush=True)
        assert int(diff.sum()) <= 2
        if diff.any():   # one ulp of the noise moves the rounded sum by at most one ulp of X
            assert np.all(np.abs(got[diff] - host[diff]) <= np.spacing(np.abs(host[diff])))


def _run_to_checkpoints(lib, ctx, Xd, ref, iters, gate, tag):
    done = checked = 0
    worst = 0.0
    for it in sorted(int(k) for k in ref["curve"]):
        if it > iters:
            continue
        ctx.step(it - done)
        done = it
        e = ctx.residual(Xd)
        e_ref = ref["curve"][str(it)]
        worst = max(worst, abs(e - e_ref))
        print(f"  {tag} it={it:4d} e_gpu={e:.8e} e_oracle={e_ref:.8e} diff={abs(e - e_ref):.2e}", flush=True)
        assert abs(e - e_ref) <= gate, it
        # the split-BF16 residual of the stopping test: within its bound of the exact one
        es, bound, exact = ctx.residual_check(Xd, 10.0)
        assert not exact and abs(es - e) <= bound <= 1.2e-4, it
        checked += 1
    assert checked >= 8
    return worst


@pytest.mark.parametrize("up", [0, 1])
def test_c5_full_size_plain_fp32_matches_oracle(lib, c5, up):
    """The paper's method at full size with the benchmark's launch configuration:
    FP32 range finder and sketches, device-drawn test matrices, cold factors; the
    update products on FP32 MFMA (up 0, the plain method) or on split-BF16 MFMA
    (up 1, as in the low-precision variants)."""
    Xd, W0d, H0d, _ = c5
    c = datagen.CONFIGS[NAME]
    ref = json.load(open(GOLDEN))[NAME]
    ctx = lib.NMF(c["m"], c["n"], c["r"], c["kp"], c["q"], seed=datagen.cfg_seed(NAME), update_prec=up)
    ctx.compress(Xd)
    ctx.init(W0d, H0d)
    assert ctx.sync() == 0
    QL, QR, _, _ = ctx.state()
    for Q in (QL, QR):
        Qd = Q.double()
        assert (Qd.T @ Qd - torch.eye(c["kp"], dtype=torch.float64, device=Qd.device)).abs().max().item() < 5e-6
    worst = _run_to_checkpoints(lib, ctx, Xd, ref, c["iters"], 1e-4, f"fp32 up={up}")
    print(f"  largest gap {worst:.2e}", flush=True)
    Wg, Hg = ctx.factors()
    assert (Wg >= 0).all().item() and (Hg >= 0).all().item()
    ctx.close()


def test_c5_full_size_fp8_refined_matches_the_oracle_low_precision_model(lib, c5):
    """FP8 e4m3 range finder (128 x 128 block scales), one refinement power
    iteration per side on X itself, the sketches and the update loop on
    split-BF16 products (the benchmark's headline configuration): the
    error at every stored checkpoint within the 1e-4 gate of the oracle's model of
    the same rounding (R_q: the quantised X and thin operands, the split
    products), and the gap to the exact FP64 run (R_true) printed.  Against R_true
    the transient differs by up to about 8e-4 (measured at iteration 2: the FP8
    basis spans a slightly different noise subspace, and the descent at this size
    is steep)."""
    golden = json.load(open(GOLDEN))
    key = "c5_fp8_refine2_lps2"
    if key not in golden:
        pytest.skip("the oracle's low-precision model at this size is not stored (make_oracle_errors.py c5:fp8:2:2)")
    Xd, W0d, H0d, _ = c5
    c = datagen.CONFIGS[NAME]
    ctx = lib.NMF(c["m"], c["n"], c["r"], c["kp"], c["q"], seed=datagen.cfg_seed(NAME), prec=lib.NMF_FP8_E4M3,
                  refine_fp32=2, lowp_sketches=2, update_prec=1)
    ctx.compress(Xd)
    ctx.init(W0d, H0d)
    assert ctx.sync() == 0
    worst = _run_to_checkpoints(lib, ctx, Xd, golden[key], c["iters"], 1e-4, "fp8 vs R_q")
    print(f"  largest gap to R_q {worst:.2e}; R_true(300) {golden[NAME]['e']:.8e}, "
          f"R_q(300) {golden[key]['e']:.8e}", flush=True)
    ctx.close()


def _index_matrix(torch_mod, rows, cols, device, block=4096):
    """X[i, j] = ((7 i + 13 j) mod 251) / 256: exact in FP32 and BF16-split, cheap
    to evaluate anywhere (formed in blocks of rows)."""
    X = torch_mod.empty(rows, cols, device=device, dtype=torch_mod.float32)
    j = torch_mod.arange(cols, device=device, dtype=torch_mod.int32)[None, :]
    for i0 in range(0, rows, block):
        i = torch_mod.arange(i0, min(rows, i0 + block), device=device, dtype=torch_mod.int32)[:, None]
        X[i0:i0 + block] = ((7 * i + 13 * j) % 251).to(torch_mod.float32) / 256.0
    return X


@pytest.mark.parametrize("m,n,k", [(65536, 4096, 64), (262144, 16384, 256)])
def test_split_products_full_size_sampled(lib, m, n, k):
    """Split-BF16 X B and X^T B at the full sizes and launch configurations of the
    two parts workloads (split-K counts, K-order rotation, 32-bit in-tile
    offsets), on an index-formula X, checked on sampled rows of the result
    against FP64 sums within the split bound."""
    print(f"split products full size {m}x{n} k={k}", flush=True)
    Xd = _index_matrix(torch, m, n, "cuda")
    g = np.random.default_rng(m + k)
    for at in (0, 1):
        K = m if at else n
        B = g.standard_normal((K, k)).astype(np.float32)
        C = lib.gemm_split(Xd, at, torch.from_numpy(B).cuda()).cpu().numpy().astype(np.float64)
        M = n if at else m
        rows = np.unique(np.concatenate([[0, 1, M - 1], g.integers(0, M, 5)]))
        kk = np.arange(K, dtype=np.int64)
        for i in rows:
            x = (((7 * kk + 13 * i) % 251) if at else ((7 * i + 13 * kk) % 251)) / 256.0   # row i of op(X)
            exact = x @ B.astype(np.float64)
            bound = (3.1 * 2.0 ** -16 + 3.0 * K * 2.0 ** -24) * (np.abs(x) @ np.abs(B.astype(np.float64))) + 1e-30
            assert np.all(np.abs(C[i] - exact) <= bound), (at, int(i))
        print(f"  at={at}: {len(rows)} rows within the bound", flush=True)
    del Xd
    torch.cuda.empty_cache()
