"""Low-precision compression extension on the GPU: quantisers bit-exact against
library casts and the oracle's block-scale model, low-precision products
against FP64 on the same rounded operands, and whole runs against the oracle."""
import numpy as np
import pytest
import torch

import datagen
from oracle import nmf as onmf
from oracle import quant

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


def _x(m, n, seed, spread=True):
    g = np.random.default_rng(seed)
    X = g.random((m, n)) * (10.0 ** g.integers(-3, 3, (m, n)) if spread else 1.0)
    X[: m // 7, : n // 5] = 0.0                       # an all-zero region (zero tiles)
    return X.astype(np.float32)


@pytest.mark.parametrize("m,n", [(300, 200), (128, 128), (1000, 36), (64, 1100), (77, 130), (2, 4)])
def test_quantize_bf16_bit_exact(lib, m, n):
    print(f"quant bf16 {m}x{n}", flush=True)
    X = _x(m, n, m + n)
    Xq, XqT, _ = lib.quantize_x(torch.from_numpy(X).cuda(), lib.NMF_BF16)
    Xq, XqT = Xq.cpu(), XqT.cpu()
    want = torch.from_numpy(X).to(torch.bfloat16).view(torch.int16)
    assert torch.equal(Xq[:, :n], want)
    assert torch.equal(XqT[:, :m], want.T.contiguous())
    assert int(Xq[:, n:].abs().sum()) == 0 and int(XqT[:, m:].abs().sum()) == 0


@pytest.mark.parametrize("m,n", [(300, 200), (256, 384), (1000, 36)])
def test_quantize_fp8_matches_block_model(lib, m, n):
    print(f"quant fp8 {m}x{n}", flush=True)
    X = _x(m, n, 7 * m + n)
    Xq, XqT, E = lib.quantize_x(torch.from_numpy(X).cuda(), lib.NMF_FP8_E4M3)
    Xq, XqT, E = Xq.cpu(), XqT.cpu(), E.cpu().numpy()
    deq_ref, E_ref, codes_ref = quant.e4m3_block_quantise(X.astype(np.float64))
    assert np.array_equal(E, E_ref)
    codes = Xq[:, :n].contiguous().view(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(codes, codes_ref)
    codesT = XqT[:, :m].contiguous().view(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(codesT, codes_ref.T)
    assert int(Xq[:, n:].to(torch.int32).sum()) == 0


@pytest.mark.parametrize("fmt,m,n,k,side", [("bf16", 1000, 300, 20, 0), ("bf16", 1000, 300, 64, 1),
                                            ("bf16", 4096, 2048, 128, 1), ("fp8", 1000, 300, 20, 0),
                                            ("fp8", 1000, 300, 64, 1), ("fp8", 2048, 4096, 128, 0),
                                            ("bf16", 300, 5000, 256, 0), ("fp8", 513, 700, 256, 1),
                                            ("fp8", 1000, 300, 21, 1), ("fp8", 3000, 260, 256, 1)])
def test_lowp_products(lib, fmt, m, n, k, side):
    print(f"lowp gemm {fmt} {m}x{n} k={k} side={side}", flush=True)
    X = _x(m, n, m + 3 * n + k, spread=False)
    prec = lib.NMF_BF16 if fmt == "bf16" else lib.NMF_FP8_E4M3
    Xd = torch.from_numpy(X).cuda()
    Xq, XqT, E = lib.quantize_x(Xd, prec)
    K = m if side else n
    B = np.random.default_rng(k).standard_normal((K, k)).astype(np.float32)
    tn = -(-n // 128)
    A = XqT if side else Xq
    ea = (1, tn) if side else (tn, 1)
    C = lib.gemm_lowp(prec, A, K, torch.from_numpy(B).cuda(), E, ea).cpu().numpy().astype(np.float64)
    Xdeq = onmf.quantize_data(X, fmt)
    Aref = Xdeq.T if side else Xdeq
    Bq = onmf.quantize_thin(B, fmt)
    ref = Aref @ Bq
    bound = 2.0 * K * 2.0 ** -24 * (np.abs(Aref) @ np.abs(Bq)) + 1e-30
    assert np.all(np.abs(C - ref) <= bound)


@pytest.mark.parametrize("fmt,m,n,k,side", [("bf16", 1000, 300, 64, 0), ("bf16", 4096, 512, 64, 1),
                                            ("fp8", 1000, 300, 64, 0), ("fp8", 4096, 512, 32, 1)])
def test_prepared_product_matches_full_product(lib, fmt, m, n, k, side):
    """The product kernel on a prepared thin operand, with its split-K partials
    summed in the library's order (z ascending, FP32), is bit-identical to the
    one-call product."""
    print(f"prepared lowp {fmt} {m}x{n} k={k} side={side}", flush=True)
    X = _x(m, n, 7 * m + n, spread=False)
    prec = lib.NMF_BF16 if fmt == "bf16" else lib.NMF_FP8_E4M3
    Xq, XqT, E = lib.quantize_x(torch.from_numpy(X).cuda(), prec)
    K = m if side else n
    B = torch.from_numpy(np.random.default_rng(k + side).standard_normal((K, k)).astype(np.float32)).cuda()
    tn = -(-n // 128)
    A = XqT if side else Xq
    ea = (1, tn) if side else (tn, 1)
    full = lib.gemm_lowp(prec, A, K, B, E, ea).cpu().numpy()
    pp = lib.LowpProduct(prec, A, K, B, E, ea)
    pp.run()
    parts = pp.part.cpu().numpy()
    acc = np.zeros_like(parts[0])
    for z in range(parts.shape[0]):
        acc = (acc + parts[z]).astype(np.float32)
    assert np.array_equal(acc, full)


@pytest.mark.parametrize("m,n,k", [(1000, 300, 64), (4096, 512, 32), (300, 200, 20), (513, 700, 128),
                                   (130, 8, 5), (65, 1028, 64)])
def test_transposed_product_matches_transposed_copy(lib, m, n, k):
    """X^T B on the row-major BF16 copy (tiles transposed in LDS) is bit-identical
    to the product on the transposed copy XqT: same tiles, same K order, rows past
    m read as zero either way."""
    print(f"bf16 X^T B transposed-in-LDS {m}x{n} k={k}", flush=True)
    X = _x(m, n, 5 * m + n, spread=False)
    Xq, XqT, _ = lib.quantize_x(torch.from_numpy(X).cuda(), lib.NMF_BF16)
    B = torch.from_numpy(np.random.default_rng(m + k).standard_normal((m, k)).astype(np.float32)).cuda()
    ref = lib.LowpProduct(lib.NMF_BF16, XqT, m, B)
    at = lib.LowpProduct(lib.NMF_BF16, Xq, m, B, at=True, Kpad=XqT.shape[1], M=n)
    assert at.splits == ref.splits and at.M == ref.M
    assert torch.equal(at.Bt, ref.Bt)
    ref.run()
    at.run()
    torch.cuda.synchronize()
    assert torch.equal(at.part, ref.part)


@pytest.mark.parametrize("rows,cols,k", [(300, 200, 64), (1000, 36, 20), (77, 130, 5), (2, 4, 1), (4096, 256, 64)])
def test_prepared_thin_operand_bit_exact(lib, rows, cols, k):
    """The transposed BF16 copy of a thin operand (K x k) is torch's
    round-to-nearest-even cast, zero in the padding columns."""
    print(f"prep thin bf16 K={rows} k={k}", flush=True)
    g = np.random.default_rng(rows + k)
    B = (g.standard_normal((rows, k)) * 10.0 ** g.integers(-4, 4, (rows, k))).astype(np.float32)
    X = _x(cols, rows, 3)
    Xq, XqT, E = lib.quantize_x(torch.from_numpy(X).cuda(), lib.NMF_BF16)
    pp = lib.LowpProduct(lib.NMF_BF16, Xq, rows, torch.from_numpy(B).cuda())
    Bt = pp.Bt.cpu()
    want = torch.from_numpy(B).to(torch.bfloat16).view(torch.int16).T.contiguous()
    assert torch.equal(Bt[:, :rows], want)
    assert int(Bt[:, rows:].abs().sum()) == 0


def _padded(X):
    """Copy of X (FP32) in a buffer whose row stride is a multiple of 4."""
    rows, cols = X.shape
    buf = torch.zeros((rows, -(-cols // 4) * 4), dtype=torch.float32)
    buf[:, :cols] = torch.from_numpy(X)
    return buf.cuda()[:, :cols]


@pytest.mark.parametrize("m,n,k,at", [(1000, 300, 20, 0), (1000, 300, 64, 1), (4096, 2048, 64, 1),
                                      (4096, 2048, 64, 0), (513, 701, 37, 0), (513, 701, 37, 1),
                                      (130, 8, 5, 1), (2, 4, 3, 0), (300, 5000, 128, 0), (20000, 64, 64, 1),
                                      (1000, 300, 200, 0), (700, 513, 256, 1), (3001, 515, 140, 0),
                                      (515, 3001, 250, 1), (600, 2000, 129, 1), (9000, 77, 256, 0)])
def test_split_products(lib, m, n, k, at):
    """Split-BF16 product against the oracle's model of the same arithmetic
    (FP64 sums of the three BF16 products), within the FP32 accumulation bound,
    and against the exact product within the split bound."""
    print(f"split gemm {m}x{n} k={k} at={at}", flush=True)
    g = np.random.default_rng(m + 7 * n + k + at)
    X = (g.random((m, n)) * 10.0 ** g.integers(-2, 2, (m, n))).astype(np.float32)
    X[: m // 5, : n // 3] = 0.0
    K = m if at else n
    B = g.standard_normal((K, k)).astype(np.float32)
    C = lib.gemm_split(_padded(X), at, torch.from_numpy(B).cuda()).cpu().numpy().astype(np.float64)
    A = X.T if at else X
    model = onmf.split_product(A, B)
    absprod = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(C - model) <= 3.0 * K * 2.0 ** -24 * absprod + 1e-30)
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.all(np.abs(C - exact) <= (3.1 * 2.0 ** -16 + 3.0 * K * 2.0 ** -24) * absprod + 1e-30)


@pytest.mark.parametrize("m,n,k,at", [(3001, 515, 140, 0), (515, 30001, 200, 1), (4096, 2048, 64, 1),
                                      (70000, 300, 256, 0)])
def test_split_product_prepared_equals_call(lib, m, n, k, at):
    """The prepared split product (thin operand split once, product kernel alone,
    partials summed in ascending order) gives nmf_gemm_split's result bit for bit."""
    print(f"split prepared {m}x{n} k={k} at={at}", flush=True)
    g = np.random.default_rng(m + n + k)
    X = _padded(g.random((m, n)).astype(np.float32))
    K = m if at else n
    B = torch.from_numpy(g.standard_normal((K, k)).astype(np.float32)).cuda()
    ref = lib.gemm_split(X, at, B)
    P = lib.SplitProduct(X, at, B)
    P.run()
    got = P.result()
    print(f"  splits {P.splits}", flush=True)
    assert torch.equal(got, ref)


def test_split_product_bad_arguments(lib):
    X = torch.zeros((64, 30), dtype=torch.float32, device="cuda")      # row stride 30: not a multiple of 4
    B = torch.zeros((30, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.NmfError):
        lib.gemm_split(X, 0, B)
    with pytest.raises(ValueError):
        lib.gemm_split(_padded(np.zeros((64, 32), np.float32)), 0, torch.zeros((31, 8), device="cuda"))


@pytest.mark.parametrize("fmt,refine,lps", [("bf16", 0, 0), ("bf16", 1, 0), ("fp8", 0, 0), ("fp8", 1, 0),
                                            ("bf16", 0, 1), ("bf16", 0, 2), ("fp8", 0, 2)])
def test_lowp_compression_runs(lib, fmt, refine, lps):
    """Whole run with low-precision range-finder products: the error after the
    iterations is compared with the oracle's model of the same rounding (R_q)
    and with the exact FP64 run (R_true); both gaps are printed.  Compared near
    convergence (400 iterations): early iterates depend sensitively on the
    basis of the sketch, which the two sides round differently."""
    print(f"lowp run {fmt} refine={refine} lowp_sketches={lps}", flush=True)
    m, n, r, kp, q, iters = 2000, 512, 10, 20, 2, 400
    seed = 4242
    X = datagen.planted_parts(m, n, r, seed)[0]
    OL = datagen.gaussian(n, kp, seed, datagen.S_OMEGA_L)
    OR = datagen.gaussian(m, kp, seed, datagen.S_OMEGA_R)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    prec = lib.NMF_BF16 if fmt == "bf16" else lib.NMF_FP8_E4M3
    ctx = lib.NMF(m, n, r, kp, q, seed=seed, prec=prec, refine_fp32=refine, lowp_sketches=lps)
    Xd = torch.from_numpy(X).cuda()
    ctx.compress(Xd, torch.from_numpy(OL).cuda(), torch.from_numpy(OR).cuda())
    ctx.init(torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda())
    ctx.step(iters)
    ep = ctx.proxy_residual()            # ||X||^2 from the quantiser when lps == 1, else the X Q_R pass
    e = ctx.residual(Xd)
    ref = onmf.fasthals_rp(X, OL, OR, q, W0, H0, iters, fmt=fmt, refine=bool(refine), lowp_sketches=lps)
    Rq = ref["e"]
    nx2 = float(np.sum(X.astype(np.float64) ** 2))
    ep_ref = onmf.proxy_rel_error(nx2, ref["Xh"], ref["QL"].T @ ref["W"], ref["Ht"])
    assert abs(ep - ep_ref) <= 1e-4
    Rt = onmf.fasthals_rp(X, OL, OR, q, W0, H0, iters)["e"]
    print(f"  e_gpu={e:.6e} R_q={Rq:.6e} R_true={Rt:.6e} |gpu-Rq|={abs(e - Rq):.2e} |gpu-Rtrue|={abs(e - Rt):.2e}",
          flush=True)
    assert abs(e - Rq) <= 1e-4
    assert abs(e - Rt) <= 1e-4
