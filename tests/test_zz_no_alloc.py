"""The allocation-free product entry point (nmf_gemm_noalloc) against nmf_gemm
with a caller workspace: two calls in a row on one GPU, the second with a
smaller, ragged input, each equal to the workspace call bit for bit (same
kernels and split-K choice) and within the FP32 accumulation bound of the FP64
product.  The size rejection is host logic and is checked without a GPU."""
import ctypes

import numpy as np
import pytest

from paper_1712_02248_amd import nmfrp


def _bound(A64, B64, K):
    # |fl(A B) - A B| <= 2 K 2^-24 |A| |B| elementwise (FP32 products and sums)
    return 2.0 * K * 2.0 ** -24 * (np.abs(A64) @ np.abs(B64))


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_point_twice():
    import torch
    nmfrp.load()
    dev = torch.device("cuda:0")
    g = np.random.default_rng(1712022480)
    # first call: X^T B at 65536 x 4096, k' = 64 (32 split-K slices, 32 MiB of partials);
    # second call: a smaller, ragged X B (fewer slices, the array keeps the first call's data)
    cases = [(65536, 4096, 64, True), (3000, 1000, 40, False)]
    for rows, cols, N, at in cases:
        X = g.random((rows, cols), dtype=np.float32)
        K, M = (rows, cols) if at else (cols, rows)
        B = g.standard_normal((K, N), dtype=np.float32)
        Xd, Bd = torch.from_numpy(X).to(dev), torch.from_numpy(B).to(dev)
        print(f"[noalloc] {'X^T B' if at else 'X B'} M={M} N={N} K={K}", flush=True)
        ref = nmfrp.gemm(Xd, Bd, a_trans=at)
        out = nmfrp.gemm_noalloc(Xd, Bd, a_trans=at)
        torch.cuda.synchronize()
        ref_h, out_h = ref.cpu().numpy(), out.cpu().numpy()
        assert np.array_equal(out_h, ref_h)
        A64 = X.astype(np.float64).T if at else X.astype(np.float64)
        B64 = B.astype(np.float64)
        exact = A64 @ B64
        assert np.all(np.abs(out_h - exact) <= _bound(A64, B64, K))


def test_noalloc_rejects_products_beyond_its_scratch():
    lib = nmfrp.load()
    # X^T B with M = 48000, N = 256, K = 512: two split-K slices of 48000 x 256
    # floats (98 MB) exceed the 64 MiB array; the call returns before any GPU work
    fake = ctypes.c_void_p(1 << 20)
    st = lib.nmf_gemm_noalloc(fake, 48000, 1, fake, 256, fake, 256, 48000, 256, 512, None)
    assert st == -1
    assert b"64 MiB" in lib.nmf_last_error(None)
