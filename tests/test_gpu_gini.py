"""Gini coefficient of B (Sec 5.1) on the GPU (nmf_gini, a device radix sort and
FP64 sums) against the oracle's gini (sort + the printed formula) and closed
forms (GPU)."""
import numpy as np
import pytest
import torch

from oracle import nmf as onmf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


@pytest.mark.parametrize("rows,cols,kind", [(1, 1, "u"), (1, 5, "u"), (7, 3, "u"), (4096, 1, "u"), (4097, 3, "u"),
                                            (1000, 37, "sparse"), (16384, 128, "sparse"), (300, 10, "ties"),
                                            (5000, 60, "wide_range"), (513, 7, "signed")])
def test_gini_matches_oracle(lib, rows, cols, kind):
    print(f"gini {rows}x{cols} {kind}", flush=True)
    g = np.random.default_rng(rows * 131 + cols)
    if kind == "u":
        B = g.random((rows, cols))
    elif kind == "sparse":      # exact zeros (ties) as the L1 term leaves them
        B = g.random((rows, cols)) * (g.random((rows, cols)) < 0.3)
    elif kind == "ties":        # few distinct values
        B = g.integers(0, 4, (rows, cols)).astype(np.float64) / 4.0
    elif kind == "wide_range":  # keys spread over many exponents
        B = np.exp(g.uniform(-40.0, 40.0, (rows, cols)))
    else:                       # negative entries and both zeros order as values
        B = g.standard_normal((rows, cols))
        B[0, 0], B[1, 1] = 0.0, -0.0
    B32 = B.astype(np.float32)
    got = lib.gini(torch.from_numpy(B32).cuda())
    ref = onmf.gini(B32.astype(np.float64))
    print(f"  gpu {got:.15f} oracle {ref:.15f}", flush=True)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_gini_strided_view(lib):
    """ldb > cols: the columns of a view of a wider matrix."""
    g = np.random.default_rng(3)
    full = g.random((2000, 48)).astype(np.float32)
    Bd = torch.from_numpy(full).cuda()[:, 5:40]
    ref = onmf.gini(full[:, 5:40].astype(np.float64))
    assert abs(lib.gini(Bd) - ref) <= 1e-12


def test_gini_closed_forms(lib):
    """A constant matrix has G = 0; one nonzero entry among N gives (N - 1) / N;
    G does not depend on the order of the entries."""
    assert abs(lib.gini(torch.full((300, 7), 2.5, device="cuda"))) <= 1e-15
    for N in (1, 2, 5000, 123457):
        B = torch.zeros(N, 1, device="cuda")
        B[N // 3, 0] = 7.0
        assert abs(lib.gini(B) - (N - 1) / N) <= 1e-14
    g = np.random.default_rng(9)
    B = g.random((4000, 16)).astype(np.float32)
    perm = g.permutation(B.size)
    a = lib.gini(torch.from_numpy(B).cuda())
    b = lib.gini(torch.from_numpy(B.reshape(-1)[perm].reshape(16, 4000).copy()).cuda())
    assert a == b


def test_gini_undefined_inputs(lib):
    with pytest.raises(lib.NmfError):
        lib.gini(torch.zeros(10, 10, device="cuda"))
    B = torch.ones(10, 10, device="cuda")
    B[3, 3] = float("nan")
    with pytest.raises(lib.NmfError):
        lib.gini(B)


def test_gini_of_a_constrained_factor(lib):
    """Sec 5.1's use: B after FastHALS-RP with the L1 term (alpha > 0) is sparser
    than without it, and the GPU Gini of the factor equals the oracle's."""
    import datagen
    m, n, r, kp, q = 512, 256, 10, 20, 2
    seed = datagen.cfg_seed("c1")
    X, _, _ = datagen.planted_c1(m, n, r, seed)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    ginis = []
    for alpha in (0.0, 0.5):
        ctx = lib.NMF(m, n, r, kp, q, seed=5, normalize=0, alpha=alpha)
        Xd = torch.from_numpy(X).cuda()
        ctx.compress(Xd)
        ctx.init(torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda())
        ctx.step(20)
        _, Hg = ctx.factors()
        gv = lib.gini(Hg)
        assert abs(gv - onmf.gini(Hg.cpu().numpy().astype(np.float64))) <= 1e-12
        ginis.append(gv)
        ctx.close()
    print(f"  Gini of B: alpha 0 {ginis[0]:.6f}, alpha 0.5 {ginis[1]:.6f}", flush=True)
    assert ginis[1] > ginis[0]
