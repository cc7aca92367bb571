"""Learned warm start on the HIP path (through the C ABI) against the FP64
oracle on the same seeded inputs: MLP loss and gradients, inference, Adam
training, column-NNLS training targets, and the per-row warm/cold selection of
nmf_init_learned (GPU)."""
import numpy as np
import pytest
import torch

import datagen
from oracle import mlp as omlp
from oracle import nmf as onmf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp
    nmfrp.load()
    return nmfrp


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def pairs(k, r, B, seed):
    """Non-negative inputs of mixed norms (one zero row) and targets."""
    g = np.random.default_rng(seed)
    X = (g.random((B, k)) * g.uniform(0.1, 20.0, (B, 1))).astype(np.float32)
    X[B // 3] = 0.0
    T = (g.random((B, r)) * np.linalg.norm(X, axis=1, keepdims=True) / np.sqrt(k)).astype(np.float32)
    return X, T


def rel_norm(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# (128, 512, 64): the network of the document-count workload (k' = 128, r = 64)
@pytest.mark.parametrize("k,hdim,r,B", [(20, 96, 10, 300), (64, 512, 32, 1024), (128, 512, 64, 1024), (5, 7, 3, 1)])
def test_loss_and_gradients_match_oracle(lib, k, hdim, r, B):
    print(f"mlp loss/grad k={k} h={hdim} r={r} B={B}", flush=True)
    p0 = datagen.mlp_he_init(k, hdim, r, seed=11)
    X, T = pairs(k, r, B, 12)
    net = lib.Mlp(k, hdim, r, dev(p0), max_batch=max(B, 64))
    L, g = net.loss_grad(dev(X), dev(T))
    P = omlp.unflatten(p0.astype(np.float64), k, hdim, r)
    Lr, gr = omlp.loss_grad(P, X.astype(np.float64), T.astype(np.float64))
    assert abs(L - Lr) <= 1e-5 * abs(Lr)
    gg = omlp.unflatten(g.cpu().numpy(), k, hdim, r)
    for name, a, b in zip(omlp.LAYER_NAMES, gg, gr):
        assert rel_norm(a, b) <= 1e-4, name


def test_inference_matches_oracle(lib):
    print("mlp inference", flush=True)
    k, hdim, r = 64, 512, 32
    p0 = datagen.mlp_he_init(k, hdim, r, seed=13)
    X, _ = pairs(k, r, 5000, 14)       # two chunks of the 4096-row workspace
    net = lib.Mlp(k, hdim, r, dev(p0), max_batch=4096)
    Y = net.infer(dev(X)).cpu().numpy()
    ref = omlp.infer(omlp.unflatten(p0.astype(np.float64), k, hdim, r), X.astype(np.float64))
    assert np.all(Y >= 0)
    assert np.all(Y[5000 // 3] == 0)
    scale = np.abs(ref).max(axis=1, keepdims=True) + 1e-30
    assert np.max(np.abs(Y - ref) / scale) <= 1e-4


def test_params_roundtrip_and_errors(lib):
    k, hdim, r = 6, 10, 3
    p0 = dev(datagen.mlp_he_init(k, hdim, r, seed=1))
    net = lib.Mlp(k, hdim, r, p0, max_batch=8)
    assert torch.equal(net.params(), p0)
    p1 = p0 * 2
    net.set_params(p1)
    assert torch.equal(net.params(), p1)
    X, T = pairs(k, r, 9, 2)
    with pytest.raises(lib.NmfError):
        net.loss_grad(dev(X), dev(T))      # batch above max_batch
    with pytest.raises(lib.NmfError):
        net.train(dev(X), dev(T), epochs=1, batch=16, lr=1e-3)


def oracle_train(p0, X, T, order, epochs, batch, lr, k, hdim, r):
    P = omlp.unflatten(p0.astype(np.float64), k, hdim, r)
    m = [np.zeros_like(p) for p in P]
    v = [np.zeros_like(p) for p in P]
    t = 0
    hist = []
    n = X.shape[0]
    for e in range(epochs):
        ls = []
        for b0 in range(0, n, batch):
            idx = order[e, b0:b0 + batch]
            L, g = omlp.loss_grad(P, X[idx].astype(np.float64), T[idx].astype(np.float64))
            t += 1
            P, m, v = omlp.adam_step(P, g, m, v, t, lr)
            ls.append(L)
        hist.append(float(np.mean(ls)))
    return P, hist


def test_adam_training_matches_oracle(lib):
    """A few Adam passes with a ragged last batch and per-pass permutations.
    Adam divides by sqrt(v), so FP32 gradient noise moves tiny-gradient entries
    by up to lr per step; the check is on the loss history and on the update
    p - p0 of each tensor (relative norm)."""
    print("mlp adam training", flush=True)
    k, hdim, r, n, epochs, batch, lr = 20, 96, 10, 700, 3, 256, 1e-3
    p0 = datagen.mlp_he_init(k, hdim, r, seed=21)
    X, T = pairs(k, r, n, 22)
    order = datagen.batch_orders(n, epochs, seed=23)
    net = lib.Mlp(k, hdim, r, dev(p0), max_batch=batch)
    hist = net.train(dev(X), dev(T), epochs, batch, lr,
                     order=torch.from_numpy(order.reshape(-1)).cuda())
    P, hr = oracle_train(p0, X, T, order, epochs, batch, lr, k, hdim, r)
    assert np.allclose(hist, hr, rtol=1e-4)
    pg = omlp.unflatten(net.params().cpu().numpy(), k, hdim, r)
    P0 = omlp.unflatten(p0.astype(np.float64), k, hdim, r)
    for name, a, b, c in zip(omlp.LAYER_NAMES, pg, P, P0):
        assert rel_norm(a - c, b - c) <= 2e-2, name
    assert hist[-1] < hist[0]


def test_training_natural_order_and_convergence(lib):
    """Natural order (no permutation) on a linear-in-x target: the loss falls by
    a large factor, and GPU and oracle agree on the first pass."""
    print("mlp training convergence", flush=True)
    k, hdim, r, n = 16, 64, 6, 2048
    g = np.random.default_rng(31)
    A = g.random((k, r))
    X = g.random((n, k)).astype(np.float32)
    T = (X @ A).astype(np.float32)
    p0 = datagen.mlp_he_init(k, hdim, r, seed=32)
    net = lib.Mlp(k, hdim, r, dev(p0), max_batch=512)
    hist = net.train(dev(X), dev(T), 40, 256, 3e-3)
    order = np.tile(np.arange(n, dtype=np.int32), (1, 1))
    _, hr = oracle_train(p0, X, T, order, 1, 256, 3e-3, k, hdim, r)
    assert abs(hist[0] - hr[0]) <= 1e-4 * hr[0]
    assert hist[-1] < 0.02 * hist[0]


@pytest.mark.parametrize("k,r,rows,sweeps", [(20, 10, 1000, 50), (64, 32, 3000, 200), (128, 64, 2000, 50),
                                             (7, 1, 5, 3)])
def test_nnls_rows_match_oracle(lib, k, r, rows, sweeps):
    print(f"nnls rows k={k} r={r} rows={rows}", flush=True)
    g = np.random.default_rng(41)
    Wh = g.random((k, r)).astype(np.float32)
    H = np.maximum(g.standard_normal((rows, r)), 0)
    Xr = (H @ Wh.T.astype(np.float64) + 0.05 * g.standard_normal((rows, k))).astype(np.float32)
    out = lib.nnls_rows(dev(Xr), dev(Wh), sweeps).cpu().numpy()
    ref = onmf.column_nnls(Xr.astype(np.float64), Wh.astype(np.float64), sweeps)
    assert np.all(out >= 0)
    scale = np.abs(ref).max() + 1e-30
    assert np.abs(out - ref).max() <= 1e-4 * scale
    # continuing from given rows
    H0 = np.maximum(g.standard_normal((rows, r)), 0).astype(np.float32)
    out2 = lib.nnls_rows(dev(Xr), dev(Wh), sweeps, out=dev(H0), warm=True).cpu().numpy()
    ref2 = onmf.column_nnls(Xr.astype(np.float64), Wh.astype(np.float64), sweeps, Ht0=H0)
    assert np.abs(out2 - ref2).max() <= 1e-4 * (np.abs(ref2).max() + 1e-30)


def test_init_learned_selection_matches_oracle(lib):
    """nmf_init_learned against the oracle run on its own compression of the same
    seeded inputs: the network's rows on the aligned inputs x-tilde = M x-hat
    (M = G^T Q_L), per-row rejection by rho(h) = ||x-hat - Q_L^T W_ref h||^2, the
    optional column-NNLS refinement, and the first iteration from the selected
    factors.  Each side forms M and Q_L^T W_ref from its own Q_L; all of these
    are independent of the basis chosen for range(Q_L)."""
    print("init_learned selection", flush=True)
    m, n, r, kp, q = 512, 256, 10, 20, 2
    seed = datagen.cfg_seed("c1")
    X = datagen.planted_c1(m, n, r, seed)[0]
    OL = datagen.gaussian(n, kp, seed, datagen.S_OMEGA_L)
    OR = datagen.gaussian(m, kp, seed, datagen.S_OMEGA_R)
    W0, _ = datagen.init_factors(X.mean(), m, n, r, seed)
    G = datagen.gaussian(m, kp, seed + 1, datagen.S_FRESH)
    Wref = datagen.uniform((m, r), seed + 2, datagen.S_FRESH)
    # cold rows: zero on even rows (an untrained net loses to them), far off on
    # odd rows (the net wins there)
    Hcold = (1e3 * datagen.uniform((n, r), seed + 3, datagen.S_FRESH)).astype(np.float32)
    Hcold[0::2] = 0.0
    hdim = 64
    p0 = datagen.mlp_he_init(kp, hdim, r, seed=52)
    # ---- oracle
    QL, QR, Xh, Xc = onmf.compress(X, OL, OR, q)
    M = G.T.astype(np.float64) @ QL
    Wh = QL.T @ Wref.astype(np.float64)
    P = omlp.unflatten(p0.astype(np.float64), kp, hdim, r)
    Hn = omlp.infer(P, Xh @ M.T)
    Hsel, rej = omlp.select_warm(Xh, Wh, Hn, Hcold)
    rho_n = np.sum((Xh - Hn @ Wh.T) ** 2, 1)
    rho_c = np.sum((Xh - Hcold.astype(np.float64) @ Wh.T) ** 2, 1)
    clear = np.abs(rho_n - rho_c) > 1e-3 * rho_c
    assert 0 < rej.sum() < n and clear.sum() > 0.9 * n        # both branches exercised
    Href = onmf.column_nnls(Xh, Wh, 7, Ht0=Hsel)
    W1, H1 = onmf.fasthals_rp_iteration(W0, Hsel, Xh, Xc, QL, QR, normalize=1)
    # ---- HIP path
    from paper_1712_02248_amd import warmstart
    ctx = lib.NMF(m, n, r, kp, q, seed=7)
    ctx.compress(dev(X), dev(OL), dev(OR))
    net = lib.Mlp(kp, hdim, r, dev(p0), max_batch=100)      # three inference chunks
    nrej = warmstart.warm_init(ctx, net, dev(G), dev(Wref), Ht_cold=dev(Hcold), W0=dev(W0), count=True)
    Wg, Hg = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    assert np.array_equal(Wg, W0.astype(np.float64))
    gpu_rej = np.all(Hg == Hcold, axis=1)
    assert np.array_equal(gpu_rej[clear], rej[clear])
    assert abs(nrej - rej.sum()) <= np.sum(~clear)
    scale = np.abs(Hsel).max(axis=1, keepdims=True) + 1e-30
    assert np.max((np.abs(Hg - Hsel) / scale)[clear]) <= 1e-4
    ctx.step(1)
    Wg1, Hg1 = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    assert rel_norm(Wg1, W1) <= 1e-4 and rel_norm(Hg1, H1) <= 1e-4
    # with the refinement sweeps
    ctx.compress(dev(X), dev(OL), dev(OR))
    warmstart.warm_init(ctx, net, dev(G), dev(Wref), Ht_cold=dev(Hcold), W0=dev(W0), refine_sweeps=7)
    _, Hr = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    assert np.max((np.abs(Hr - Href) / (np.abs(Href).max(axis=1, keepdims=True) + 1e-30))[clear]) <= 1e-4
    rho_r = np.sum((Xh - Hr @ Wh.T) ** 2, 1)
    assert np.all(rho_r <= np.minimum(rho_n, rho_c) * (1 + 1e-4))    # never worse than cold
    # the same from the reference fit itself (alignment products formed inside the library)
    ctx.compress(dev(X), dev(OL), dev(OR))
    nrej2 = ctx.init_learned_ref(net, dev(G), dev(Wref), Ht_cold=dev(Hcold))
    Wg2, Hg2 = (t.cpu().numpy().astype(np.float64) for t in ctx.factors())
    assert np.array_equal(Wg2, Wref.astype(np.float32).astype(np.float64))
    assert np.array_equal(np.all(Hg2 == Hcold, axis=1)[clear], rej[clear])
    assert abs(nrej2 - rej.sum()) <= np.sum(~clear)
    assert np.max((np.abs(Hg2 - Hsel) / scale)[clear]) <= 1e-4
    # a second warm start on the same compression, and one after set_state (the
    # alignment products then start from the context's stream): the same rows
    ctx.init_learned_ref(net, dev(G), dev(Wref), Ht_cold=dev(Hcold))
    Hg3 = ctx.factors()[1].cpu().numpy().astype(np.float64)
    assert np.array_equal(Hg3, Hg2)
    other = lib.NMF(m, n, r, kp, q, seed=7)
    other.set_state(*ctx.state())
    other.init_learned_ref(net, dev(G), dev(Wref), Ht_cold=dev(Hcold))
    Hg4 = other.factors()[1].cpu().numpy().astype(np.float64)
    assert np.array_equal(Hg4, Hg2)
    with pytest.raises(ValueError):
        ctx.init_learned_ref(net, dev(G)[:, :kp - 1].contiguous(), dev(Wref))   # wrong shape (binding)
    fresh = lib.NMF(m, n, r, kp, q, seed=7)
    with pytest.raises(lib.NmfError):
        fresh.init_learned_ref(net, dev(G), dev(Wref))                         # not compressed (library)


def test_init_learned_rejects_bad_arguments(lib):
    m, n, r, kp = 64, 32, 4, 8
    X = datagen.planted_c1(m, n, r, 3)[0]
    ctx = lib.NMF(m, n, r, kp, 1, seed=1)
    net = lib.Mlp(kp, 16, r, dev(datagen.mlp_he_init(kp, 16, r, 1)), max_batch=16)
    Wh = torch.zeros(kp, r, device="cuda")
    with pytest.raises(lib.NmfError):
        ctx.init_learned(net, Wh)                           # not compressed yet
    ctx.compress(dev(X))
    other = lib.Mlp(kp, 16, r + 1, dev(datagen.mlp_he_init(kp, 16, r + 1, 1)), max_batch=16)
    with pytest.raises(lib.NmfError):
        ctx.init_learned(other, Wh)                         # wrong output width
    assert ctx.init_learned(net, Wh) >= 0
