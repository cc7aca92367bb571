"""What the trained network adds to the warm start (GPU).

The warm start has three parts: W = W_ref (the reference fit's dictionary), H from
the network with per-row rejection, and NNLS sweeps.  The control keeps W_ref and
the sweeps and drops the network (cold rows of H).  On a parts problem drawn
from the generator the network was trained on (same dictionary, new
coefficients), the network's rows must give a lower error than the cold rows
after the same small number of sweeps, and reach eps in fewer FastHALS-RP
iterations.  With enough sweeps both reach the rows' NNLS solution (at r = 16
twenty sweeps from cold rows do), and the network can only tie; at r = 128
(the 262144 x 16384 workload) twenty sweeps do not converge and the network
halves the iterations to eps there (measured in the benchmark)."""
import numpy as np
import pytest
import torch

import datagen
from datagen import device as ddev

pytestmark = pytest.mark.gpu

M, N, R, KP, Q = 16384, 2048, 16, 32, 2
SEED = 4242


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1712_02248_amd import nmfrp, warmstart
    nmfrp.load()
    W0gen = torch.from_numpy(datagen.parts_w0(M, R, SEED).astype(np.float32)).cuda()
    fresh = lambda ncols, chunk: ddev.parts_fresh_columns(torch, nmfrp.gaussian, W0gen, ncols, SEED, chunk)
    # reference fit on one draw of the generator
    Xt = fresh(N, 50)
    ctx = nmfrp.NMF(M, N, R, KP, Q, seed=SEED + 1)
    Wi, Hi = datagen.init_factors(float(Xt.mean()), M, N, R, SEED + 1)
    ctx.compress(Xt)
    ctx.init(torch.from_numpy(Wi).cuda(), torch.from_numpy(Hi).cuda())
    ctx.step(300)
    Q_train = ctx.left_basis()
    W_ref, _ = ctx.factors()
    Wh_star = warmstart.compressed_factor(Q_train, W_ref)
    ctx.close()
    # training pairs from new columns, held-out pairs, Adam training
    Xin, T = [], []
    for c in range(8):
        a, b = warmstart.make_pairs(Q_train, Wh_star, fresh(4096, 51 + c), sweeps=100)
        Xin.append(a)
        T.append(b)
    Xin, T = torch.cat(Xin), torch.cat(T)
    p0 = torch.from_numpy(datagen.mlp_he_init(KP, 512, R, SEED)).cuda()
    net = nmfrp.Mlp(KP, 512, R, p0, max_batch=4096)
    order = torch.from_numpy(datagen.batch_orders(Xin.shape[0], 20, SEED).reshape(-1)).cuda()
    losses = net.train(Xin, T, 20, 1024, 1e-3, order=order)
    print(f"warm gain: training loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    # the new problem and its cold factors
    X = fresh(N, 0)
    W0, H0 = datagen.init_factors(float(X.mean()), M, N, R, SEED)
    W0d, H0d = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
    c0 = nmfrp.NMF(M, N, R, KP, Q, seed=SEED)
    c0.compress(X)
    c0.init(W0d, H0d)
    c0.step(300)
    eps = (1.0 + 1e-3) * c0.residual(X)
    c0.close()
    yield nmfrp, warmstart, net, Q_train, W_ref, X, H0d, eps
    del X, Xin, T


def _ctx(nmfrp, X):
    ctx = nmfrp.NMF(M, N, R, KP, Q, seed=SEED)
    ctx.compress(X)
    return ctx


def test_network_rows_beat_cold_rows_after_equal_sweeps(setup):
    nmfrp, warmstart, net, Q_train, W_ref, X, H0d, _ = setup
    for sweeps in (0, 5, 20):
        cn = _ctx(nmfrp, X)
        rej = warmstart.warm_init(cn, net, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps, count=True)
        e_net = cn.residual(X)
        cn.close()
        cc = _ctx(nmfrp, X)
        cc.init_learned_ref(None, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps)
        e_ctrl = cc.residual(X)
        cc.close()
        print(f"  {sweeps:2d} sweeps: e(network) {e_net:.6e} (rejected rows {rej}), e(cold rows) {e_ctrl:.6e}",
              flush=True)
        if sweeps < 20:
            assert e_net < 0.9 * e_ctrl, sweeps
        else:           # both at the NNLS rows (up to the sweeps' own convergence)
            assert e_net <= e_ctrl * (1 + 1e-5), sweeps


@pytest.mark.parametrize("sweeps", [0, 5, 20])
def test_network_reaches_eps_in_fewer_iterations(setup, sweeps):
    nmfrp, warmstart, net, Q_train, W_ref, X, H0d, eps = setup
    cn = _ctx(nmfrp, X)
    warmstart.warm_init(cn, net, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps)
    it_net, e_net = cn.fit(X, 300, eps, check_every=1)
    cn.close()
    cc = _ctx(nmfrp, X)
    cc.init_learned_ref(None, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps)
    it_ctrl, e_ctrl = cc.fit(X, 300, eps, check_every=1)
    cc.close()
    print(f"  {sweeps:2d} sweeps, to eps {eps:.6e}: network {it_net} iterations (e {e_net:.6e}), "
          f"control {it_ctrl} iterations (e {e_ctrl:.6e})", flush=True)
    assert e_net <= eps and e_ctrl <= eps
    if sweeps < 20:
        assert it_net < it_ctrl
    else:
        assert it_net <= it_ctrl
