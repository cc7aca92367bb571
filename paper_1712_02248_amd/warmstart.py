"""Learned warm start of H: pair generation and the warm initialisation of a
new compressed problem, as sequences of library calls (every arithmetic step
runs in the library's kernels).

Protocol: a reference fit on data of one generator gives a basis Q_train
(m x k', its left sketch basis) and the dictionary W_ref (m x r).  Training
pairs are compressed columns x-hat = Q_train^T x of new columns x and their
non-negative least-squares rows h* against Wh* = Q_train^T W_ref.  A new
problem whose columns come from the same generator (same dictionary, new
coefficients) is compressed with its own Q_L; W starts from W_ref, and H from
the net on the compressed columns mapped into the training basis,
x-tilde = (Q_train^T Q_L) x-hat, each net row being checked against the cold
row on ||x-hat - (Q_L^T W_ref) h||^2.
"""
import torch

from . import nmfrp


def _pad_cols(A, mult=4):
    c = A.shape[1]
    cp = -(-c // mult) * mult
    if cp == c and A.is_contiguous():
        return A
    out = torch.zeros(A.shape[0], cp, dtype=A.dtype, device=A.device)
    out[:, :c] = A
    return out


def compressed_factor(Q, W):
    """Q^T W (k' x r) on the library GEMM (contraction over the m rows)."""
    r = W.shape[1]
    return nmfrp.gemm(Q, _pad_cols(W), a_trans=True)[:, :r].contiguous()


def make_pairs(Q_train, Wh_ref, X_cols, sweeps=100):
    """Pairs for the columns of X_cols (m x c): inputs X_cols^T Q_train (c x k')
    and targets argmin_{h >= 0} ||x-hat - Wh_ref h|| (c x r)."""
    Xin = nmfrp.gemm(X_cols, Q_train, a_trans=True)
    T = nmfrp.nnls_rows(Xin, Wh_ref, sweeps)
    return Xin, T


def warm_init(ctx, net, Q_train, W_ref, Ht_cold=None, W0=None, init_scale=1.0, refine_sweeps=0, count=False):
    """Warm initialisation of a compressed context from a trained net: W = W0
    (default: the dictionary W_ref), H from the net with per-row rejection to
    Ht_cold, then refine_sweeps column-NNLS sweeps against Q_L^T W_ref.
    Returns the number of cold rows kept (None unless count)."""
    if W0 is None:   # the alignment products are formed inside the library
        return ctx.init_learned_ref(net, Q_train, W_ref, Ht_cold=Ht_cold, init_scale=init_scale,
                                    refine_sweeps=refine_sweeps, count=count)
    QL = ctx.left_basis()
    M = nmfrp.gemm(Q_train, QL, a_trans=True)           # Q_train^T Q_L, k' x k'
    Wh_ref = compressed_factor(QL, W_ref)                # Q_L^T W_ref, k' x r
    return ctx.init_learned(net, Wh_ref, align_M=M, W0=W_ref if W0 is None else W0, Ht_cold=Ht_cold,
                            init_scale=init_scale, refine_sweeps=refine_sweeps, count=count)
