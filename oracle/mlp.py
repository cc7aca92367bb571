"""FP64 oracle of the learned warm start for H (test infrastructure only).

The paper has no learned component; this is the project extension that maps a
compressed column x-hat_j (a row of Xh = X^T Q_L, length k') to an initial
column h_j of H (a row of Ht, length r).  Definitions used on both sides:

  net:      z1 = x W1 + b1, a1 = relu(z1)            (k'  -> 512)
            z2 = a1 W2 + b2, a2 = relu(z2)           (512 -> 512)
            z3 = a2 W3 + b3, y = softplus(z3)        (512 -> r)
            weights stored [fan_in][fan_out], row-major.
  scaling:  the net sees x / ||x||_2 and its output is multiplied by ||x||_2
            (H is positively homogeneous in X); a zero row maps to h = 0.
  loss:     L = 1/(2B) sum_b || y_b - t_b / ||x_b|| ||^2 over a batch of B pairs.
  Adam:     m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
            p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps),
            b1 = 0.9, b2 = 0.999, eps = 1e-8 (Kingma & Ba, ICLR 2015).
  init:     He normal, W ~ N(0, 2 / fan_in), b = 0.
  selection: keep the net's h for column j iff
            ||x-hat_j - Wh_ref h_net||^2 <= ||x-hat_j - Wh_ref h_cold||^2.
"""
import numpy as np

LAYER_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(k_in, hidden, r_out):
    return [(k_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, r_out), (r_out,)]


def n_params(k_in, hidden, r_out):
    return sum(int(np.prod(s)) for s in shapes(k_in, hidden, r_out))


def unflatten(flat, k_in, hidden, r_out):
    out, off = [], 0
    for s in shapes(k_in, hidden, r_out):
        cnt = int(np.prod(s))
        out.append(np.asarray(flat[off:off + cnt], dtype=np.float64).reshape(s))
        off += cnt
    return out


def flatten(params):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in params])


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def scale_rows(X):
    nrm = np.sqrt(np.sum(np.asarray(X, dtype=np.float64) ** 2, axis=1))
    inv = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1.0), 0.0)
    return nrm, inv


def forward(params, X):
    """Net on already-scaled inputs; returns (y, cache)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1 + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2 + b2
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ W3 + b3
    return softplus(z3), (X, z1, a1, z2, a2, z3)


def infer(params, Xin):
    """h = ||x|| * net(x / ||x||) for every row of Xin."""
    nrm, inv = scale_rows(Xin)
    y, _ = forward(params, np.asarray(Xin, dtype=np.float64) * inv[:, None])
    return y * nrm[:, None]


def loss_grad(params, Xin, T):
    """Loss L and gradients (same order as params) on one batch of raw rows."""
    W1, b1, W2, b2, W3, b3 = params
    B = Xin.shape[0]
    _, inv = scale_rows(Xin)
    Xs = np.asarray(Xin, dtype=np.float64) * inv[:, None]
    Ts = np.asarray(T, dtype=np.float64) * inv[:, None]
    y, (X, z1, a1, z2, a2, z3) = forward(params, Xs)
    d = y - Ts
    L = 0.5 * np.sum(d * d) / B
    dz3 = (d / B) * sigmoid(z3)
    gW3 = a2.T @ dz3
    gb3 = dz3.sum(axis=0)
    dz2 = (dz3 @ W3.T) * (z2 > 0)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (z1 > 0)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    return L, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new params, m, v."""
    P, M, V = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mhat = mm / (1 - b1 ** t)
        vhat = vv / (1 - b2 ** t)
        P.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        M.append(mm)
        V.append(vv)
    return P, M, V


def select_warm(Xh_rows, Wh_ref, H_net, H_cold):
    """Per-row choice between the net's and the cold initial H rows.
    Returns (H_init, rejected mask)."""
    Xh_rows = np.asarray(Xh_rows, dtype=np.float64)
    rho_net = np.sum((Xh_rows - np.asarray(H_net, np.float64) @ Wh_ref.T) ** 2, axis=1)
    rho_cold = np.sum((Xh_rows - np.asarray(H_cold, np.float64) @ Wh_ref.T) ** 2, axis=1)
    reject = rho_net > rho_cold
    return np.where(reject[:, None], H_cold, H_net), reject
