"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module draws random inputs only; it holds none of the method's arithmetic.
Every array is produced once on the host with NumPy's PCG64 and handed
byte-identically to both sides (as FP32).

Workloads (X is m x n, rows are datapoints):
  c1   512 x 256:      W0, H0 ~ U[0,1) (rank 10); X = W0 H0 + 0.01 |N(0,1)|.
  c2   65536 x 4096:   sparse parts, W0_ij ~ Bernoulli(0.2) U[0,1), H0 ~ U[0,1)
                       (rank 32); X = max(0, W0 H0 + 0.01 N(0,1)).
  c3   100000 x 20000: topic-model counts, theta_i ~ Dir(0.1), Zipf(1.1) word
                       distributions per topic, X_iw ~ Poisson(200 (theta_i Phi)_w).
  c5   262144 x 16384: the c2 family with rank 128, its factors rounded to
                       multiples of 2^-8 (W0 = Bernoulli(0.2) floor(256 U) / 256,
                       H0 = floor(256 U) / 256), so that W0 H0 is exact in FP32
                       in any summation order; the noise is N(0,1) from
                       Philox4x32-10 (stream 2, key = the workload seed, element
                       (i, j) at flat index i n + j), and
                       X = max(0, fl32(W0 H0 + fl32(0.01 z))) in FP32.  Either
                       side forms X from these numbers (the device in HBM, the
                       oracle in host row panels).
  P1   400 x 4096:     stand-in for the paper's dense image data: the c2 family
                       with 40 parts, rescaled to [0, 1] and quantised to 256 levels.
  P2   5000 x 1000:    stand-in for the paper's sparse word counts: the c3 family
                       with 20 topics.
Initial factors: W, Ht ~ U[0,1) * c with c = 2 sqrt(mean(X) / r), so that
E[W Ht^T] = mean(X).
"""
import numpy as np

BASE_SEED = 1712022480

CONFIGS = {
    "c1": dict(idx=0, m=512, n=256, r=10, kp=20, q=2, iters=200, family="c1", r_true=10, prec="fp32"),
    "c2": dict(idx=1, m=65536, n=4096, r=32, kp=64, q=2, iters=500, family="parts", r_true=32, prec="fp32"),
    "c3": dict(idx=2, m=100000, n=20000, r=64, kp=128, q=2, iters=150, family="lda", r_true=64, prec="bf16"),
    "c5": dict(idx=4, m=262144, n=16384, r=128, kp=256, q=1, iters=300, family="dyadic_parts", r_true=128,
               prec="fp8"),
    "P1": dict(idx=10, m=400, n=4096, r=20, kp=25, q=4, iters=500, family="parts_q256", r_true=40, prec="fp32"),
    "P2": dict(idx=11, m=5000, n=1000, r=60, kp=72, q=9, iters=150, family="lda", r_true=20, prec="fp32"),
}

# sub-stream ids
S_W0, S_H0, S_NOISE, S_OMEGA_L, S_OMEGA_R, S_WINIT, S_HINIT, S_MLP, S_BATCH, S_FRESH = range(10)


def rng(seed, sub):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(sub)])))


def cfg_seed(name):
    return BASE_SEED + CONFIGS[name]["idx"]


def planted_c1(m, n, r, seed, noise=0.01):
    W0 = rng(seed, S_W0).random((m, r))
    H0 = rng(seed, S_H0).random((r, n))
    X = W0 @ H0 + noise * np.abs(rng(seed, S_NOISE).standard_normal((m, n)))
    return X.astype(np.float32), W0, H0


def parts_w0(m, r, seed, density=0.2):
    """Basis of the parts family: W0_ij ~ Bernoulli(density) U[0,1)."""
    g = rng(seed, S_W0)
    return (g.random((m, r)) < density) * g.random((m, r))


def planted_parts(m, n, r, seed, noise=0.01, density=0.2, block=8192):
    W0 = parts_w0(m, r, seed, density)
    H0 = rng(seed, S_H0).random((r, n))
    X = np.empty((m, n), dtype=np.float32)
    gn = rng(seed, S_NOISE)
    for i in range(0, m, block):
        blk = W0[i:i + block] @ H0
        blk += noise * gn.standard_normal(blk.shape, dtype=np.float32)
        np.maximum(blk, 0.0, out=blk)
        X[i:i + block] = blk
    return X, W0, H0


def dyadic_parts_factors(m, n, r, seed, density=0.2):
    """Factors of the dyadic parts family (c5): W0 = Bernoulli(density) U8 and
    H0 = U8, U8 = floor(256 U[0,1)) / 256, as FP32 (exact).  Every product of
    two entries is a multiple of 2^-16 below 1, so the r-term sums of W0 H0 are
    exact in FP32 (24-bit significand) for r <= 128, in any order."""
    g = rng(seed, S_W0)
    W0 = (g.random((m, r)) < density) * np.floor(256.0 * g.random((m, r))) / 256.0
    H0 = np.floor(256.0 * rng(seed, S_H0).random((r, n))) / 256.0
    return W0.astype(np.float32), H0.astype(np.float32)


DYADIC_NOISE = np.float32(0.01)   # noise scale of the dyadic parts family
DYADIC_NOISE_STREAM = S_NOISE     # Philox stream of its noise


def planted_parts_q256(m, n, r, seed):
    X, W0, H0 = planted_parts(m, n, r, seed)
    X = np.round(255.0 * X / X.max()) / 255.0
    return X.astype(np.float32), W0, H0


def topic_counts(m, n, r, seed, alpha=0.1, zipf=1.1, tokens=200.0, block=4096):
    g = rng(seed, S_W0)
    theta = g.dirichlet(alpha * np.ones(r), size=m)          # m x r
    gp = rng(seed, S_H0)
    Phi = np.empty((r, n))
    for t in range(r):
        ranks = gp.permutation(n) + 1.0
        p = ranks ** (-zipf)
        Phi[t] = p / p.sum()
    X = np.empty((m, n), dtype=np.float32)
    gn = rng(seed, S_NOISE)
    for i in range(0, m, block):
        lam = tokens * (theta[i:i + block] @ Phi)
        X[i:i + block] = gn.poisson(lam).astype(np.float32)
    return X, theta, Phi


def make_x(name, m=None, n=None, r_true=None, seed=None):
    """Data matrix of workload `name` (FP32, C order).  Sizes may be overridden
    to draw a smaller instance of the same family."""
    c = CONFIGS[name]
    m = c["m"] if m is None else m
    n = c["n"] if n is None else n
    r_true = c["r_true"] if r_true is None else r_true
    seed = cfg_seed(name) if seed is None else seed
    fam = c["family"]
    if fam == "c1":
        return planted_c1(m, n, r_true, seed)[0]
    if fam == "parts":
        return planted_parts(m, n, r_true, seed)[0]
    if fam == "dyadic_parts":
        raise ValueError("the dyadic parts family (c5) is formed in row panels by its consumer, "
                         "from dyadic_parts_factors and Philox noise")
    if fam == "parts_q256":
        return planted_parts_q256(m, n, r_true, seed)[0]
    if fam == "lda":
        return topic_counts(m, n, r_true, seed)[0]
    raise ValueError(fam)


def init_factors(X_mean, m, n, r, seed):
    """Initial W (m x r) and Ht (n x r), U[0,1) * 2 sqrt(mean(X)/r), FP32."""
    c = 2.0 * np.sqrt(max(float(X_mean), 1e-30) / r)
    W = (rng(seed, S_WINIT).random((m, r)) * c).astype(np.float32)
    Ht = (rng(seed, S_HINIT).random((n, r)) * c).astype(np.float32)
    return W, Ht


def gaussian(rows, cols, seed, sub):
    """N(0,1) test matrix drawn on the host (FP32)."""
    return rng(seed, sub).standard_normal((rows, cols), dtype=np.float32)


def uniform(shape, seed, sub):
    return rng(seed, sub).random(shape).astype(np.float32)


# ---------------------------------------------------------------- warm start

def fresh_h(r, ncols, seed, chunk):
    """Fresh coefficient columns U[0,1) (r x ncols) for chunk `chunk` of new
    columns of a planted family (same W0, new H0)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), S_FRESH, int(chunk)])))
    return g.random((r, ncols))


def fresh_parts_columns(W0, ncols, seed, chunk, noise=0.01):
    """New columns of the parts family on the host: max(0, W0 h + noise N(0,1)),
    returned as an m x ncols FP32 block (small instances only)."""
    H = fresh_h(W0.shape[1], ncols, seed, chunk)
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), S_FRESH, int(chunk), 1])))
    X = W0 @ H + noise * g.standard_normal((W0.shape[0], ncols))
    return np.maximum(X, 0.0).astype(np.float32)


def mlp_he_init(k_in, hidden, r_out, seed):
    """He-normal initial weights N(0, 2 / fan_in) and zero biases, flat FP32 in
    the order W1 (k_in x hidden), b1, W2, b2, W3 (hidden x r_out), b3."""
    g = rng(seed, S_MLP)
    parts = []
    for fi, fo in ((k_in, hidden), (hidden, hidden), (hidden, r_out)):
        parts.append((g.standard_normal((fi, fo)) * np.sqrt(2.0 / fi)).ravel())
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32)


def batch_orders(npairs, epochs, seed):
    """One random permutation of the training pairs per pass (epochs x npairs, int32)."""
    g = rng(seed, S_BATCH)
    return np.stack([g.permutation(npairs) for _ in range(epochs)]).astype(np.int32)
