"""Device-side synthesis of the inputs too large to draw on the host: the
dyadic parts family (262144 x 16384) and new columns of the parts families,
formed in HBM from the same numbers as the host recipe in this package.

Input synthesis only (none of the method's arithmetic): the factors come from
dyadic_parts_factors / fresh_h on the host, the N(0,1) noise from a Philox
generator passed in as `gaussian(rows, cols, stream, seed) -> device tensor`
(the element layout of the host oracle's Philox), products and elementwise
steps from torch.  Each elementwise step is its own FP32 operation, in the order
of the host recipe: fl32(0.01 z), then fl32(W0 H0 + that), then max(0, .)."""
import numpy as np

from . import (CONFIGS, DYADIC_NOISE, DYADIC_NOISE_STREAM, cfg_seed, dyadic_parts_factors, fresh_h)


def dyadic_parts_x(torch, gaussian, name="c5", block=16384, device="cuda"):
    """X (m x n FP32, device) of the dyadic parts family of workload `name`, and
    the basis W0 (device) and the FP64 mean of X.  The noise buffer becomes X in
    place, one block of rows at a time (peak memory: X plus one block)."""
    c = CONFIGS[name]
    m, n, r = c["m"], c["n"], c["r_true"]
    seed = cfg_seed(name)
    W0, H0 = dyadic_parts_factors(m, n, r, seed)
    W0d = torch.from_numpy(W0).to(device)
    H0d = torch.from_numpy(H0).to(device)
    X = gaussian(m, n, DYADIC_NOISE_STREAM, seed)
    total = torch.zeros((), dtype=torch.float64, device=device)
    for i in range(0, m, block):
        Z = X[i:i + block]
        Z.mul_(float(DYADIC_NOISE))
        Z.add_(W0d[i:i + block] @ H0d)
        Z.clamp_min_(0.0)
        total += Z.sum(dtype=torch.float64)
    return X, W0d, float(total) / (m * n)


def dyadic_fresh_columns(torch, gaussian, W0d, ncols, seed, chunk):
    """New columns of the dyadic parts family (same basis W0, new coefficients
    floor(256 U) / 256 from chunk `chunk`'s stream, noise from Philox stream
    1000 + chunk): an m x ncols FP32 device block."""
    r = W0d.shape[1]
    H = (np.floor(256.0 * fresh_h(r, ncols, seed, chunk)) / 256.0).astype(np.float32)
    Z = gaussian(W0d.shape[0], ncols, 1000 + chunk, seed)
    Z.mul_(float(DYADIC_NOISE))
    Z.add_(W0d @ torch.from_numpy(H).to(W0d.device))
    return Z.clamp_min_(0.0)


def parts_fresh_columns(torch, gaussian, W0d, ncols, seed, chunk, noise=0.01):
    """New columns of the parts family (same basis W0, U[0,1) coefficients from
    chunk `chunk`'s stream, noise from Philox stream 1000 + chunk):
    max(0, W0 h + noise z), an m x ncols FP32 device block."""
    H = torch.from_numpy(fresh_h(W0d.shape[1], ncols, seed, chunk).astype(np.float32)).to(W0d.device)
    N = gaussian(W0d.shape[0], ncols, 1000 + chunk, seed)
    return torch.clamp_min(W0d @ H + noise * N, 0.0)
