"""Writes oracle_errors.json: FP64 oracle relative errors of FastHALS-RP on the
seeded synthetic workloads, with the test matrices drawn by the oracle's own
Philox4x32-10 (streams 3 and 4, key = workload seed), i.e. the same numbers the
device draws when no Omega is passed.  Calls only oracle/ and datagen/.

usage: python tests/golden/make_oracle_errors.py [c1 c2 ...]
"""
import concurrent.futures
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
from oracle import nmf, philox  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_errors.json")
CHECKPOINTS = (1, 2, 5, 10, 20, 50, 100, 150, 200, 300, 400, 500)


def dyadic_parts_x(name, panel=4096, threads=8):
    """X of the dyadic parts family (FP32, host): per row panel
    max(0, fl32(W0 H0 + fl32(0.01 z))), z from the oracle's Philox (stream 2,
    flat index i n + j), the product exact in FP32 by construction."""
    c = datagen.CONFIGS[name]
    m, n = c["m"], c["n"]
    seed = datagen.cfg_seed(name)
    W0, H0 = datagen.dyadic_parts_factors(m, n, c["r_true"], seed)
    X = np.empty((m, n), dtype=np.float32)

    def fill(i):
        rows = min(panel, m - i)
        z = philox.normal(rows, n, datagen.DYADIC_NOISE_STREAM, seed, row0=i).astype(np.float32)
        z *= datagen.DYADIC_NOISE
        z += W0[i:i + rows] @ H0
        np.maximum(z, np.float32(0.0), out=z)
        X[i:i + rows] = z

    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(0, m, panel)))
    return X


def run(name):
    c = datagen.CONFIGS[name]
    m, n, r, kp, q, iters = c["m"], c["n"], c["r"], c["kp"], c["q"], c["iters"]
    seed = datagen.cfg_seed(name)
    t0 = time.perf_counter()
    big = c["family"] == "dyadic_parts"
    if big:   # too large for FP64 in memory: FP32 X, products over FP64 row panels
        X32 = dyadic_parts_x(name)
        mean = float(np.sum(X32, dtype=np.float64)) / (m * n)
        X = nmf.RowPanels(X32)
        print(name, "X formed", time.perf_counter() - t0, flush=True)
    else:
        X = datagen.make_x(name)
        mean = X.mean()
    W0, H0 = datagen.init_factors(mean, m, n, r, seed)
    OL = philox.normal(n, kp, 3, seed).astype(np.float32)
    OR = philox.normal(m, kp, 4, seed).astype(np.float32)
    t1 = time.perf_counter()
    QL, QR, Xh, Xc = nmf.compress(X, OL, OR, q)
    t2 = time.perf_counter()
    W, Ht = W0.astype(np.float64), H0.astype(np.float64)
    curve = {0: nmf.rel_error(X, W, Ht)}
    t_iter = 0.0
    for it in range(1, iters + 1):
        ta = time.perf_counter()
        W, Ht = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR)
        t_iter += time.perf_counter() - ta
        if it in CHECKPOINTS or it == iters:
            curve[it] = nmf.rel_error(X, W, Ht)
            if big:
                print(f"{name} it={it} e={curve[it]:.10e} ({t_iter / it:.2f} s per iteration)", flush=True)
    res = dict(m=m, n=n, r=r, kp=kp, q=q, iters=iters, seed=seed, omega="philox streams 3/4",
               e=curve[iters], curve={str(k): v for k, v in curve.items()},
               oracle_seconds=dict(data=t1 - t0, compress=t2 - t1, per_iteration=t_iter / iters),
               normX2=nmf.frob_sq_diff(X, W[:, :0], Ht[:, :0])[1])
    if big:
        res.update(x_mean=mean, family="dyadic parts: X = max(0, fl32(W0 H0 + fl32(0.01 z))), z Philox stream 2")
    print(name, json.dumps(res["curve"]), res["oracle_seconds"], flush=True)
    return res


def main(names):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        out[name] = run(name)
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
