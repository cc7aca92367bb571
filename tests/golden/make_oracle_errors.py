"""Writes oracle_errors.json: FP64 oracle relative errors of FastHALS-RP on the
seeded synthetic workloads, with the test matrices drawn by the oracle's own
Philox4x32-10 (streams 3 and 4, key = workload seed), i.e. the same numbers the
device draws when no Omega is passed.  Calls only oracle/ and datagen/.

usage: python tests/golden/make_oracle_errors.py [c1 c2 ...]
"""
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


def run(name):
    c = datagen.CONFIGS[name]
    m, n, r, kp, q, iters = c["m"], c["n"], c["r"], c["kp"], c["q"], c["iters"]
    seed = datagen.cfg_seed(name)
    t0 = time.perf_counter()
    X = datagen.make_x(name)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
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
    res = dict(m=m, n=n, r=r, kp=kp, q=q, iters=iters, seed=seed, omega="philox streams 3/4",
               e=curve[iters], curve={str(k): v for k, v in curve.items()},
               oracle_seconds=dict(data=t1 - t0, compress=t2 - t1, per_iteration=t_iter / iters),
               normX2=float(np.sum(X.astype(np.float64) ** 2)))
    print(name, json.dumps(res["curve"]), res["oracle_seconds"], flush=True)
    return res


def main(names):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        out[name] = run(name)
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
