"""Writes oracle_errors.json: FP64 oracle relative errors of FastHALS-RP on the
seeded synthetic workloads, with the test matrices drawn by the oracle's own
Philox4x32-10 (streams 3 and 4, key = workload seed), i.e. the same numbers the
device draws when no Omega is passed.  Calls only oracle/ and datagen/.

usage: python tests/golden/make_oracle_errors.py [c1 c2 ... | c5:fp8:2:2 ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402
from oracle import inputs, nmf, philox  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_errors.json")
CHECKPOINTS = (1, 2, 5, 10, 20, 50, 100, 150, 200, 300, 400, 500)


def run_lowp(name, fmt, refine, lps):
    """The oracle's model of the low-precision compression (compress_lowp: the
    quantised X and thin operands in the range finder, the refinement and the
    projected data as configured), then FastHALS-RP from the same cold factors:
    the reference the GPU's low-precision path is checked against (R_q)."""
    c = datagen.CONFIGS[name]
    m, n, r, kp, q, iters = c["m"], c["n"], c["r"], c["kp"], c["q"], c["iters"]
    seed = datagen.cfg_seed(name)
    t0 = time.perf_counter()
    if c["family"] == "dyadic_parts":
        X32 = inputs.dyadic_parts_rows(name)
        mean = float(np.sum(X32, dtype=np.float64)) / (m * n)
    else:
        X32 = datagen.make_x(name)
        mean = X32.mean()
    X = nmf.RowPanels(X32)
    W0, H0 = datagen.init_factors(mean, m, n, r, seed)
    OL = philox.normal(n, kp, 3, seed).astype(np.float32)
    OR = philox.normal(m, kp, 4, seed).astype(np.float32)
    t1 = time.perf_counter()
    QL, QR, Xh, Xc = nmf.compress_lowp(X, OL, OR, q, fmt, refine=refine, lowp_sketches=lps)
    t2 = time.perf_counter()
    print(name, fmt, "compressed", t2 - t1, flush=True)
    W, Ht = W0.astype(np.float64), H0.astype(np.float64)
    curve = {0: nmf.rel_error(X, W, Ht)}
    for it in range(1, iters + 1):
        W, Ht = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR)
        if it in CHECKPOINTS or it == iters:
            curve[it] = nmf.rel_error(X, W, Ht)
            print(f"{name} {fmt} it={it} e={curve[it]:.10e}", flush=True)
    return dict(m=m, n=n, r=r, kp=kp, q=q, iters=iters, seed=seed, omega="philox streams 3/4", fmt=fmt,
                refine=refine, lowp_sketches=lps, e=curve[iters], curve={str(k): v for k, v in curve.items()},
                oracle_seconds=dict(data=t1 - t0, compress=t2 - t1))


def run(name):
    c = datagen.CONFIGS[name]
    m, n, r, kp, q, iters = c["m"], c["n"], c["r"], c["kp"], c["q"], c["iters"]
    seed = datagen.cfg_seed(name)
    t0 = time.perf_counter()
    big = c["family"] == "dyadic_parts"
    if big:   # too large for FP64 in memory: FP32 X, products over FP64 row panels
        X32 = inputs.dyadic_parts_rows(name)
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
    """Names: a workload (c1, c2, c3, c5), or workload:fmt:refine:lowp_sketches for
    the low-precision model (e.g. c5:fp8:2:2)."""
    for name in names:
        if ":" in name:
            w, fmt, refine, lps = name.split(":")
            key = f"{w}_{fmt}_refine{refine}_lps{lps}"
            res = run_lowp(w, fmt, int(refine), int(lps))
        else:
            key, res = name, run(name)
        out = json.load(open(OUT)) if os.path.exists(OUT) else {}
        out[key] = res
        json.dump(out, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2"])
