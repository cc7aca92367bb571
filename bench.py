#!/usr/bin/env python3
"""Time-to-relative-error for compressed NMF (FastHALS-RP) on one MI355X:
low-precision compression with a learned warm start of H, against plain FP32.

One step = the whole hot path on the workload's X, which is resident in HBM
when the clock starts: compress (device-drawn Gaussian test matrices, range
finder with power iterations and FP64 CholeskyQR2, sketch products), set the
initial factors, then FastHALS-RP iterations with an exact FP64 residual check
schedule until e <= eps.  eps = (1 + 1e-3) * e_oracle, where e_oracle is the FP64
oracle's error after the workload's iteration count (stored by
tests/golden/make_oracle_errors.py, which calls only the oracle).

Workloads (default c5):
  c5  X 262144 x 16384 (16 GiB, dyadic parts family formed on the device),
      r = 128, k' = 256, q = 1, 300 iterations.  Headline `fp8_warm`: e4m3
      range-finder products with 128 x 128 block scales, one refinement power
      iteration per side on X (split-BF16 products), split-BF16 sketch products,
      then the learned warm start: W from the reference dictionary, H rows from
      the network on the compressed columns, each kept only if it beats the cold
      row on the compressed residual, then column-NNLS sweeps; the iterations'
      products on split-BF16 MFMA (`fp8_warm_fp32_updates` keeps them FP32).
  c2  X 65536 x 4096 (parts family), r = 32, k' = 64, q = 2, 500 iterations.
      Headline `bf16_warm`: BF16 range finder, split-BF16 sketches, warm start.
  c3  X 100000 x 20000 Poisson document counts from 64 planted topics, r = 64,
      k' = 128, q = 2, 150 iterations: BF16 range finder (FP32 or split-BF16
      sketches) against plain FP32, both from the cold factors (new columns of a
      topic model are new words, which its generator does not define, so there
      is no warm start here).  The default c5 run appends this block as "c3".
Every workload also times plain FP32 FastHALS-RP from the cold factors (the
paper's method) and variants that separate what each part contributes: the
network replaced by the cold rows with the same dictionary and sweeps
(`*_ctrl_no_net`), the network with a cold W (`*_net_cold_w`), no sweeps
(`*_net_no_sweeps`), cold starts of each precision.
The network is trained before timing on pairs from new columns of the same
generator (same basis W0, new coefficients): a reference fit on one new draw
gives Q_train and W_ref; every pair is (Q_train^T x, NNLS row of x against
Q_train^T W_ref).  Training time is reported separately.

Prints one JSON line (rank 0).  --gpus above 1 is refused: the path is built
and measured on a single GPU.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_errors.json")
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP8_TFLOPS = 5000.0
PEAK_HBM_GBS = 8000.0
# the headline variant per workload: low-precision range finder, split-BF16
# sketches (and refinement), learned warm start
HEADLINE = {"c2": "bf16_warm", "c5": "fp8_warm"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--check-every", type=int, default=0, help="0: adaptive residual checks")
    ap.add_argument("--max-iters", type=int, default=0, help="0: the workload's iteration count")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0, help="rows of X in the oracle sample (0: per workload)")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations timed in the sample (0: per workload)")
    ap.add_argument("--pairs", type=int, default=200000, help="training pairs (rounded up to 4096)")
    ap.add_argument("--epochs", type=int, default=50, help="most training passes")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--nnls-sweeps", type=int, default=100)
    ap.add_argument("--refine-sweeps", type=int, default=20,
                    help="column-NNLS sweeps on the warm rows against the reference dictionary")
    ap.add_argument("--headline-only", action="store_true", help="time only plain and the headline variant")
    ap.add_argument("--variants", default="", help="comma list of variants to time (default: all)")
    ap.add_argument("--sweep", default="", help="parameter study instead of the bench: P1, P2 or c2 "
                    "(components r x power iterations q, FastHALS-RP against FastHALS, sketch spectrum)")
    ap.add_argument("--sweep-seeds", type=int, default=3, help="test-matrix seeds per sweep point (median)")
    ap.add_argument("--probe-kernels", action="store_true",
                    help="only a copy of known size and the dominant kernel (for counter runs); at c5 then "
                         "the FP8 range-finder products and iterations with FP32 and split-BF16 updates")
    ap.add_argument("--c4", action="store_true",
                    help="the warm-start study on new columns instead of the bench: the network trained "
                         "on the 65536 x 4096 parts workload's generator, applied to --c4-cols fresh columns, "
                         "then 20 iterations against the cold start and the controls")
    ap.add_argument("--c4-cols", type=int, default=50000)
    ap.add_argument("--no-c3", action="store_true", help="leave out the c3 block of the default c5 run")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads", 0) for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def cpu_baseline(cfg, X, W0, H0, iters_needed, rows, iters_sample):
    """The FP64 oracle on a row sample of X, scaled linearly to the full workload.
    X None: the rows are formed by the oracle's own generator (the dyadic parts
    family lives on the device only); that generation is not timed."""
    import datagen
    from oracle import inputs, nmf, philox
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    ms = min(rows, m)
    seed = datagen.cfg_seed(cfg["name"])
    Xs = X[:ms] if X is not None else inputs.dyadic_parts_rows(cfg["name"], 0, ms)
    OL = philox.normal(n, kp, 3, seed).astype(np.float32)
    OR = philox.normal(ms, kp, 4, seed).astype(np.float32)
    t0 = time.perf_counter()
    QL, QR, Xh, Xc = nmf.compress(Xs, OL, OR, q)
    t1 = time.perf_counter()
    W, Ht = W0[:ms].astype(np.float64), H0.astype(np.float64)
    nit = max(1, min(iters_needed, iters_sample))
    for _ in range(nit):
        W, Ht = nmf.fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR)
    t2 = time.perf_counter()
    t3 = time.perf_counter()
    nmf.rel_error(Xs, W, Ht)
    t4 = time.perf_counter()
    full = ((t1 - t0) * (m / ms) + (t2 - t1) / nit * iters_needed * (m + n) / (ms + n)
            + (t4 - t3) * (m / ms))
    sample = (f"FP64 oracle of the plain method (the oracle has no trained network): compress on rows "
              f"0..{ms - 1} of X ({ms}/{m}), {nit} FastHALS-RP iterations and one residual there; "
              f"scaled by rows and iterations to the {iters_needed} iterations the plain FP32 GPU path "
              f"needs to reach eps, one residual, no intermediate checks (measured {t4 - t0:.1f} s)")
    return dict(value=round(full, 3), unit="s", cores=blas_threads(), kind="oracle", sample=sample)


def marker_push(torch, name):
    """Names a range for a profiler's marker trace (no effect without one)."""
    try:
        torch.cuda.nvtx.range_push(name)
    except Exception:
        pass


def marker_pop(torch):
    try:
        torch.cuda.nvtx.range_pop()
    except Exception:
        pass


def train_warm_start(torch, nmfrp, cfg, seed, args, fresh):
    """Reference fit, pair generation and Adam training (all untimed).
    fresh(ncols, chunk): new columns of the workload's generator (device)."""
    import datagen
    from paper_1712_02248_amd import warmstart
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    info = {}
    t0 = time.perf_counter()
    # reference fit on one new draw of the generator (FP32 compression)
    Xt = fresh(n, 0)
    mean_t = float(Xt.sum(dtype=torch.float64)) / (m * n)
    ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed + 1)
    Wi, Hi = datagen.init_factors(mean_t, m, n, r, seed + 1)
    ctx.compress(Xt)
    ctx.init(torch.from_numpy(Wi).cuda(), torch.from_numpy(Hi).cuda())
    _, e_ref = ctx.fit(Xt, cfg["iters"], 0.0, cfg["iters"])
    Q_train = ctx.left_basis()
    W_ref, _ = ctx.factors()
    Wh_star = warmstart.compressed_factor(Q_train, W_ref)
    del Xt, ctx
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # pairs from new columns
    chunk = 4096
    nchunks = -(-args.pairs // chunk)
    npairs = nchunks * chunk
    Xin = torch.empty(npairs, kp, device="cuda")
    T = torch.empty(npairs, r, device="cuda")
    for c in range(nchunks):
        Xf = fresh(chunk, 1 + c)
        a, b = warmstart.make_pairs(Q_train, Wh_star, Xf, sweeps=args.nnls_sweeps)
        Xin[c * chunk:(c + 1) * chunk] = a
        T[c * chunk:(c + 1) * chunk] = b
        del Xf
    Xv = fresh(chunk, 1 + nchunks)
    Xin_v, T_v = warmstart.make_pairs(Q_train, Wh_star, Xv, sweeps=args.nnls_sweeps)
    del Xv
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # Adam training in rounds of 5 passes; the learning rate drops 3x when the
    # held-out loss improves by less than 1 % in a round, training stops after
    # the third drop or at the pass limit
    hidden = 512
    p0 = torch.from_numpy(datagen.mlp_he_init(kp, hidden, r, seed)).cuda()
    net = nmfrp.Mlp(kp, hidden, r, p0, max_batch=4096)
    order = torch.from_numpy(datagen.batch_orders(npairs, args.epochs, seed).reshape(-1)).cuda()
    hist, val = [], []
    best = float("inf")
    ep, lr, drops = 0, args.lr, 0
    while ep < args.epochs:
        e5 = min(5, args.epochs - ep)
        hist += net.train(Xin, T, e5, 1024, lr, order=order[ep * npairs:(ep + e5) * npairs])
        ep += e5
        v, _ = net.loss_grad(Xin_v, T_v)
        val.append(v)
        log(f"[bench] warm-start training: {ep} passes, lr {lr:.1e}, train loss {hist[-1]:.4e}, held-out {v:.4e}")
        if v > 0.99 * best:
            drops += 1
            if drops == 3:
                break
            lr /= 3.0
        best = min(best, v)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    info.update(reference_fit=dict(iters=cfg["iters"], rel_err=e_ref, seconds=round(t1 - t0, 3)),
                pairs=dict(count=npairs, held_out=chunk, nnls_sweeps=args.nnls_sweeps,
                           seconds=round(t2 - t1, 3)),
                training=dict(net=f"{kp}->{hidden}->{hidden}->{r}", passes=ep, batch=1024, lr=args.lr,
                              lr_final=lr,
                              loss_first=hist[0], loss_last=hist[-1], held_out_loss=val,
                              seconds=round(t3 - t2, 3)))
    return net, Q_train, W_ref, info


def warm_start(ctx, warm, W0d, H0d, count=False):
    """The initialisation of a warm variant.  warm = (net, Q_train, W_ref, sweeps,
    mode): mode "ref" sets W = W_ref and H from the network with rejection, then
    the sweeps; "no_net" the same without the network (cold rows, then the
    sweeps); "cold_w" H from the network with rejection and the sweeps, W from the
    cold draw."""
    from paper_1712_02248_amd import warmstart
    net, Q_train, W_ref, sweeps, mode = warm
    if mode == "no_net":
        return ctx.init_learned_ref(None, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps, count=count)
    if mode == "cold_w":
        return warmstart.warm_init(ctx, net, Q_train, W_ref, Ht_cold=H0d, W0=W0d, refine_sweeps=sweeps,
                                   count=count)
    return warmstart.warm_init(ctx, net, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps, count=count)


def time_variant(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, prec, refine, warm, steps, warmup,
                 label="", lps=0, up=0):
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    max_iters = args.max_iters or cfg["iters"]
    ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed, prec=prec, refine_fp32=refine, lowp_sketches=lps, update_prec=up)

    def start(count=False):
        ctx.compress(Xd)
        if warm is None:
            ctx.init(W0d, H0d)
            return None
        return warm_start(ctx, warm, W0d, H0d, count=count)

    def step():
        start()
        return ctx.fit(Xd, max_iters, eps, args.check_every)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times, its, es = [], [], []
    marker_push(torch, f"{label}: timed steps")
    for _ in range(steps):
        t0 = time.perf_counter()
        it, e = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(it)
        es.append(e)
    marker_pop(torch)
    # error right after the initialisation and after 20 iterations, then the
    # stage split (library events) of a repeat of the last step's work, ending
    # with the stopping test the fit runs (split-BF16 residual, exact near eps)
    nrej = start(count=True)
    e0 = ctx.residual(Xd)
    ctx.step(20)
    e20 = ctx.residual(Xd)
    start()
    ctx.step(its[-1])
    ctx.residual_check(Xd, eps)
    st = ctx.stage_times()
    e_fixed = ctx.residual(Xd)
    ctx.close()
    return dict(times=times, iters=its, e=es, e_init=e0, e_20=e20, e_fixed=e_fixed, stages=st, rejected=nrej)


def time_uncompressed(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, steps, warmup):
    """Textbook FastHALS (Sec 2.2) on X itself to eps, from the same cold factors:
    the paper's no-RP reference for the compressed update.  Chunks between exact
    residual checks follow the fit's rule (by the gap to eps, then 1.5x the
    straight-line extrapolation of the last two values, 5..50)."""
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    max_iters = args.max_iters or cfg["iters"]
    ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed)

    def step():
        ctx.init(W0d, H0d)
        done, e, prev = 0, None, None
        chunk = 50
        while done < max_iters:
            chunk = min(chunk, max_iters - done)
            ctx.fasthals_step(Xd, chunk)
            done += chunk
            e = ctx.residual(Xd)
            if e <= eps:
                break
            if prev is not None and prev[1] > e:
                slope = (prev[1] - e) / (done - prev[0])
                chunk = int(min(50, max(5, -(-1.5 * (e - eps) // slope))))
            else:
                gap = (e - eps) / eps
                chunk = 50 if gap > 0.1 else 20 if gap > 0.01 else 10 if gap > 0.003 else 5
            prev = (done, e)
        return done, e

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    times, its, es = [], [], []
    marker_push(torch, "fasthals_uncompressed: timed steps")
    for _ in range(steps):
        t0 = time.perf_counter()
        it, e = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(it)
        es.append(e)
    marker_pop(torch)
    # per-iteration time from a run of 20 iterations between HIP events
    ctx.init(W0d, H0d)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.fasthals_step(Xd, 20)
    e1.record()
    torch.cuda.synchronize()
    return dict(median_s=round(statistics.median(times), 6), times_s=[round(t, 6) for t in times],
                iters_to_eps=its, e_at_stop=es, per_iteration_ms=round(e0.elapsed_time(e1) / 20, 4))


# committed HBM-counter summary of the dominant kernel per workload, and the
# source file it was taken on
TRAFFIC = {"c2": ("gemm_bf16_c2_traffic.md", "gemm_lp.hip"), "c5": ("gemm_split_c5_traffic.md", "gemm_split.hip")}


def source_digest(path):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or was taken on a different source."""
    if name not in TRAFFIC:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC[name][0])
    src = os.path.join(ROOT, "paper_1712_02248_amd", "csrc", TRAFFIC[name][1])
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source sha256/16") != source_digest(src):
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def lowp_products(torch, nmfrp, Xd, m, n, kp, prec):
    """The range-finder products of the workload's precision at its shapes, on
    prepared thin operands (X B and X^T B as the range finder issues them): BF16
    reads the one row-major copy (X^T B transposed in LDS), FP8 its two copies."""
    dev = Xd.device
    B_n = torch.randn(n, kp, device=dev)
    B_m = torch.randn(m, kp, device=dev)
    Xq, XqT, E = nmfrp.quantize_x(Xd, prec)
    if prec == nmfrp.NMF_BF16 and kp <= 128:
        P1 = nmfrp.LowpProduct(prec, Xq, n, B_n)
        P2 = nmfrp.LowpProduct(prec, Xq, m, B_m, at=True, Kpad=-(-m // 128) * 128, M=n)
        del XqT
    else:
        tn = E.shape[1] if E is not None else 0
        P1 = nmfrp.LowpProduct(prec, Xq, n, B_n, E, (tn, 1))
        P2 = nmfrp.LowpProduct(prec, XqT, m, B_m, E, (1, tn))
    return P1, P2


def kernel_timing(torch, nmfrp, Xd, m, n, kp, reps, prec, name):
    """Per-launch times of the compression products at the workload's shapes.
    The low-precision range-finder products and (c5) the split-BF16 products are
    timed alone on prepared operands (X B and X^T B alternating, as the range
    finder issues them); the FP32 products and the split-BF16 products are also
    timed per library call (product plus split-K sum).  The dominant kernel of
    the headline path, which the roofline object describes, is the BF16
    range-finder product at c2 and the split-BF16 product at c5 (its refinement
    power iteration and projected data)."""
    dev = Xd.device
    B_n = torch.randn(n, kp, device=dev)
    B_m = torch.randn(m, kp, device=dev)
    Y_m = torch.empty(m, kp, device=dev)
    Y_n = torch.empty(n, kp, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, count):
        fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1) / (reps * count)

    flops = 2.0 * m * n * kp
    res = {}
    for label, fn in (("fp32 X*B (call)", lambda: nmfrp.gemm(Xd, B_n, False, Y_m)),
                      ("fp32 X^T*B (call)", lambda: nmfrp.gemm(Xd, B_m, True, Y_n)),
                      ("split-bf16 X*B (call)", lambda: nmfrp.gemm_split(Xd, 0, B_n)),
                      ("split-bf16 X^T*B (call)", lambda: nmfrp.gemm_split(Xd, 1, B_m))):
        ms = timed(fn, 1)
        res[label] = dict(ms=round(ms, 5), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                          frac_fp32_mfma=round(flops / (ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                          x_gbs=round(4.0 * m * n / (ms * 1e-3) / 1e9, 1))
        log(f"[bench] {label}: {ms:.4f} ms  {res[label]['tflops']:.1f} TFLOP/s  X at {res[label]['x_gbs']} GB/s")
    del Y_m, Y_n
    P1, P2 = lowp_products(torch, nmfrp, Xd, m, n, kp, prec)
    es = 2 if prec == nmfrp.NMF_BF16 else 1
    fmt = "bf16" if prec == nmfrp.NMF_BF16 else "fp8"
    alg = float(es) * m * n                     # bytes of X per launch
    for label, fn, cnt in ((f"{fmt} X*B (kernel)", P1.run, 1), (f"{fmt} X^T*B (kernel)", P2.run, 1),
                           (f"{fmt} both (kernel)", lambda: (P1.run(), P2.run()), 2)):
        ms = timed(fn, cnt)
        res[label] = dict(ms=round(ms, 5), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                          x_gbs=round(alg / (ms * 1e-3) / 1e9, 1))
        log(f"[bench] {label}: {ms:.4f} ms  {res[label]['tflops']:.1f} TFLOP/s  X at {res[label]['x_gbs']} GB/s")
    if name == "c5":
        S1, S2 = nmfrp.SplitProduct(Xd, 0, B_n), nmfrp.SplitProduct(Xd, 1, B_m)
        for label, fn, cnt in (("split-bf16 X*B (kernel)", S1.run, 1), ("split-bf16 X^T*B (kernel)", S2.run, 1),
                               ("split-bf16 both (kernel)", lambda: (S1.run(), S2.run()), 2)):
            ms = timed(fn, cnt)
            res[label] = dict(ms=round(ms, 5), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                              x_gbs=round(4.0 * m * n / (ms * 1e-3) / 1e9, 1))
            log(f"[bench] {label}: {ms:.4f} ms  {res[label]['tflops']:.1f} TFLOP/s  "
                f"X at {res[label]['x_gbs']} GB/s")
        dom = res["split-bf16 both (kernel)"]
        # three BF16 MFMA products per product term: the split arithmetic's peak is a third of BF16's
        peak = PEAK_BF16_TFLOPS / 3.0
        achieved = flops / (dom["ms"] * 1e-3) / 1e12
        res["roofline"] = dict(
            bound="mfma",
            kernel="gemm_split_wide_kernel (split-BF16 product on FP32 X: the refinement power iteration and the "
                   "projected data; X B and X^T B alternating, split-K partials)",
            achieved=round(achieved, 2), peak=round(peak, 2), unit="TFLOP/s", frac=round(achieved / peak, 4),
            traffic=measured_traffic(name), algorithmic_flops_per_launch=flops,
            units_per_launch=f"{m}x{n} X elements x {kp} thin columns, 2 flops each",
            launch_us=round(dom["ms"] * 1e3, 2), splits=[S1.splits, S2.splits],
            peak_note="BF16 dense 2500 TFLOP/s / 3 (hi hi + hi lo + lo hi per term)",
            x_gbs=dom["x_gbs"], x_hbm_frac=round(dom["x_gbs"] / PEAK_HBM_GBS, 4))
        del S1, S2
        return res
    dom = res[f"{fmt} both (kernel)"]
    achieved = alg / (dom["ms"] * 1e-3) / 1e9
    peak_mfma = PEAK_BF16_TFLOPS if fmt == "bf16" else PEAK_FP8_TFLOPS
    kname = ("gemm_bf16_nt_kernel (BF16 range-finder product; X B and X^T B alternating on the one row-major BF16 "
             "copy, split-K partials)" if fmt == "bf16" and kp <= 128 else
             f"gemm_{fmt}_nt_kernel ({fmt.upper()} range-finder product; X B on the copy of X and X^T B on the copy "
             "of X^T, alternating, split-K partials)")
    res["roofline"] = dict(
        bound="hbm", kernel=kname,
        achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4),
        traffic=measured_traffic(name), algorithmic_bytes_per_launch=alg,
        units_per_launch=f"{m}x{n} X elements, {es} B each",
        launch_us=round(dom["ms"] * 1e3, 2), splits=[P1.splits, P2.splits],
        mfma_tflops=dom["tflops"], mfma_peak_tflops=peak_mfma,
        mfma_frac=round(dom["tflops"] / peak_mfma, 4))
    return res


def probe_kernels(torch, nmfrp, Xd, m, n, kp, reps, prec, name):
    """For hardware-counter runs: a plain copy of known size, then the dominant
    kernel at the workload's shapes (reps launches of each shape)."""
    src = torch.empty(m * n, dtype=torch.float32, device=Xd.device).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    del src, dst
    if name == "c5":   # the split-BF16 product on FP32 X
        S1 = nmfrp.SplitProduct(Xd, 0, torch.randn(n, kp, device=Xd.device))
        S2 = nmfrp.SplitProduct(Xd, 1, torch.randn(m, kp, device=Xd.device))
        for _ in range(reps):
            S1.run()
            S2.run()
        torch.cuda.synchronize()
        splits = [S1.splits, S2.splits]
        del S1, S2
        # then the FP8 range-finder products, and reps FastHALS-RP iterations with
        # FP32 and with split-BF16 update products (FP8 compression, cold factors)
        P1, P2 = lowp_products(torch, nmfrp, Xd, m, n, kp, nmfrp.NMF_FP8_E4M3)
        for _ in range(reps):
            P1.run()
            P2.run()
        torch.cuda.synchronize()
        del P1, P2
        import datagen
        cfg = datagen.CONFIGS[name]
        r = cfg["r"]
        g = torch.Generator(device=Xd.device)
        g.manual_seed(7)
        W0 = torch.rand(m, r, device=Xd.device, generator=g)
        H0 = torch.rand(n, r, device=Xd.device, generator=g)
        for up in (0, 1):
            ctx = nmfrp.NMF(m, n, r, kp, cfg["q"], seed=1, prec=nmfrp.NMF_FP8_E4M3, refine_fp32=2, lowp_sketches=2,
                            update_prec=up)
            ctx.compress(Xd)
            ctx.init(W0, H0)
            ctx.step(reps)
            ctx.sync()
            ctx.close()
        print(json.dumps(dict(probe="kernels", copy_bytes=4 * m * n, x_bytes=4 * m * n, splits=splits,
                              M=[m, n], N=kp, reps=reps,
                              source_sha256_16=source_digest(os.path.join(ROOT, "paper_1712_02248_amd", "csrc",
                                                                          "gemm_split.hip")))), flush=True)
        return
    P1, P2 = lowp_products(torch, nmfrp, Xd, m, n, kp, prec)
    for _ in range(reps):
        P1.run()
        P2.run()
    torch.cuda.synchronize()
    es = 2 if prec == nmfrp.NMF_BF16 else 1
    print(json.dumps(dict(probe="kernels", copy_bytes=4 * m * n, x_bytes=es * m * n,
                          splits=[P1.splits, P2.splits], M=[m, n], N=kp, reps=reps,
                          source_sha256_16=source_digest(os.path.join(ROOT, "paper_1712_02248_amd", "csrc",
                                                                      "gemm_lp.hip")))), flush=True)


# Parameter study grids (Sec 5.2): components r, oversampling r_ov (k' = r + r_ov),
# power iterations q.  P1 and P2 stand in for the two data sets of that section
# (their grids), c2 is the workload of the same name.
SWEEPS = {
    "P1": dict(rs=[10, 20, 30, 40, 50], r_ov=5, qs=[1, 2, 3, 4, 5]),
    "P2": dict(rs=[50, 60, 70, 80, 90], r_ov=12, qs=[1, 3, 5, 7, 9, 11]),
    "c2": dict(rs=[16, 32, 48, 64], r_ov=32, qs=[0, 1, 2, 3, 4]),
}


def run_sweep(torch, nmfrp, datagen, name, args):
    """FastHALS-RP (median over test-matrix seeds) and FastHALS after the workload's
    iteration count, for every (r, q) of the grid, with the compressed data's
    singular values and their decay fits (both readings of the decay law)."""
    cfg = dict(datagen.CONFIGS[name])
    grid = SWEEPS[name]
    m, n, iters = cfg["m"], cfg["n"], cfg["iters"]
    seed = datagen.cfg_seed(name)
    log(f"[sweep] generating {name} X {m}x{n}")
    X = datagen.make_x(name)
    Xd = torch.from_numpy(X).cuda()
    points, unc, skipped = [], {}, []
    spec = None
    for r in grid["rs"]:
        kp = r + grid["r_ov"]
        if r > 128 or kp > 128 or kp > min(m, n):
            skipped.append(dict(r=r, kp=kp, why="r > 128 or k' > 128 (the sketch spectrum's limit) or k' > min(m, n)"))
            continue
        W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
        W0d, H0d = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
        ctx = nmfrp.NMF(m, n, r, kp, 0, seed=seed)
        ctx.init(W0d, H0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.fasthals_step(Xd, iters)
        torch.cuda.synchronize()
        unc[r] = dict(r=r, e=ctx.residual(Xd), iters_ms=round((time.perf_counter() - t0) * 1e3, 3))
        del ctx
        for q in grid["qs"]:
            es, tc, ti = [], [], []
            for s_ in range(args.sweep_seeds):
                ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed + 1000 * s_)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.compress(Xd)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                ctx.init(W0d, H0d)
                ctx.step(iters)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                es.append(ctx.residual(Xd))
                tc.append(t1 - t0)
                ti.append(t2 - t1)
                if s_ == 0:
                    sig = ctx.sketch_spectrum().numpy()
                del ctx
            pt = dict(r=r, kp=kp, q=q, e_median=statistics.median(es), e=es,
                      compress_ms=round(statistics.median(tc) * 1e3, 3), iters_ms=round(statistics.median(ti) * 1e3, 3),
                      e_fasthals=unc[r]["e"])
            points.append(pt)
            log(f"[sweep] r={r} k'={kp} q={q}: e_rp {pt['e_median']:.6e} (FastHALS {unc[r]['e']:.6e}), "
                f"compress {pt['compress_ms']} ms, {iters} iterations {pt['iters_ms']} ms")
            spec = (r, kp, q, sig)
    best = {}
    for pt in points:
        b = best.get(pt["r"])
        if b is None or pt["e_median"] < b["e_median"]:
            best[pt["r"]] = pt
    out = dict(study="parameter sweep (Sec 5.2)", workload=name, m=m, n=n, iters=iters, r_ov=grid["r_ov"],
               seeds=args.sweep_seeds, data="synthetic", points=points, fasthals=list(unc.values()),
               best_q={r: b["q"] for r, b in best.items()}, skipped=skipped)
    if spec is not None:
        r, kp, q, sig = spec
        j = np.arange(1, kp + 1, dtype=np.float64)
        ls = np.log(np.maximum(sig, 1e-300))
        out["spectrum"] = dict(r=r, kp=kp, q=q, sigma=[float(v) for v in sig],
                               decay_power=float(-np.polyfit(np.log(j), ls, 1)[0]),
                               decay_exp=float(-np.polyfit(j, ls, 1)[0]))
    print(json.dumps(out), flush=True)


def run_c4(torch, nmfrp, datagen, args):
    """The warm-start experiment on new columns: a network trained on pairs from
    the 65536 x 4096 parts workload's generator (the bench's protocol) is applied
    to a new problem of --c4-cols columns from the same generator (same parts W0,
    new coefficients), compressed as the c2 headline compresses (BF16 range
    finder, split-BF16 sketches).  Reported: the error right after each
    initialisation and after 20 FastHALS-RP iterations, for the cold factors,
    the warm start (W_ref, network rows with rejection, 20 NNLS sweeps), the
    control without the network, the network with a cold W, and the warm start
    without sweeps."""
    from datagen import device as ddev
    cfg = dict(datagen.CONFIGS["c2"])
    cfg["name"] = "c2"
    m, r, kp, q = cfg["m"], cfg["r"], cfg["kp"], cfg["q"]
    seed = datagen.cfg_seed("c2")
    W0gen = torch.from_numpy(datagen.parts_w0(m, cfg["r_true"], seed).astype(np.float32)).cuda()
    fresh = lambda ncols, chunk: ddev.parts_fresh_columns(torch, nmfrp.gaussian, W0gen, ncols, seed, chunk)
    log("[c4] training the warm-start network")
    net, Q_train, W_ref, info = train_warm_start(torch, nmfrp, cfg, seed, args, fresh)
    n4 = args.c4_cols
    X4 = fresh(n4, 100000)      # a chunk id the training does not use
    mean = float(X4.sum(dtype=torch.float64)) / (m * n4)
    W0, H0 = datagen.init_factors(mean, m, n4, r, seed + 7)
    W0d, H0d = torch.from_numpy(W0).cuda(), torch.from_numpy(H0).cuda()
    ctx = nmfrp.NMF(m, n4, r, kp, q, seed=seed, prec=nmfrp.NMF_BF16, lowp_sketches=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.compress(X4)
    torch.cuda.synchronize()
    t_comp = time.perf_counter() - t0
    sw = args.refine_sweeps
    rows = {}
    for label, warm in (("cold", None), ("warm", (net, Q_train, W_ref, sw, "ref")),
                        ("ctrl_no_net", (net, Q_train, W_ref, sw, "no_net")),
                        ("net_cold_w", (net, Q_train, W_ref, sw, "cold_w")),
                        ("warm_no_sweeps", (net, Q_train, W_ref, 0, "ref"))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if warm is None:
            ctx.init(W0d, H0d)
            nrej = None
        else:
            nrej = warm_start(ctx, warm, W0d, H0d, count=True)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        e0 = ctx.residual(X4)
        ctx.step(20)
        e20 = ctx.residual(X4)
        rows[label] = dict(e_after_init=e0, e_after_20_iters=e20, init_ms=round(t_init * 1e3, 3), rejected_rows=nrej)
        log(f"[c4] {label}: e after init {e0:.6e}, after 20 iterations {e20:.6e}, init {t_init * 1e3:.2f} ms, "
            f"rejected {nrej}")
    ctx.close()
    print(json.dumps(dict(study="warm start on new columns", m=m, n=n4, r=r, k_sketch=kp, q=q, data="synthetic",
                          generator="parts (same W0 as the 65536 x 4096 workload, new coefficients)",
                          compress_ms=round(t_comp * 1e3, 3), refine_sweeps=sw, training=info, results=rows)),
          flush=True)


def run_c3(torch, nmfrp, datagen, args, steps=3, warmup=1):
    """c3 time to eps: the BF16 range finder (FP32 sketches, as the parity test and
    the oracle's BF16 model have them, and split-BF16 sketches) against plain FP32,
    from the cold factors, eps = (1 + 1e-3) e_oracle(150 it); and the BF16
    range-finder product at c3's shapes (X B and X^T B on the one row-major BF16
    copy).  X is drawn on the host (untimed) and resident in HBM when the clock
    starts."""
    name = "c3"
    cfg = dict(datagen.CONFIGS[name])
    cfg["name"] = name
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    seed = datagen.cfg_seed(name)
    e_oracle = json.load(open(GOLDEN))[name]["e"]
    eps = (1.0 + 1e-3) * e_oracle
    dev = torch.device("cuda:0")
    log(f"[bench] c3: generating X {m}x{n} on the host (untimed)")
    X = datagen.make_x(name)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    Xd = torch.from_numpy(X).to(dev)
    del X
    W0d, H0d = torch.from_numpy(W0).to(dev), torch.from_numpy(H0).to(dev)
    torch.cuda.synchronize()
    F32, BF = nmfrp.NMF_FP32, nmfrp.NMF_BF16
    out = {}
    for vname, prec, lps in (("plain", F32, 0), ("bf16", BF, 0), ("bf16_split_sketches", BF, 2)):
        v = time_variant(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, prec, 0, None, steps, warmup,
                         label=f"c3 {vname}", lps=lps)
        st, it = v["stages"], v["iters"][-1]
        out[vname] = dict(median_s=round(statistics.median(v["times"]), 6), times_s=[round(t, 6) for t in v["times"]],
                          iters_to_eps=v["iters"], reached_eps=all(e <= eps for e in v["e"]), e_at_stop=v["e"],
                          stage_ms=dict(compress=round(st["compress_ms"], 3), iterations=round(st["step_ms"], 3),
                                        per_iteration=round(st["step_ms"] / max(it, 1), 4),
                                        residual=round(st["residual_ms"], 4)))
        log(f"[bench] c3 {vname}: median {out[vname]['median_s'] * 1e3:.2f} ms, iters {v['iters']}, "
            f"e {v['e'][-1]:.8e}")
    kt = kernel_timing(torch, nmfrp, Xd, m, n, kp, args.kernel_reps, BF, name)
    best = min(("bf16", "bf16_split_sketches"), key=lambda k: out[k]["median_s"])
    res = dict(workload=f"c3: X {m}x{n} FP32 synthetic (Poisson counts of {cfg['r_true']} planted topics), r={r}, "
                        f"k'={kp}, q={q}, eps=(1+1e-3) e_oracle({cfg['iters']} it); BF16 range finder vs plain FP32, "
                        "cold factors",
               eps=eps, e_oracle=e_oracle, variants=out, fastest_bf16=best,
               speedup_vs_plain=round(out["plain"]["median_s"] / out[best]["median_s"], 3),
               gemm=kt)
    del Xd, W0d, H0d
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this compressed-NMF build runs and is measured on one GPU only; "
              "--gpus N with N > 1 is not supported (row sharding across GPUs is a design note, "
              "not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    import datagen
    from paper_1712_02248_amd import nmfrp

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    nmfrp.load()
    if args.sweep:
        run_sweep(torch, nmfrp, datagen, args.sweep, args)
        return
    if args.c4:
        run_c4(torch, nmfrp, datagen, args)
        return
    name = args.workload
    if name == "c3":
        print(json.dumps(run_c3(torch, nmfrp, datagen, args, args.steps, args.warmup)), flush=True)
        return
    cfg = dict(datagen.CONFIGS[name])
    cfg["name"] = name
    if cfg["family"] not in ("parts", "dyadic_parts"):
        sys.exit("bench.py: the warm-start protocol draws new columns of the parts families (c2, c5); "
                 "c3 runs with --workload c3")
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    iters_cfg = cfg["iters"]
    seed = datagen.cfg_seed(name)
    head_name = HEADLINE[name]
    BF, F8, F32 = nmfrp.NMF_BF16, nmfrp.NMF_FP8_E4M3, nmfrp.NMF_FP32
    lp_prec = F8 if name == "c5" else BF

    golden = json.load(open(GOLDEN)).get(name) if os.path.exists(GOLDEN) else None
    if args.probe_kernels:   # counters do not depend on the values of X
        g = torch.Generator(device="cuda:0")
        g.manual_seed(seed)
        probe_kernels(torch, nmfrp, torch.rand(m, n, device="cuda:0", generator=g), m, n, kp, 5, lp_prec, name)
        return
    from datagen import device as ddev
    dev = torch.device("cuda:0")
    if cfg["family"] == "dyadic_parts":
        log(f"[bench] forming {name} X {m}x{n} on the device")
        Xd, W0gen, mean = ddev.dyadic_parts_x(torch, nmfrp.gaussian, name)
        X = None
        fresh = lambda ncols, chunk: ddev.dyadic_fresh_columns(torch, nmfrp.gaussian, W0gen, ncols, seed, chunk)
    else:
        log(f"[bench] generating {name} X {m}x{n} on the host")
        X = datagen.make_x(name)
        mean = X.mean()
        Xd = torch.from_numpy(X).to(dev)
        W0gen = torch.from_numpy(datagen.parts_w0(m, cfg["r_true"], seed).astype(np.float32)).to(dev)
        fresh = lambda ncols, chunk: ddev.parts_fresh_columns(torch, nmfrp.gaussian, W0gen, ncols, seed, chunk)
    W0, H0 = datagen.init_factors(mean, m, n, r, seed)
    W0d = torch.from_numpy(W0).to(dev)
    H0d = torch.from_numpy(H0).to(dev)
    torch.cuda.synchronize()

    if golden is not None:
        e_oracle = golden["e"]
        eps = (1.0 + 1e-3) * e_oracle
        eps_src = "oracle"
    else:  # no stored oracle value: plain FP32 run of the configured length
        c0 = nmfrp.NMF(m, n, r, kp, q, seed=seed)
        c0.compress(Xd)
        c0.init(W0d, H0d)
        _, e_ref = c0.fit(Xd, iters_cfg, 0.0, iters_cfg)
        e_oracle = None
        eps = (1.0 + 1e-3) * e_ref
        eps_src = "gpu-fp32-reference"
        del c0
    log(f"[bench] eps = {eps:.6e} ({eps_src})")

    log("[bench] training the warm-start network (untimed)")
    net, Q_train, W_ref, warm_info = train_warm_start(torch, nmfrp, cfg, seed, args, fresh)
    sw = args.refine_sweeps

    def warm(mode="ref", sweeps=sw):
        return (net, Q_train, W_ref, sweeps, mode)

    # (name, prec, refinement (0 none, 1 FP32, 2 split-BF16), warm start, sketch
    #  products (0 FP32, 1 low precision, 2 split BF16), steps, warmup[, update
    #  products (0 FP32, 1 split BF16)])
    S, W_ = args.steps, args.warmup
    if name == "c5":
        variants = [("plain", F32, 0, None, 0, S, W_),
                    (head_name, F8, 2, warm(), 2, S, W_, 1)]
        extra = [("fp8_warm_fp32_updates", F8, 2, warm(), 2, 2, 1, 0),
                 ("fp8_warm_fp32_refine", F8, 1, warm(), 2, 2, 1, 1),
                 ("fp8_ctrl_no_net", F8, 2, warm("no_net"), 2, 2, 1, 1),
                 ("fp8_net_cold_w", F8, 2, warm("cold_w"), 2, 2, 1, 1),
                 ("fp8_net_no_sweeps", F8, 2, warm(sweeps=0), 2, 2, 1, 1),
                 ("fp8_refine", F8, 2, None, 2, 2, 1, 1),
                 ("bf16_warm", BF, 0, warm(), 2, 3, 1, 1),
                 ("bf16", BF, 0, None, 2, 2, 1, 1),
                 ("fp32_warm", F32, 0, warm(), 2, 2, 1)]
    else:
        variants = [("plain", F32, 0, None, 0, S, W_),
                    (head_name, BF, 0, warm(), 2, S, W_)]
        extra = [("bf16_warm_fp32_sketches", BF, 0, warm(), 0, 3, 1),
                 ("bf16_warm_lowp_sketches", BF, 0, warm(), 1, 3, 1),
                 ("bf16_ctrl_no_net", BF, 0, warm("no_net"), 2, 3, 1),
                 ("bf16_net_cold_w", BF, 0, warm("cold_w"), 2, 3, 1),
                 ("bf16_net_no_sweeps", BF, 0, warm(sweeps=0), 2, 3, 1),
                 ("bf16", BF, 0, None, 0, 3, 1),
                 ("bf16_lowp_sketches", BF, 0, None, 1, 3, 1),
                 ("bf16_refine", BF, 1, None, 0, 3, 1),
                 ("fp8_refine", F8, 1, None, 0, 3, 1),
                 ("fp8_refine_warm", F8, 1, warm(), 0, 3, 1),
                 ("fp32_warm", F32, 0, warm(), 0, 3, 1),
                 ("fp8_warm", F8, 0, warm(), 2, 3, 1)]
    if not args.headline_only:
        variants += extra
    if args.variants:
        keep = args.variants.split(",")
        variants = [v for v in variants if v[0] in keep]
    out = {}
    for vname, prec, refine, w, lps, steps, warmup, *up in variants:
        v = time_variant(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, prec, refine, w, steps, warmup,
                         label=vname, lps=lps, up=up[0] if up else 0)
        out[vname] = v
        log(f"[bench] {vname}: median {statistics.median(v['times']) * 1e3:.2f} ms, iters {v['iters']}, "
            f"e_init {v['e_init']:.4e}, e {v['e'][-1]:.6e}, rejected {v['rejected']}")
    unc = None
    if not args.headline_only and (not args.variants or "fasthals_uncompressed" in args.variants.split(",")):
        unc = time_uncompressed(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, 2 if name == "c5" else 3, 1)
        log(f"[bench] fasthals_uncompressed: median {unc['median_s'] * 1e3:.2f} ms, iters {unc['iters_to_eps']}, "
            f"{unc['per_iteration_ms']:.3f} ms per iteration")
    head = out.get(head_name) or next(iter(out.values()))
    plain = out.get("plain")
    total_head = sum(head["times"])

    # ---- kernel timing at the exact shapes of the compression, HIP events on the
    # stream the kernels are launched on (the current torch stream).
    kt = kernel_timing(torch, nmfrp, Xd, m, n, kp, args.kernel_reps, lp_prec, name)
    roofline = kt.pop("roofline")

    def summary(v):
        st = v["stages"]
        it = v["iters"][-1]
        return dict(median_s=round(statistics.median(v["times"]), 6), times_s=[round(t, 6) for t in v["times"]],
                    iters_to_eps=v["iters"], reached_eps=all(e <= eps for e in v["e"]), e_at_stop=v["e"],
                    e_after_init=v["e_init"],
                    e_after_20_iters=v["e_20"],
                    e_after_same_iters=v["e_fixed"],
                    rejected_rows=v["rejected"],
                    stage_ms=dict(compress=round(st["compress_ms"], 3), iterations=round(st["step_ms"], 3),
                                  per_iteration=round(st["step_ms"] / max(it, 1), 4),
                                  residual=round(st["residual_ms"], 4)))

    ref_v = plain or head
    per_iter_ms = ref_v["stages"]["step_ms"] / max(ref_v["iters"][-1], 1)
    upd_bytes = 8.0 * (m + n) * (kp + r)
    upd_flops = 2.0 * r * (m + n) * (2 * kp + r)
    vmed = statistics.median(head["times"])
    pmed = statistics.median(plain["times"]) if plain else None
    hdesc = ("FP8 e4m3 range finder (128 x 128 block scales) with one split-BF16 refinement power iteration per "
             "side, split-BF16 sketches and update products" if name == "c5" else
             "BF16 range finder, split-BF16 sketches")
    line = dict(
        metric=f"time-to-rel-error eps (s), {'FP8' if name == 'c5' else 'BF16'} compression + learned warm start "
               "(plain FP32 alongside)",
        value=round(vmed, 6), unit="s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(total_head / args.steps * 1e3, 3), higher_is_better=False,
        scaling="weak", vs_baseline=None, dtype="fp8" if name == "c5" else "bf16", data="synthetic",
        config=dict(workload=f"{name}: X {m}x{n} FP32 synthetic ({cfg['family']} family, r_true="
                    f"{cfg['r_true']}), r={r}, k'={kp}, q={q}, eps=(1+1e-3) e_oracle({iters_cfg} it); "
                    f"{hdesc}, MLP warm start of H ({sw} NNLS sweeps) vs plain FP32",
                    m=m, n=n, r=r, k_sketch=kp, q=q, iters_cfg=iters_cfg, check_every=args.check_every,
                    refine_sweeps=sw),
        eps=eps, eps_source=eps_src, e_oracle=e_oracle,
        plain_fp32=dict(value=round(pmed, 6), **summary(plain)) if plain else None,
        speedup_vs_plain=round(pmed / vmed, 3) if plain else None,
        variants={k: summary(v) for k, v in out.items()},
        # the paper's RP vs no-RP comparison (Sec 2.2 vs eq fastHALS_a), both FP32 and cold
        fasthals_uncompressed=(dict(unc, speedup_of_rp_plain=round(unc["median_s"] / pmed, 3) if plain else None)
                               if unc else None),
        warm_start=warm_info,
        gemm=kt,
        update_loop=dict(algorithmic_bytes_per_iteration=upd_bytes, algorithmic_flops_per_iteration=upd_flops,
                         per_iteration_ms=round(per_iter_ms, 4),
                         gbs=round(upd_bytes / (per_iter_ms * 1e-3) / 1e9, 1),
                         tflops=round(upd_flops / (per_iter_ms * 1e-3) / 1e12, 2),
                         frac_fp32_mfma=round(upd_flops / (per_iter_ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)),
        roofline=roofline,
    )
    if name == "c5" and not (args.headline_only or args.variants or args.no_c3):
        # c3, the BF16 configuration: the c5 data leave HBM first
        del Xd, W0d, H0d, net, Q_train, W_ref, W0gen
        torch.cuda.empty_cache()
        line["c3"] = run_c3(torch, nmfrp, datagen, args)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a row sample (cpu_baseline)")
        rows = args.cpu_rows or (8192 if name == "c5" else 65536)
        its = args.cpu_iters or (10 if name == "c5" else 300)
        line["cpu_baseline"] = cpu_baseline(cfg, X, W0, H0, ref_v["iters"][-1], rows, its)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
