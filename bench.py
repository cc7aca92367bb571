#!/usr/bin/env python3
"""Time-to-relative-error for compressed NMF (FastHALS-RP) on one MI355X:
BF16 compression with a learned warm start of H, against plain FP32.

One step = the whole hot path on the workload's X, which is resident in HBM
when the clock starts: compress (device-drawn Gaussian test matrices, range
finder with power iterations and FP64 CholeskyQR2, sketch products), set the
initial factors, then FastHALS-RP iterations with an exact FP64 residual check
schedule until e <= eps.  eps = (1 + 1e-3) * e_oracle, where e_oracle is the FP64
oracle's error after the workload's iteration count (stored by
tests/golden/make_oracle_errors.py, which calls only the oracle).

Variants (same X, same cold factors):
  plain      FP32 range finder, cold start (the paper's method).
  bf16_warm  BF16 range-finder products with FP32 accumulation, split-BF16
             sketch products on X (three BF16 products per term, about 16
             significant bits), then the learned warm start: W from the reference
             dictionary, H rows from the network on the compressed columns,
             each kept only if it beats the cold row on the compressed
             residual, then column-NNLS sweeps.  The step includes the
             alignment products, inference, selection and sweeps; it excludes
             training.
  others     FP32 sketch products (bf16_warm_fp32_sketches), BF16 sketches
             (their error floor lies above eps at c2), bf16 / fp8 (+ FP32
             refinement) cold starts, fp32_warm and fp8_warm, reported
             alongside.
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
PEAK_HBM_GBS = 8000.0
# the headline variant: BF16 range finder, split-BF16 sketches, learned warm start
HEADLINE = "bf16_warm"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--check-every", type=int, default=0, help="0: adaptive residual checks")
    ap.add_argument("--max-iters", type=int, default=0, help="0: the workload's iteration count")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=65536, help="rows of X in the oracle sample")
    ap.add_argument("--cpu-iters", type=int, default=300, help="oracle iterations timed in the sample")
    ap.add_argument("--pairs", type=int, default=200000, help="training pairs (rounded up to 4096)")
    ap.add_argument("--epochs", type=int, default=50, help="most training passes")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--nnls-sweeps", type=int, default=100)
    ap.add_argument("--refine-sweeps", type=int, default=20,
                    help="column-NNLS sweeps on the warm rows against the reference dictionary")
    ap.add_argument("--headline-only", action="store_true", help="time only plain and bf16_warm")
    ap.add_argument("--variants", default="", help="comma list of variants to time (default: all)")
    ap.add_argument("--sweep", default="", help="parameter study instead of the bench: P1, P2 or c2 "
                    "(components r x power iterations q, FastHALS-RP against FastHALS, sketch spectrum)")
    ap.add_argument("--sweep-seeds", type=int, default=3, help="test-matrix seeds per sweep point (median)")
    ap.add_argument("--probe-kernels", action="store_true",
                    help="only a copy of known size and the dominant kernel (for counter runs)")
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
    """The FP64 oracle on a row sample of X, scaled linearly to the full workload."""
    import datagen
    from oracle import nmf, philox
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    ms = min(rows, m)
    seed = datagen.cfg_seed(cfg["name"])
    Xs = X[:ms]
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


def gpu_fresh_columns(torch, nmfrp, W0d, ncols, seed, chunk, noise=0.01):
    """New columns of the parts family drawn on the device (input synthesis,
    untimed): max(0, W0 h + noise N(0,1)) with h from the chunk's own stream."""
    import datagen
    H = torch.from_numpy(datagen.fresh_h(W0d.shape[1], ncols, seed, chunk).astype(np.float32)).cuda()
    N = nmfrp.gaussian(W0d.shape[0], ncols, 1000 + chunk, seed)
    return torch.clamp_min(W0d @ H + noise * N, 0.0)


def train_warm_start(torch, nmfrp, cfg, seed, args):
    """Reference fit, pair generation and Adam training (all untimed)."""
    import datagen
    from paper_1712_02248_amd import warmstart
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    info = {}
    W0gen = torch.from_numpy(datagen.parts_w0(m, cfg["r_true"], seed).astype(np.float32)).cuda()
    t0 = time.perf_counter()
    # reference fit on one new draw of the generator
    Xt = gpu_fresh_columns(torch, nmfrp, W0gen, n, seed, 0)
    ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed + 1)
    Wi, Hi = datagen.init_factors(float(Xt.mean()), m, n, r, seed + 1)
    ctx.compress(Xt)
    ctx.init(torch.from_numpy(Wi).cuda(), torch.from_numpy(Hi).cuda())
    _, e_ref = ctx.fit(Xt, cfg["iters"], 0.0, cfg["iters"])
    Q_train = ctx.left_basis()
    W_ref, _ = ctx.factors()
    Wh_star = warmstart.compressed_factor(Q_train, W_ref)
    del Xt
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # pairs from new columns
    chunk = 4096
    nchunks = -(-args.pairs // chunk)
    npairs = nchunks * chunk
    Xin = torch.empty(npairs, kp, device="cuda")
    T = torch.empty(npairs, r, device="cuda")
    for c in range(nchunks):
        Xf = gpu_fresh_columns(torch, nmfrp, W0gen, chunk, seed, 1 + c)
        a, b = warmstart.make_pairs(Q_train, Wh_star, Xf, sweeps=args.nnls_sweeps)
        Xin[c * chunk:(c + 1) * chunk] = a
        T[c * chunk:(c + 1) * chunk] = b
    Xv = gpu_fresh_columns(torch, nmfrp, W0gen, chunk, seed, 1 + nchunks)
    Xin_v, T_v = warmstart.make_pairs(Q_train, Wh_star, Xv, sweeps=args.nnls_sweeps)
    del Xf, Xv
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


def time_variant(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, prec, refine, warm, steps, warmup,
                 label="", lps=0):
    from paper_1712_02248_amd import warmstart
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    max_iters = args.max_iters or cfg["iters"]
    ctx = nmfrp.NMF(m, n, r, kp, q, seed=seed, prec=prec, refine_fp32=refine, lowp_sketches=lps)

    def step():
        ctx.compress(Xd)
        if warm is None:
            ctx.init(W0d, H0d)
        else:
            net, Q_train, W_ref, sweeps = warm
            warmstart.warm_init(ctx, net, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps)
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
    # stage split (library events) of a repeat of the last step's work
    def start():
        ctx.compress(Xd)
        if warm is None:
            ctx.init(W0d, H0d)
            return None
        net, Q_train, W_ref, sweeps = warm
        return warmstart.warm_init(ctx, net, Q_train, W_ref, Ht_cold=H0d, refine_sweeps=sweeps, count=True)

    nrej = start()
    e0 = ctx.residual(Xd)
    ctx.step(20)
    e20 = ctx.residual(Xd)
    start()
    ctx.step(its[-1])
    e_fixed = ctx.residual(Xd)
    st = ctx.stage_times()
    return dict(times=times, iters=its, e=es, e_init=e0, e_20=e20, e_fixed=e_fixed, stages=st, rejected=nrej,
                ctx=ctx)


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


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_bf16_c2_traffic.md")
DOMINANT_SRC = os.path.join(ROOT, "paper_1712_02248_amd", "csrc", "gemm_lp.hip")


def source_digest(path):
    import hashlib
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or was taken on a different source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source sha256/16") != source_digest(DOMINANT_SRC):
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def kernel_timing(torch, nmfrp, Xd, m, n, kp, reps):
    """Per-launch times of the compression products at the workload's shapes.
    The dominant kernel of the BF16 path, the BF16 product, is timed alone on
    prepared operands (X B and X^T B alternating, as the range finder issues
    them); the FP32 products are timed per library call (product plus split-K
    sum)."""
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
                      ("fp32 X^T*B (call)", lambda: nmfrp.gemm(Xd, B_m, True, Y_n))):
        ms = timed(fn, 1)
        res[label] = dict(ms=round(ms, 5), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                          frac_fp32_mfma=round(flops / (ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4),
                          x_gbs=round(4.0 * m * n / (ms * 1e-3) / 1e9, 1))
    Xq, _, _ = nmfrp.quantize_x(Xd, nmfrp.NMF_BF16)
    P1 = nmfrp.LowpProduct(nmfrp.NMF_BF16, Xq, n, B_n)
    # X^T B reads the same row-major copy, its tiles transposed in LDS (as in the range finder)
    P2 = nmfrp.LowpProduct(nmfrp.NMF_BF16, Xq, m, B_m, at=True, Kpad=-(-m // 128) * 128, M=n)
    alg = 2.0 * m * n                     # bytes of X per launch (BF16)
    for label, fn, cnt in (("bf16 X*B (kernel)", P1.run, 1), ("bf16 X^T*B (kernel)", P2.run, 1),
                           ("bf16 both (kernel)", lambda: (P1.run(), P2.run()), 2)):
        ms = timed(fn, cnt)
        res[label] = dict(ms=round(ms, 5), tflops=round(flops / (ms * 1e-3) / 1e12, 2),
                          x_gbs=round(alg / (ms * 1e-3) / 1e9, 1))
        log(f"[bench] {label}: {ms:.4f} ms  {res[label]['tflops']:.1f} TFLOP/s  X at {res[label]['x_gbs']} GB/s")
    dom = res["bf16 both (kernel)"]
    achieved = alg / (dom["ms"] * 1e-3) / 1e9
    traffic = measured_traffic()
    res["roofline"] = dict(
        bound="hbm", kernel="gemm_bf16_nt_kernel<128,64,2,2,*> (BF16 range-finder product; X B and X^T B "
                            "alternating on the one row-major BF16 copy, split-K partials)",
        achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s", frac=round(achieved / PEAK_HBM_GBS, 4),
        traffic=traffic, algorithmic_bytes_per_launch=alg, units_per_launch=f"{m}x{n} X elements, 2 B each",
        launch_us=round(dom["ms"] * 1e3, 2), splits=[P1.splits, P2.splits],
        mfma_tflops=dom["tflops"], mfma_frac_bf16=round(dom["tflops"] / 2500.0, 4))
    return res


def probe_kernels(torch, nmfrp, Xd, m, n, kp, reps):
    """For hardware-counter runs: a plain copy of known size, then the dominant
    kernel at the workload's shapes (reps launches of each shape)."""
    src = torch.empty(m * n, dtype=torch.float32, device=Xd.device).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    B_n = torch.randn(n, kp, device=Xd.device)
    B_m = torch.randn(m, kp, device=Xd.device)
    Xq, _, _ = nmfrp.quantize_x(Xd, nmfrp.NMF_BF16)
    P1 = nmfrp.LowpProduct(nmfrp.NMF_BF16, Xq, n, B_n)
    P2 = nmfrp.LowpProduct(nmfrp.NMF_BF16, Xq, m, B_m, at=True, Kpad=-(-m // 128) * 128, M=n)
    for _ in range(reps):
        P1.run()
        P2.run()
    torch.cuda.synchronize()
    print(json.dumps(dict(probe="kernels", copy_bytes=4 * m * n, bf16_x_bytes=2 * m * n,
                          splits=[P1.splits, P2.splits], M=[m, n], N=kp, reps=reps,
                          source_sha256_16=source_digest(DOMINANT_SRC))), flush=True)


# Parameter study grids (Sec 5.2): components r, oversampling r_ov (k' = r + r_ov),
# power iterations q.  P1 and P2 stand in for the two data sets of that section
# (their grids; r above 64 exceeds this build's kernels), c2 is the bench workload.
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
        if r > 64 or kp > 128 or kp > min(m, n):
            skipped.append(dict(r=r, kp=kp, why="r > 64 or k' > 128 exceeds this build's kernels"))
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
    name = args.workload
    cfg = dict(datagen.CONFIGS[name])
    cfg["name"] = name
    if cfg["family"] != "parts":
        sys.exit("bench.py: the warm-start protocol draws new columns of the parts family (c2, c5)")
    m, n, r, kp, q = cfg["m"], cfg["n"], cfg["r"], cfg["kp"], cfg["q"]
    iters_cfg = cfg["iters"]
    seed = datagen.cfg_seed(name)

    golden = json.load(open(GOLDEN)).get(name) if os.path.exists(GOLDEN) else None
    if args.probe_kernels:   # counters do not depend on the values of X
        g = torch.Generator(device="cuda:0")
        g.manual_seed(seed)
        probe_kernels(torch, nmfrp, torch.rand(m, n, device="cuda:0", generator=g), m, n, kp, 5)
        return
    log(f"[bench] generating {name} X {m}x{n} on the host")
    X = datagen.make_x(name)
    W0, H0 = datagen.init_factors(X.mean(), m, n, r, seed)
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    W0d = torch.from_numpy(W0).to(dev)
    H0d = torch.from_numpy(H0).to(dev)

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
    log(f"[bench] eps = {eps:.6e} ({eps_src})")

    log("[bench] training the warm-start network (untimed)")
    net, Q_train, W_ref, warm_info = train_warm_start(torch, nmfrp, cfg, seed, args)
    warm = (net, Q_train, W_ref, args.refine_sweeps)
    warm_net_only = (net, Q_train, W_ref, 0)

    # (name, prec, FP32 refinement, warm start, sketch products (0 FP32, 1 low precision,
    #  2 split BF16), steps, warmup)
    BF, F8, F32 = nmfrp.NMF_BF16, nmfrp.NMF_FP8_E4M3, nmfrp.NMF_FP32
    variants = [("plain", F32, 0, None, 0, args.steps, args.warmup),
                (HEADLINE, BF, 0, warm, 2, args.steps, args.warmup)]
    if not args.headline_only:
        variants += [("bf16_warm_fp32_sketches", BF, 0, warm, 0, 3, 1),
                     ("bf16_warm_lowp_sketches", BF, 0, warm, 1, 3, 1),
                     ("bf16", BF, 0, None, 0, 3, 1),
                     ("bf16_lowp_sketches", BF, 0, None, 1, 3, 1),
                     ("bf16_refine", BF, 1, None, 0, 3, 1),
                     ("fp8_refine", F8, 1, None, 0, 3, 1),
                     ("fp8_refine_warm", F8, 1, warm, 0, 3, 1),
                     ("fp32_warm", F32, 0, warm, 0, 3, 1),
                     ("bf16_warm_net_only", BF, 0, warm_net_only, 0, 3, 1),
                     ("fp8_warm", F8, 0, warm, 2, 3, 1)]
    if args.variants:
        keep = args.variants.split(",")
        variants = [v for v in variants if v[0] in keep]
    out = {}
    for vname, prec, refine, w, lps, steps, warmup in variants:
        v = time_variant(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, prec, refine, w, steps, warmup,
                         label=vname, lps=lps)
        out[vname] = v
        log(f"[bench] {vname}: median {statistics.median(v['times']) * 1e3:.2f} ms, iters {v['iters']}, "
            f"e_init {v['e_init']:.4e}, e {v['e'][-1]:.6e}, rejected {v['rejected']}")
    unc = None
    if not args.headline_only and (not args.variants or "fasthals_uncompressed" in args.variants.split(",")):
        unc = time_uncompressed(torch, nmfrp, cfg, seed, Xd, W0d, H0d, eps, args, 3, 1)
        log(f"[bench] fasthals_uncompressed: median {unc['median_s'] * 1e3:.2f} ms, iters {unc['iters_to_eps']}, "
            f"{unc['per_iteration_ms']:.3f} ms per iteration")
    head = out.get(HEADLINE) or next(iter(out.values()))
    plain = out.get("plain")
    total_head = sum(head["times"])

    # ---- kernel timing at the exact shapes of the compression, HIP events on the
    # stream the kernels are launched on (the current torch stream).
    kt = kernel_timing(torch, nmfrp, Xd, m, n, kp, args.kernel_reps)
    roofline = kt.pop("roofline")

    def summary(v):
        st = v["stages"]
        it = v["iters"][-1]
        return dict(median_s=round(statistics.median(v["times"]), 6), times_s=[round(t, 6) for t in v["times"]],
                    iters_to_eps=v["iters"], e_at_stop=v["e"], e_after_init=v["e_init"],
                    e_after_20_iters=v["e_20"],
                    e_after_same_iters=v["e_fixed"],
                    rejected_rows=v["rejected"],
                    stage_ms=dict(compress=round(st["compress_ms"], 3), iterations=round(st["step_ms"], 3),
                                  per_iteration=round(st["step_ms"] / max(it, 1), 4),
                                  residual=round(st["residual_ms"], 4)))

    ref_v = plain or head
    per_iter_ms = ref_v["stages"]["step_ms"] / max(ref_v["iters"][-1], 1)
    upd_bytes = 8.0 * (m + n) * (kp + r)
    vmed = statistics.median(head["times"])
    pmed = statistics.median(plain["times"]) if plain else None
    line = dict(
        metric="time-to-rel-error eps (s), BF16 compression + learned warm start (plain FP32 alongside)",
        value=round(vmed, 6), unit="s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(total_head / args.steps * 1e3, 3), higher_is_better=False,
        scaling="weak", vs_baseline=None, dtype="bf16", data="synthetic",
        config=dict(workload=f"{name}: X {m}x{n} FP32 synthetic ({cfg['family']} family, r_true="
                    f"{cfg['r_true']}), r={r}, k'={kp}, q={q}, eps=(1+1e-3) e_oracle({iters_cfg} it); "
                    f"BF16 range finder, split-BF16 sketches, MLP warm start of H ({args.refine_sweeps} NNLS "
                    f"sweeps) vs plain FP32",
                    m=m, n=n, r=r, k_sketch=kp, q=q, iters_cfg=iters_cfg, check_every=args.check_every,
                    refine_sweeps=args.refine_sweeps),
        eps=eps, eps_source=eps_src, e_oracle=e_oracle,
        plain_fp32=dict(value=round(pmed, 6), **summary(plain)) if plain else None,
        speedup_vs_plain=round(pmed / vmed, 3) if plain else None,
        variants={k: summary(v) for k, v in out.items()},
        # the paper's RP vs no-RP comparison (Sec 2.2 vs eq fastHALS_a), both FP32 and cold
        fasthals_uncompressed=(dict(unc, speedup_of_rp_plain=round(unc["median_s"] / pmed, 3) if plain else None)
                               if unc else None),
        warm_start=warm_info,
        gemm=kt,
        update_loop=dict(algorithmic_bytes_per_iteration=upd_bytes, per_iteration_ms=round(per_iter_ms, 4),
                         gbs=round(upd_bytes / (per_iter_ms * 1e-3) / 1e9, 1)),
        roofline=roofline,
    )
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a row sample (cpu_baseline)")
        line["cpu_baseline"] = cpu_baseline(cfg, X, W0, H0, ref_v["iters"][-1], args.cpu_rows, args.cpu_iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
