/*
 * nmfrp -- compressed non-negative matrix factorisation on AMD MI355X (gfx950).
 *
 * Method: G. Torre, M. Graber, "An Efficient Algorithm for Non-Negative Matrix
 * Factorization with Random Projections" (arXiv 1712.02248).  Given X >= 0
 * (m x n, rows are datapoints, Sec 2) and a rank r, find W >= 0 (m x r, the
 * paper's A) and Ht >= 0 (n x r, the paper's B) with X ~ W Ht^T (eq 2.1),
 * minimising 1/2 ||X - W Ht^T||_F^2 (eq 2.2).  X is compressed once into two
 * sketches (Sec 3.1, eq 3.5; Sec 4):
 *   Q_L (m x k') orthonormal basis of (X X^T)^q X Omega_L,   Xh = X^T Q_L (n x k'),
 *   Q_R (n x k') orthonormal basis of (X^T X)^q X^T Omega_R, Xc = X Q_R   (m x k'),
 * and the FastHALS-RP updates (eq fastHALS_a) run on the sketches only.
 *
 * Conventions for every call below
 *  - Matrices are row-major.  Pointers named X, W, Ht, Q*, X*, omega_*, and the
 *    buffers of the MLP calls are DEVICE pointers; sizes are element counts.
 *  - The second factor crosses the boundary as Ht (n x r), the transpose of an
 *    r x n H: row j of Ht is the coefficient vector of data column j, the unit
 *    the H sweep, the column NNLS and the warm-start network work on.  A caller
 *    holding H (r x n, row-major) passes it as Ht by transposing.
 *  - All work is queued on the HIP stream given at creation; calls return after
 *    queueing unless documented as synchronising.  Asynchronous HIP faults and
 *    device-side flags surface at the next synchronising call.
 *  - The library never allocates device memory: the caller passes a workspace
 *    of nmf_workspace_bytes() bytes that it owns and keeps alive until
 *    nmf_destroy().  X is borrowed: it is read by nmf_compress, nmf_residual and
 *    nmf_fit only while those calls run on the stream.
 *  - Errors: every call returns an nmf_status; nothing is thrown across the ABI.
 *    nmf_last_error() gives a message for the last failure on a context (or,
 *    with NULL, for the last failure of a context-free call in this thread).
 */
#ifndef NMFRP_H
#define NMFRP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NMFRP_ABI_VERSION 1

typedef struct nmf_ctx nmf_ctx;
typedef struct nmf_mlp nmf_mlp;

typedef enum {
  NMF_OK = 0,
  NMF_EINVAL = -1,      /* bad argument, size or alignment */
  NMF_ENOMEM = -2,      /* workspace smaller than nmf_workspace_bytes() */
  NMF_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
  NMF_ESTATE = -4,      /* call out of order (e.g. step before compress/init) */
  NMF_EBREAKDOWN = -5,  /* Cholesky breakdown even after the shift */
  NMF_ENONFINITE = -6   /* non-finite input or result */
} nmf_status;

typedef enum { NMF_FP32 = 0, NMF_BF16 = 1, NMF_FP8_E4M3 = 2 } nmf_prec;

typedef struct {
  int64_t m, n;          /* X is m x n */
  int32_t r;             /* number of components (the paper's k) */
  int32_t k_sketch;      /* k' = r + r_ov (Sec 3); r < k' <= min(m, n) (Sec 3.1) */
  int32_t q;             /* power iterations (the paper's w, eq 3.5) */
  int32_t prec;          /* nmf_prec of the range-finder products (extension); the
                            projected data Xh, Xc follow lowp_sketches */
  int32_t refine_fp32;   /* with a low-precision prec: one power iteration per
                            side on X itself after the low-precision range finder,
                            its products in FP32 (1) or split-BF16 (2, as
                            nmf_gemm_split: about 16 significant bits per term) */
  int32_t normalize;     /* a_j <- a_j/||a_j|| after the A sweep (end of Sec 4):
                            0 none, 1 with b_j <- b_j ||a_j|| (default), 2 literal */
  float alpha, beta;     /* sparsity / smoothness on B (Sec 4.1); 0, 0 = plain rule */
  uint64_t seed;         /* Philox4x32-10 key for device-drawn Omega and factors */
  int32_t lowp_sketches; /* the projected data Xh, Xc (extension): 0 FP32 products on
                            X; 1 (prec != FP32 only) products on the low-precision
                            copy of X like the range finder; 2 split-BF16 products on
                            X (see nmf_gemm_split), about 16 significant bits per
                            term.  ||X||^2 for nmf_proxy_residual comes from the
                            X Q_R pass (0, 2) or the quantiser (1). */
  int32_t update_prec;   /* products of the update loop (extension): 0 FP32 MFMA; 1
                            BF16 MFMA on split operands with FP32 accumulation:
                            the gradient a = S C - F U with three parts per value
                            (v = hi + mid + lo exactly; six part products, FP32
                            accuracy: a nearly cancels as the sweep converges),
                            Q^T F with two (v = hi + lo, within 2^-16 |v|; terms
                            hi hi + hi lo + lo hi).  1 needs the wide-factor
                            half-steps (r > 64 or k' > 128), else NMF_EINVAL. */
} nmf_params;

/* ---------------------------------------------------------------- context */

/* Bytes of device workspace a context with these parameters needs (0 if the
 * parameters are invalid).  Buffers are carved from it at 256-byte alignment. */
size_t nmf_workspace_bytes(const nmf_params* p);

/* Creates a context over a caller-owned device workspace (256-byte aligned) and
 * a HIP stream (hipStream_t; NULL = the null stream).  The context struct
 * itself is host memory owned by the library until nmf_destroy(), as are one
 * internal HIP stream and two events used by nmf_compress. */
nmf_status nmf_create(const nmf_params* p, void* workspace, size_t ws_bytes, void* hip_stream,
                      nmf_ctx** out);
void nmf_destroy(nmf_ctx* ctx);
const char* nmf_last_error(const nmf_ctx* ctx);

/* Checks X >= 0 and finite (the problem statement of Sec 2).  Synchronising.
 * NMF_EINVAL if an entry is negative, NMF_ENONFINITE if one is not finite. */
nmf_status nmf_validate(nmf_ctx* ctx, const float* X, int64_t ldx);

/* Randomised two-sided compression (Sec 3, eqs 3.4-3.5; Sec 3.1; Sec 4):
 * Q_L = orth((X X^T)^q X Omega_L), Q_R = orth((X^T X)^q X^T Omega_R), with an
 * orthonormalisation (FP64 CholeskyQR2, shifted CholeskyQR3 on breakdown)
 * after every product, then Xh = X^T Q_L and Xc = X Q_R.
 * X: device, m x n, leading dimension ldx (ldx % 4 == 0, 16-byte aligned).
 * omega_L: n x k' and omega_R: m x k' (leading dimension k'), device; NULL
 * draws them on the device from Philox4x32-10 (streams 3 and 4, key = seed).
 * The right range finder runs on a second stream owned by the context (default
 * priority), forked from and joined back to the context stream within the call,
 * so the work is ordered on the context stream as usual. */
nmf_status nmf_compress(nmf_ctx* ctx, const float* X, int64_t ldx, const float* omega_L,
                        const float* omega_R);

/* Sets the initial factors (copied): W0 m x r, Ht0 n x r, device.  NULL draws
 * U[0,1) * init_scale from Philox (streams 5 and 6).  Needs no sketches (the
 * uncompressed nmf_fasthals_step runs on the factors alone); when the context
 * is or later gets compressed, Q_R^T Ht for nmf_step follows. */
nmf_status nmf_init(nmf_ctx* ctx, const float* W0, const float* Ht0, float init_scale);

/* `iters` FastHALS-RP iterations (eq fastHALS_a): the whole W sweep against
 * (Xc, Hc = Q_R^T Ht), column normalisation, then the whole H sweep against
 * (Xh, Wh = Q_L^T W).  Needs the sketches (nmf_compress or nmf_set_state) and
 * the factors (nmf_init), in either order.  Asynchronous. */
nmf_status nmf_step(nmf_ctx* ctx, int32_t iters);

/* `iters` iterations of uncompressed FastHALS (Sec 2.2) on X itself (m x n,
 * ldx >= n, ldx % 4 == 0, 16-byte aligned): the W sweep against X Ht and
 * Ht^T Ht, the column normalisation of nmf_params.normalize, then the H sweep
 * against X^T W and W^T W (FP32 MFMA products over X, FP64 Grams, FP32 sweeps).
 * The reference against which the compressed update (nmf_step) is compared.
 * Starts from the context's factors (nmf_init; a pending normalisation of the
 * compressed steps is applied first) and leaves them in place; the compressed
 * state (Q_R^T Ht) is refreshed when the context is compressed.  Asynchronous. */
nmf_status nmf_fasthals_step(nmf_ctx* ctx, const float* X, int64_t ldx, int32_t iters);

/* Exact e = ||X - W Ht^T||_F / ||X||_F in FP64 (eq 2.2).  Synchronising. */
nmf_status nmf_residual(nmf_ctx* ctx, const float* X, int64_t ldx, double* rel_err);

/* e of eq 2.2 for a stopping test against eps: from split-BF16 products of
 * W diag(sw) and Ht (v = hi + lo with hi = bf16(v), lo = bf16(v - hi); the
 * terms hi hi + hi lo + lo hi on BF16 MFMA with FP32 accumulation, one pass over
 * X, FP64 sums of squares), with the bound |e_s - e| <= beta,
 * beta = (g (1 + e_s) + u' e_s) / (1 - g) + 3 KR 2^-126 sqrt(m n) / ||X|| + 1e-12 e_s,
 * u = 2^-23, u' = u / (1 - u), g = g0 / (1 - g0),
 * g0 = 2^-24 + 3.03 2^-16 + 1.02 (3 KR) u, KR = 64 for r <= 64 and 128 for
 * r <= 128, which holds for W, Ht >= 0 (the factors after any step).
 * When |e_s - eps| <= beta the side of eps is open and the exact FP64 residual
 * (nmf_residual) runs instead: *exact = 1, *bound = 0, *rel_err exact.
 * Otherwise *exact = 0, *bound = beta, *rel_err = e_s, and e_s <= eps exactly
 * when e <= eps.  bound and exact may be NULL.  Synchronising. */
nmf_status nmf_residual_check(nmf_ctx* ctx, const float* X, int64_t ldx, double eps, double* rel_err,
                              double* bound, int32_t* exact);

/* Sketch-only estimate of e from the left sketch (Sec 3: X ~ Q_L Q_L^T X):
 *   e_p^2 = (||X||^2 - ||Xh||^2 + sum_j ||xh_j - Wh h_j||^2) / ||X||^2,
 * with Wh = Q_L^T W of the last H sweep; equal to e when the columns of W lie
 * in range(Q_L), otherwise an approximation (no pass over X).  ||X||^2 is
 * accumulated in FP64 by nmf_compress (in the quantiser's pass over X in
 * low-precision runs with lowp_sketches 1 or 2, else in the X Q_R product).  Needs at
 * least one nmf_step since the last init and a compression by nmf_compress
 * (not nmf_set_state); NMF_ESTATE otherwise.  Synchronising. */
nmf_status nmf_proxy_residual(nmf_ctx* ctx, double* rel_err);

/* Singular values of the compressed data X-hat = Q_L^T X (Sec 4; k' x n),
 * sigma_1 >= ... >= sigma_k', written to sigma (host memory, k' doubles).  For
 * every j they are at most sigma_j(X), and the leading ones approach sigma_j(X)
 * as the basis captures the dominant subspace (Sec 3.1; the power iterations of
 * eq 3.5 sharpen it).  Their decay is what the paper's parameter study relates
 * the best power-iteration count to (Sec 5.2).  Computed as the square roots of
 * the eigenvalues of X-hat X-hat^T (FP64 Gram of the stored X-hat, FP64 Jacobi;
 * see nmf_sym_eigvals).  Needs a compression (nmf_compress or nmf_set_state),
 * NMF_ESTATE otherwise; NMF_ENONFINITE for non-finite compressed data.
 * Synchronising; uses the range finder's scratch, so it must not overlap an
 * nmf_compress on the same context. */
nmf_status nmf_sketch_spectrum(nmf_ctx* ctx, double* sigma);

/* Runs steps in chunks, evaluating the residual after each chunk, until
 * e <= eps or max_iters iterations (the paper leaves the stopping rule open:
 * Alg 1-4).  check_every > 0: fixed chunks, each ending with the exact
 * residual.  check_every == 0 after nmf_compress: after every chunk (5 first,
 * then 1.2 times the iterations a straight-line extrapolation of the last two
 * readings needs to reach the target, 5..50; with one reading 20, 10 or 5 by
 * its distance from it) the residual is estimated on a sample of the rows
 * (split-BF16 products over every s-th 256-row strip, s = strips / 64, split
 * into column parts; all strips for m <= 16384; the ratio of the sampled sums
 * of (X - P)^2 and X^2).  The target is eps - beta, beta the bound of
 * nmf_residual_check's split value, below which that value decides e <= eps by
 * itself.  The split residual over all of X runs once the estimate reaches the
 * target, once it is within 1 % of eps with the target out of reach (more than
 * 20 further iterations at the current rate, or no progress), and after the
 * last chunk.  A split value within its bound of eps is followed by a few more
 * iterations and a second split residual when the target is at most 10
 * iterations away, and otherwise (or on a second such value, or after the last
 * chunk) by the exact FP64 residual.  Each stop decision is that of the exact
 * e; an estimate that errs high only delays a stop by a chunk.
 * check_every == 0 after nmf_set_state: the
 * exact residual after every chunk, starting with e at the current factors,
 * each chunk 1.5 times the iterations a straight-line extrapolation of the last
 * two values needs (5..50; 50, 20, 10 or 5 by the gap to eps when there is no
 * slope).  max_iters == 0 only evaluates e (exactly).
 * Synchronising.  *iters_done and *rel_err report the iterations run and the
 * last e (exact, or within nmf_residual_check's bound of it). */
nmf_status nmf_fit(nmf_ctx* ctx, const float* X, int64_t ldx, int32_t max_iters, double eps,
                   int32_t check_every, int32_t* iters_done, double* rel_err);

/* Copies the current factors to device buffers W (m x r) and Ht (n x r),
 * applying any pending column normalisation.  Asynchronous. */
nmf_status nmf_get_factors(nmf_ctx* ctx, float* W, float* Ht);

/* Sketch export / import (checkpoint, tests): QL m x k', QR n x k', Xh n x k',
 * Xc m x k', device, leading dimension k'.  Any pointer may be NULL (skipped).
 * set_state marks the context compressed.  Asynchronous. */
nmf_status nmf_get_state(nmf_ctx* ctx, float* QL, float* QR, float* Xh, float* Xc);
nmf_status nmf_set_state(nmf_ctx* ctx, const float* QL, const float* QR, const float* Xh,
                         const float* Xc);

/* Waits for the stream and reports device-side flags (Cholesky breakdown).
 * *shifted (may be NULL) receives the number of orthonormalisations that
 * needed the shifted fallback since the last nmf_compress. */
nmf_status nmf_sync(nmf_ctx* ctx, int32_t* shifted);

/* Stage times in milliseconds of the last compress / step / residual call
 * (HIP events on the context stream).  Synchronising. */
nmf_status nmf_stage_times(nmf_ctx* ctx, double* compress_ms, double* step_ms, double* residual_ms);

/* ------------------------------------------------- kernel-level entry points */

/* N(0,1) matrix (rows x cols, leading dimension ld) from Philox4x32-10 and
 * Box-Muller (the Gaussian test matrix of Sec 3): element e = row*cols + col
 * uses counter (e/4, 0, stream_id, 0) [64-bit e/4 in words 0-1], key = seed,
 * word e % 4; words (0,1) and (2,3) are Box-Muller pairs with
 * u = (x + 0.5) 2^-32, evaluated in FP64.  Asynchronous on hip_stream. */
nmf_status nmf_gaussian(float* out, int64_t rows, int64_t cols, int64_t ld, uint32_t stream_id,
                        uint64_t seed, void* hip_stream);
/* U[0,1) * scale with 24-bit resolution: (x >> 8) 2^-24 on the same layout. */
nmf_status nmf_uniform(float* out, int64_t rows, int64_t cols, int64_t ld, uint32_t stream_id,
                       uint64_t seed, float scale, void* hip_stream);

/* C (M x N, ldc) = op(A) B on FP32 MFMA: a_trans = 0: A is M x K (lda);
 * a_trans = 1: A is stored K x M (lda) and used transposed (X^T B).  B is K x N
 * (ldb).  N <= 256; lda, ldb multiples of 4 and A, B 16-byte aligned; K % 4 == 0
 * when a_trans = 0, M % 4 == 0 when a_trans = 1.  workspace: device scratch of
 * nmf_gemm_workspace_bytes() bytes for split-K partials.  Asynchronous. */
size_t nmf_gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int32_t a_trans);
nmf_status nmf_gemm(const float* A, int64_t lda, int32_t a_trans, const float* B, int64_t ldb,
                    float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* workspace,
                    size_t ws_bytes, void* hip_stream);

/* nmf_gemm for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product, kernels and split-K choice, with the split-K partials in a static
 * per-GPU device array of NMF_NOALLOC_SCRATCH_BYTES instead of a workspace.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library routine);
 * the caller passes A, B and C as for nmf_gemm.  Products whose partials need
 * more than the array (splits x M x N floats, see nmf_gemm_workspace_bytes)
 * return NMF_EINVAL without launching.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (other streams or threads) race.  The
 * array is looked up on the first call on each device and held until the
 * process ends.  Asynchronous on hip_stream. */
#define NMF_NOALLOC_SCRATCH_BYTES (64u << 20)
nmf_status nmf_gemm_noalloc(const float* A, int64_t lda, int32_t a_trans, const float* B, int64_t ldb,
                            float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* hip_stream);

/* Low-precision copies of X for the range-finder products (extension): writes
 * Xq (m x ldq) and its transpose XqT (n x ldqt), zero padded; ldq >= n and
 * ldqt >= m, both multiples of 128.  prec = NMF_BF16: uint16 BF16 bit patterns,
 * round to nearest even.  prec = NMF_FP8_E4M3: OCP e4m3 codes of x 2^-e, where e
 * is the exponent of the 128 x 128 tile holding x (smallest e with
 * amax(tile) <= 448 2^e, 0 for an all-zero tile), round to nearest even with
 * saturation; tile_exp receives ceil(m/128) x ceil(n/128) exponents (row-major,
 * device).  Asynchronous. */
nmf_status nmf_quantize_x(const float* X, int64_t ldx, int64_t m, int64_t n, int32_t prec, void* Xq,
                          int64_t ldq, void* XqT, int64_t ldqt, int32_t* tile_exp, void* hip_stream);

/* C (M x N, ldc) = A (M x Kpad, low precision, K-contiguous) times B (K x N FP32,
 * ldb), FP32 accumulation.  B is rounded to the same format (and transposed) in
 * the workspace first; for FP8 with one power-of-two scale per 128-row block of B.
 * FP8 A carries tile exponents: tile (ti, tk) of A at EA[ti * ea_i + tk * ea_k].
 * Kpad >= K is a multiple of 128 and A's columns K..Kpad-1 are zero.  N <= 256.
 * workspace: nmf_gemm_lowp_workspace_bytes() bytes, 256-byte aligned.  Asynchronous. */
size_t nmf_gemm_lowp_workspace_bytes(int64_t M, int64_t N, int64_t Kpad);
nmf_status nmf_gemm_lowp(int32_t prec, const void* A, int64_t lda, const int32_t* EA, int64_t ea_i,
                         int64_t ea_k, const float* B, int64_t ldb, int64_t K, int64_t N, float* C,
                         int64_t ldc, int64_t M, int64_t Kpad, void* workspace, size_t ws_bytes,
                         void* hip_stream);

/* The same product in parts, for callers that keep the thin operand prepared
 * (and for timing the product kernel alone).  nmf_lowp_prepare_thin rounds B
 * (K x N FP32, ldb) to the format and transposes it into Bt (N x Kpad, zero
 * padded; FP8 also writes the Kpad/128 block exponents EB).
 * nmf_gemm_lowp_splits gives the split-K count nmf_gemm_lowp uses.
 * nmf_gemm_lowp_prepared launches only the product kernel: with splits == 1 it
 * writes C (M x N, ldc); with splits > 1 it writes partial z (M x N, leading
 * dimension N) at C + z M N, which the caller sums.  Asynchronous. */
nmf_status nmf_lowp_prepare_thin(int32_t prec, const float* B, int64_t ldb, int64_t K, int64_t N, void* Bt,
                                 int64_t Kpad, int32_t* EB, void* hip_stream);
int32_t nmf_gemm_lowp_splits(int64_t M, int64_t N, int64_t Kpad);
nmf_status nmf_gemm_lowp_prepared(int32_t prec, const void* A, int64_t lda, const int32_t* EA, int64_t ea_i,
                                  int64_t ea_k, const void* Bt, const int32_t* EB, int64_t N, float* C,
                                  int64_t ldc, int64_t M, int64_t Kpad, int32_t splits, void* hip_stream);

/* The X^T B product of the BF16 range finder on the row-major BF16 copy itself
 * (extension): C = A^T Bt^T with A the K x M BF16 matrix (row-major, lda >= M,
 * lda % 8 == 0, 16-byte aligned; it is read in chunks of 8 columns up to lda,
 * rows K..Kpad-1 count as zero) and Bt prepared by nmf_lowp_prepare_thin (N x
 * Kpad, Kpad % 128 == 0, N <= 128).  Tiles of A are transposed while staged
 * into LDS; the result is bit-identical to nmf_gemm_lowp_prepared on A's
 * transpose (same tiles, same K order).  splits as for nmf_gemm_lowp_prepared
 * (nmf_gemm_lowp_splits(M, N, Kpad)): with splits > 1 partial z goes to
 * C + z M N.  Asynchronous. */
nmf_status nmf_gemm_bf16_at_prepared(const void* A, int64_t lda, int64_t K, const void* Bt, int64_t N, float* C,
                                     int64_t ldc, int64_t M, int64_t Kpad, int32_t splits, void* hip_stream);

/* Split-BF16 product on FP32 X (extension; the projected data X^T Q_L and
 * X Q_R of Sec 4 when lowp_sketches = 2): C (M x N, ldc) = op(X) B with
 * at = 0: X is M x K, at = 1: X is K x M (ldx >= columns, ldx % 4 == 0, X
 * 16-byte aligned); B is K x N FP32 (ldb), N <= 256.  Every value v of X and B
 * is used as hi + lo, hi = bf16(v), lo = bf16(v - hi) (nearest even); a product
 * term is hi hi + hi lo + lo hi with FP32 accumulation, within about
 * 3 * 2^-16 |x| |b| of the exact term.  workspace: nmf_gemm_split_workspace_bytes()
 * bytes, 256-byte aligned (the split thin operand and split-K partials).
 * Asynchronous on hip_stream. */
size_t nmf_gemm_split_workspace_bytes(int64_t M, int64_t N, int64_t K);
nmf_status nmf_gemm_split(const float* X, int64_t ldx, int32_t at, const float* B, int64_t ldb, int64_t K,
                          int64_t N, float* C, int64_t ldc, int64_t M, void* workspace, size_t ws_bytes,
                          void* hip_stream);

/* The split-BF16 product in parts (callers that keep the thin operand
 * prepared; timing the product kernel alone).  nmf_split_prepare_thin writes
 * the hi and lo BF16 parts of B (K x N FP32, ldb, N <= 256) transposed into BtH
 * and BtL (N x ldbt each, ldbt % 64 == 0, ldbt >= K rounded up to 64, zero
 * padded).  nmf_gemm_split_splits gives the split-K count nmf_gemm_split uses.
 * nmf_gemm_split_prepared launches only the product kernel of nmf_gemm_split:
 * with splits == 1 it writes C (M x N, ldc); with splits > 1 it writes partial
 * z (M x N, leading dimension N) at C + z M N, which the caller sums.
 * Asynchronous on hip_stream. */
nmf_status nmf_split_prepare_thin(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* BtH, uint16_t* BtL,
                                  int64_t ldbt, void* hip_stream);
int32_t nmf_gemm_split_splits(int64_t M, int64_t N, int64_t K);
nmf_status nmf_gemm_split_prepared(const float* X, int64_t ldx, int32_t at, const uint16_t* BtH, const uint16_t* BtL,
                                   int64_t ldbt, int64_t K, int64_t N, float* C, int64_t ldc, int64_t M,
                                   int32_t splits, void* hip_stream);

/* In-place orthonormalisation of Y (rows x k, ldy % 4 == 0) by FP64
 * CholeskyQR2 (shifted CholeskyQR3 on breakdown), k <= 256.  Synchronising;
 * *shifted (may be NULL) = 1 if the shifted fallback ran. */
size_t nmf_orth_workspace_bytes(int64_t rows, int32_t k);
nmf_status nmf_orth(float* Y, int64_t ldy, int64_t rows, int32_t k, void* workspace,
                    size_t ws_bytes, void* hip_stream, int32_t* shifted);

/* Eigenvalues of a symmetric k x k FP64 matrix (device, row-major, lda >= k;
 * only the lower triangle, column <= row, is read), 1 <= k <= 128, written to w
 * (device, k doubles) in descending order.  Cyclic Jacobi in parallel
 * (round-robin) order in one workgroup (Golub and Van Loan, Sec 8.5), until the
 * off-diagonal Frobenius norm is below 1e-13 of the matrix's (at most 40
 * sweeps), so each eigenvalue is within that bound.  The building block of
 * nmf_sketch_spectrum.  Synchronising; *sweeps (may be NULL) = sweeps used.
 * NMF_ENONFINITE (w not written) if an entry read is not finite. */
nmf_status nmf_sym_eigvals(const double* A, int64_t lda, int32_t k, double* w, void* hip_stream,
                           int32_t* sweeps);

/* Gini coefficient of a rows x cols FP32 matrix (device, row-major, ldb >= cols),
 * the sparsity measure of Sec 5.1 for B:
 *   G = sum_i (2 i - N - 1) b_(i) / (N sum_i b_i),  i = 1..N = rows cols,
 * over the entries sorted ascending (b_(1) <= ... <= b_(N)).  G is 0 for a
 * constant matrix and approaches 1 when one entry carries all of the sum.  The
 * entries are sorted on the device (radix sort of order-preserving 32-bit keys)
 * and both sums are formed in FP64 over the sorted order; equal values give the
 * same sums in any order, so the result does not depend on how ties are broken.
 * workspace: device, 256-byte aligned, nmf_gini_workspace_bytes(rows, cols)
 * bytes, caller-owned.  Synchronising (the result is written to *gini on the
 * host).  NMF_EINVAL for rows or cols < 1, N >= 2^32, ldb < cols, a null pointer
 * or a workspace too small; NMF_ENONFINITE if an entry or the sum is not finite
 * or the sum is 0 (G undefined). */
size_t nmf_gini_workspace_bytes(int64_t rows, int64_t cols);
nmf_status nmf_gini(const float* B, int64_t ldb, int64_t rows, int64_t cols, void* workspace, size_t ws_bytes,
                    void* hip_stream, double* gini);


/* --------------------------------------------------- learned warm start of H
 * Extension (the paper has no learned component): a multilayer perceptron maps
 * a compressed column x-hat (a row of Xh, length k') to an initial H row
 * (length r).  Net: z1 = x W1 + b1, a1 = relu(z1); z2 = a1 W2 + b2,
 * a2 = relu(z2); z3 = a2 W3 + b3, y = softplus(z3).  Parameters are one flat
 * FP32 vector in the order W1 (k' x hidden), b1, W2 (hidden x hidden), b2,
 * W3 (hidden x r), b3, each weight row-major [fan_in][fan_out].  The net sees
 * x / ||x||_2 and its output is multiplied by ||x||_2 (H is positively
 * homogeneous in X); a zero row maps to 0.  Training loss on a batch of B pairs
 * (x, t): L = 1/(2B) sum ||y - t / ||x|| ||^2; optimiser Adam (beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8, bias-corrected).  All MLP buffers are device
 * memory; every call queues on the stream given at creation. */

/* Length of the flat parameter vector (0 for invalid sizes). */
int64_t nmf_mlp_n_params(int32_t k_in, int32_t hidden, int32_t r_out);

/* Device workspace (caller-owned, 256-byte aligned) for a net that processes at
 * most max_batch rows per pass: parameters, gradients, Adam moments and
 * activations.  0 for invalid sizes (1 <= k_in <= 1024, 1 <= hidden <= 4096,
 * 1 <= r_out <= 256, 1 <= max_batch <= 65536). */
size_t nmf_mlp_workspace_bytes(int32_t k_in, int32_t hidden, int32_t r_out, int32_t max_batch);

/* Creates a net over the workspace; params (device, nmf_mlp_n_params floats) are
 * copied as the initial parameters and the Adam state is zeroed. */
nmf_status nmf_mlp_create(int32_t k_in, int32_t hidden, int32_t r_out, int32_t max_batch,
                          const float* params, void* workspace, size_t ws_bytes, void* hip_stream,
                          nmf_mlp** out);
void nmf_mlp_destroy(nmf_mlp* net);
const char* nmf_mlp_last_error(const nmf_mlp* net);

/* Parameter export / import (flat layout above, device).  set_params also zeroes
 * the Adam moments and step count.  Asynchronous. */
nmf_status nmf_mlp_get_params(nmf_mlp* net, float* flat);
nmf_status nmf_mlp_set_params(nmf_mlp* net, const float* flat);

/* Loss and gradients of one batch without an update: in_rows batch x k'
 * (ld_in), tgt_rows batch x r (ld_tgt), batch <= max_batch.  grads_flat
 * (device, may be NULL) receives the gradient in the flat layout; *loss (host,
 * may be NULL; then the call is asynchronous) receives L. */
nmf_status nmf_mlp_loss_grad(nmf_mlp* net, const float* in_rows, int64_t ld_in, const float* tgt_rows,
                             int64_t ld_tgt, int32_t batch, double* loss, float* grads_flat);

/* Adam training over npairs pairs for `epochs` passes in batches of `batch`
 * rows (the last batch of a pass may be smaller).  order (device int32,
 * epochs x npairs, may be NULL = natural order): pass e visits pairs
 * order[e*npairs .. e*npairs+npairs-1], each a permutation of 0..npairs-1
 * drawn by the caller.  epoch_loss (host, epochs doubles, may be NULL; then
 * the call is asynchronous) receives the mean batch loss of every pass. */
nmf_status nmf_mlp_train(nmf_mlp* net, const float* in_rows, int64_t ld_in, const float* tgt_rows,
                         int64_t ld_tgt, int64_t npairs, const int32_t* order, int32_t epochs,
                         int32_t batch, float lr, double* epoch_loss);

/* out_rows (rows x r, ld_out) = ||x|| softplus(net(x / ||x||)) for every row x of
 * in_rows (rows x k', ld_in).  Asynchronous. */
nmf_status nmf_mlp_infer(nmf_mlp* net, const float* in_rows, int64_t ld_in, int64_t rows,
                         float* out_rows, int64_t ld_out);

/* Training targets: for every row x of Xr (rows x k, ldx) the non-negative
 * least-squares row h = argmin_{h >= 0} ||x - Wh h||^2, Wh k x r (row-major),
 * approximated by `sweeps` H sweeps of eq fastHALS_a with Wh fixed, from h = 0
 * (warm_start = 0) or from the rows already in Ht (warm_start = 1).  r <= 64
 * and (k + R + 1) R 4 bytes <= 64 KiB with R = 16, 32 or 64, the smallest
 * that holds r.  Ht: rows x r (ldh).  Asynchronous. */
nmf_status nmf_nnls_rows(const float* Xr, int64_t ldx, int64_t rows, int32_t k, const float* Wh,
                         int32_t r, int32_t sweeps, int32_t warm_start, float* Ht, int64_t ldh,
                         void* hip_stream);

/* Warm start of a compressed context: Ht row j is the net's output on the
 * aligned compressed column x-tilde_j = M x-hat_j (align_M: k' x k' device,
 * row-major, typically M = Q_train^T Q_L for the basis Q_train the net was
 * trained in; NULL = identity), unless the cold row does better on the
 * compressed residual rho(h) = ||x-hat_j - Wh_ref h||^2 (FP64), in which case
 * the cold row is kept.  Wh_ref: k' x r device (e.g. Q_L^T W of a reference
 * fit).  Cold rows: Ht_cold (n x r device) or, with NULL, U[0,1) * init_scale
 * from Philox stream 6.  refine_sweeps > 0 then runs that many column-NNLS
 * sweeps (as nmf_nnls_rows) against Wh_ref from the selected rows; each sweep
 * can only lower a row's rho, so no row ends worse than its cold row.  W is
 * set as by nmf_init (W0, typically the reference dictionary, or Philox stream
 * 5), so the first nmf_step update is the W half-step.  The net must have
 * k_in = k' and r_out = r; it runs on the context's stream.  net = NULL is the
 * same initialisation without a network (the control that measures what the
 * network adds): every row starts from its cold row, then the refine_sweeps.
 * *n_rejected (host, may be NULL; then the call is asynchronous) receives the
 * number of cold rows kept (n without a network). */
nmf_status nmf_init_learned(nmf_ctx* ctx, nmf_mlp* net, const float* align_M, const float* Wh_ref,
                            const float* W0, const float* Ht_cold, float init_scale,
                            int32_t refine_sweeps, int64_t* n_rejected);

/* nmf_init_learned with the alignment and the reference factor formed inside
 * the library from the reference fit itself: align_M = Q_train^T Q_L and
 * Wh_ref = Q_L^T W_ref (FP64 sums over the m rows, rounded to FP32; the two
 * products run concurrently on the context's two streams), W = W_ref.
 * Q_train: m x k' (ldq >= k'), W_ref: m x r (ldw >= r), device, read only.
 * The other arguments are those of nmf_init_learned. */
nmf_status nmf_init_learned_ref(nmf_ctx* ctx, nmf_mlp* net, const float* Q_train, int64_t ldq,
                                const float* W_ref, int64_t ldw, const float* Ht_cold, float init_scale,
                                int32_t refine_sweeps, int64_t* n_rejected);

#ifdef __cplusplus
}
#endif
#endif /* NMFRP_H */
