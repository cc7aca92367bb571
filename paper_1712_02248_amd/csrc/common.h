// Shared device/host definitions for the gfx950 compressed-NMF kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

#define NMF_DEV __device__ __forceinline__

__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ static inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---------------------------------------------------------------------------
// Kernel launch helpers (all take the caller's stream).  Each returns the
// hipError_t of the launch.
// ---------------------------------------------------------------------------

// Philox4x32-10 draws (philox.hip).
hipError_t launch_philox_normal(float* out, int64_t rows, int64_t cols, int64_t ld,
                                uint32_t stream_id, uint64_t seed, hipStream_t st);
hipError_t launch_philox_uniform(float* out, int64_t rows, int64_t cols, int64_t ld,
                                 uint32_t stream_id, uint64_t seed, float scale, hipStream_t st);

// FP32 MFMA GEMM (gemm_f32.hip): C[M x N] = op(A)[M x K] * B[K x N].
//   a_trans = 0: A is M x K row-major, element (i,k) at A[i*lda + k]
//   a_trans = 1: A is given as K x M row-major, element (i,k) at A[k*lda + i]
//   B is K x N row-major (ldb).  C is M x N row-major (ldc).
//   With splits > 1 the K range is split; partials go to `part` (splits*M*N
//   floats) and are summed in fixed order by a second kernel.
size_t gemm_f32_part_floats(int64_t M, int64_t N, int splits);
// sq (optional, A not transposed): FP64 sum of squares of A per workgroup, gemm_f32_sq_parts() values
int gemm_f32_sq_parts(int64_t M, int64_t N, int64_t K, int splits);
hipError_t launch_gemm_f32(const float* A, int64_t lda, int a_trans, const float* B, int64_t ldb,
                           float* C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                           int splits, float* part, hipStream_t st, double* sq = nullptr);
int gemm_f32_pick_splits(int64_t M, int64_t N, int64_t K, int a_trans);

// Low-precision copies of X and of the thin operand (quant.hip).  Xq is m x ldq,
// XqT is n x ldqt; ldq, ldqt are multiples of 128 and the padding is zero.
int quant_sq_parts(int64_t m, int64_t n, int64_t ldq, int64_t ldqt);
hipError_t launch_quant_bf16(const float* X, int64_t ldx, int64_t m, int64_t n, uint16_t* Xq,
                             int64_t ldq, uint16_t* XqT, int64_t ldqt, hipStream_t st, double* sq_part = nullptr, double* sq_out = nullptr);
// Xq only (row-major), for the transposing X^T product: n % 4 == 0, aligned X and Xq.
hipError_t launch_quant_bf16_rows(const float* X, int64_t ldx, int64_t m, int64_t n, uint16_t* Xq, int64_t ldq,
                                  hipStream_t st, double* sq_part = nullptr, double* sq_out = nullptr);
// E: ceil(m/128) x ceil(n/128) tile exponents (row-major).
hipError_t launch_quant_fp8(const float* X, int64_t ldx, int64_t m, int64_t n, int* E, uint8_t* Xq,
                            int64_t ldq, uint8_t* XqT, int64_t ldqt, hipStream_t st, double* sq_part = nullptr, double* sq_out = nullptr);
hipError_t launch_prep_b_bf16(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* Bt,
                              int64_t ldbt, hipStream_t st);
// Ebt: ceil(K/128) exponents, one per 128-row block of B.
hipError_t launch_prep_b_fp8(const float* B, int64_t ldb, int64_t K, int64_t N, int* Ebt, uint8_t* Bt,
                             int64_t ldbt, hipStream_t st);

// Low-precision NT products (gemm_lp.hip): C[M x N] = A[M x Kpad] Bt[N x Kpad]^T.
int gemm_lp_pick_splits(int64_t M, int64_t N, int64_t Kpad, int bm);
// 1: rotate the K order per XCD (thin operand too large to stay in L2), 0: per workgroup
int rot_per_xcd(int64_t N, int64_t kchunk, int splits, int elem_bytes);
// C[i][j] = sum over z ascending of part[z][i][j] (splits x M x N FP32 partials)
hipError_t launch_splitk_reduce_lp(const float* part, int splits, float* C, int64_t ldc, int64_t M, int64_t N,
                                   hipStream_t st);

// Split-BF16 products on FP32 X (gemm_split.hip), for the projected data.
// Thin operand B (K x N FP32, ldb) -> BtH (and BtL if not NULL: split lo part),
// N x ldbt BF16, zero for k >= K; ldbt % 64 == 0.  Also the BF16 copy of the
// range-finder products (BtL NULL).
hipError_t launch_prep_bt(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* BtH, uint16_t* BtL,
                          int64_t ldbt, hipStream_t st);
// C[M x N] = op(X) B: at = 0, X is M x K (ldx); at = 1, X is K x M.  ldx % 4 == 0,
// 16-byte aligned X; ldbt >= round_up(K, 64).  splits > 1: partials in part
// (splits x M x N), summed in fixed order.  sq (at = 0): FP64 sum of squares of X
// per workgroup, gemm_split_sq_parts() values.
int gemm_split_pick_splits(int64_t M, int64_t N, int64_t K);
int gemm_split_sq_parts(int64_t M, int64_t N, int splits);
hipError_t launch_gemm_split(const float* X, int64_t ldx, int at, const uint16_t* BtH, const uint16_t* BtL,
                             int64_t ldbt, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int splits,
                             float* part, hipStream_t st, double* sq = nullptr);
// the product kernel alone (splits > 1: partials z at part + z M N, not summed)
hipError_t launch_gemm_split_kernel(const float* X, int64_t ldx, int at, const uint16_t* BtH, const uint16_t* BtL,
                             int64_t ldbt, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int splits,
                             float* part, hipStream_t st, double* sq = nullptr);
// a_trans = 1 (N <= 128): A is the K x lda copy of X itself (C = A^T Bt^T, M
// columns of A, rows at or past K read as zero), not a K-contiguous copy.
hipError_t launch_gemm_bf16_nt(const uint16_t* A, int64_t lda, const uint16_t* Bt, int64_t ldbt,
                               float* C, int64_t ldc, int64_t M, int64_t N, int64_t Kpad, int splits,
                               float* part, hipStream_t st, bool reduce = true, int a_trans = 0,
                               int64_t K = 0);
// EA: exponent of A's 128 x 128 tile (ti, tk) at EA[ti * ea_i + tk * ea_k]; EB per 128-row block.
hipError_t launch_gemm_fp8_nt(const uint8_t* A, int64_t lda, const int* EA, int64_t ea_i, int64_t ea_k,
                              const uint8_t* Bt, int64_t ldbt, const int* EB, float* C, int64_t ldc,
                              int64_t M, int64_t N, int64_t Kpad, int splits, float* part,
                              hipStream_t st, bool reduce = true);

// Tall-skinny QR pieces (qr.hip).
// G = Y^T Y in FP64: split partials, then the deterministic sum into G (k x k).
hipError_t launch_gram_f64(const float* Y, int64_t ldy, int64_t rows, int k, double* part,
                           int splits, double* G, const int* skip_flag, hipStream_t st);
int gram_pick_splits(int64_t rows, int k);
// Eigenvalues of a symmetric k x k FP64 matrix (k <= 128; lower triangle read) by
// parallel cyclic Jacobi in one workgroup (eig.hip): w descending, or their clamped
// square roots with sqrt_out; info[0] = sweeps, info[1] = 1 for a non-finite entry.
hipError_t launch_sym_eig(const double* A, int64_t lda, int k, int sqrt_out, double* w, int* info, hipStream_t st);
// C (ka x kb, row-major FP32) = A^T B over `rows` rows, FP64 accumulation (ka, kb <= the
// Gram's k; part: splits x ka x kb doubles; C64: ka x kb doubles).
hipError_t launch_atb_f32out(const float* A, int64_t lda, int ka, const float* B, int64_t ldb, int kb,
                             int64_t rows, double* part, int splits, double* C64, float* C, hipStream_t st);
hipError_t launch_cholesky(const double* G, int k, int64_t rows, double* Rinv, int* status,
                           int attempt, hipStream_t st);
// Bt != NULL (k <= 64): write the transposed BF16 copy of the result (k x ldbt,
// ldbt % 64 == 0, zero past rows) instead of Y, for the next BF16 product.
hipError_t launch_apply_rinv(float* Y, int64_t ldy, int64_t rows, int k, const double* Rinv,
                             const int* status, int attempt, hipStream_t st, uint16_t* Bt = nullptr,
                             int64_t ldbt = 0);

// Fused HALS half-step (hals.hip).  The kernel derives its compressed factor C
// and Gram G from the other side's summed partials (acc_in), sweeps the rows of
// F, and leaves its own summed partials in acc_out (Qb^T F, then the column sums
// of F^2) for the next half-step.
struct HalfStepArgs {
  const float* S;       // N x kp sketch (ld lds): Xc for the W side, Xh for the H side
  int64_t lds;
  const double* acc_in; // kp*r + r: the other side's Qb'^T F' and column sums of F'^2
  int norm_in;          // 1: acc_in comes from the W side; normalise C by its column norms
  int normalize;        // 0 none, 1 compensated, 2 literal
  float* F;             // N x r factor updated in place (ld r): W or Ht
  const float* scale;   // r column scales for F on load when norm_in == 0 (NULL = 1)
  float* scale_pub;     // workgroup 0 writes 1/||a_j|| here (NULL = skip)
  float* C_pub;         // workgroup 0 writes C (kp x r) here (NULL = skip)
  float* G_pub;         // workgroup 0 writes G (r x r) here (NULL = skip)
  const float* Qb;      // N x kp basis (ld ldq) for re-compression: Q_L or Q_R
  int64_t ldq;
  int64_t N;
  int kp, r;
  float* part;          // nblk x (kp*r + r) workgroup partials
  double* acc_out;      // kp*r + r summed partials of this half-step
  float alpha, beta;    // sparsity / smoothness (0, 0 = plain rule)
  float* gbuf;          // N x r scratch (wide-factor path, with a sweep)
  float* aux;           // halfstep_big_aux_floats() scratch (wide-factor path)
  int split;            // wide-factor path: 1 = products on split-BF16 MFMA instead of FP32 MFMA
};
int halfstep_blocks(int64_t N);
size_t halfstep_part_floats(int64_t N, int kp, int r);
hipError_t launch_halfstep(const HalfStepArgs& a, int do_sweep, hipStream_t st);
// Wide factors (r <= 128, k' <= 256, beyond the fused kernel's r <= 64, k' <= 128):
// prep, gradient product, row sweep and partial products as separate launches.
bool halfstep_big(int kp, int r);
size_t halfstep_big_aux_floats();
hipError_t launch_halfstep_big(const HalfStepArgs& a, int do_sweep, hipStream_t st);
// Uncompressed FastHALS (Sec 2.2): one sweep over the rows of F against P and G
// (FP64, r x r); sq (optional) gets hals_rows_blocks(N) x r column sums of F^2.
int hals_rows_blocks(int64_t N);
hipError_t launch_hals_rows(const float* P, int64_t ldp, const double* G, int64_t N, int r, float* F, int64_t ldf,
                            float* sq, hipStream_t st);
// a_j /= sqrt(sumsq[j]) in W (M x r, ld); mode 1 also b_j *= sqrt(sumsq[j]) in Ht (N x r, ld);
// mode 0: nothing.
hipError_t launch_col_normalise(float* W, int64_t M, float* Ht, int64_t N, int r, int64_t ld, const double* sumsq,
                                int mode, hipStream_t st);
// out[e] = sum_s part[s * ne + e] in FP64, fixed order (skip: NULL or flag; skipped when *skip == 0).
hipError_t launch_sum_partials_f32(const float* part, int nparts, int64_t ne, double* out,
                                   hipStream_t st);
hipError_t launch_sum_partials_f64(const double* part, int nparts, int64_t ne, double* out,
                                   const int* skip, hipStream_t st);

// Gini coefficient (gini.hip): out2[0] = sum_i (2 i - N - 1) b_(i) (sorted
// ascending, i from 1), out2[1] = sum_i b_i, both FP64.
size_t gini_workspace_bytes(int64_t rows, int64_t cols);
hipError_t launch_gini(const float* B, int64_t ldb, int64_t rows, int64_t cols, void* ws, double* out2,
                       hipStream_t st);

// Residual (residual.hip): sum (X - W diag(sw) Ht^T)^2 and sum X^2 in FP64.
int residual_blocks(int64_t m, int64_t n);
int proxy_blocks(int64_t n);
hipError_t launch_proxy(const float* Xh, int64_t ldx, const float* Ht, int r, const float* Wh, int kp, int64_t n,
                        double* part, hipStream_t st);
hipError_t launch_residual(const float* X, int64_t ldx, int64_t m, int64_t n, const float* W,
                           const float* sw, const float* Ht, int r, double* part, double* out,
                           unsigned* counter, hipStream_t st, const double* gate = nullptr,
                           double gate_thr2 = 0.0);
// The same sums from split-BF16 products (stopping tests): KR = r padded (64 or
// 128, 0 when r > 128); ws holds residual_split_halves() BF16 values (the splits
// of W diag(sw) and Ht); fewer partials than residual_blocks().
int residual_split_kr(int r);
size_t residual_split_halves(int64_t m, int64_t n, int r);
hipError_t launch_residual_split(const float* X, int64_t ldx, int64_t m, int64_t n, const float* W, const float* sw,
                                 const float* Ht, int r, uint16_t* ws, double* part, double* out, unsigned* counter,
                                 hipStream_t st, const double* gate = nullptr, double gate_thr2 = 0.0,
                                 int64_t sstep = 1);   // sstep > 1: every sstep-th 256-row strip only

// Small utilities (util.hip).
hipError_t launch_fill_f32(float* p, int64_t count, float v, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st);
hipError_t launch_gather_host(const double* po, const double* ro, const int* qs, double* out, hipStream_t st);
hipError_t launch_copy2d(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows,
                         int64_t cols, hipStream_t st);
hipError_t launch_scale_cols(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows,
                             int cols, const float* scale, hipStream_t st);
hipError_t launch_check_nonneg(const float* X, int64_t ldx, int64_t m, int64_t n, int* flags,
                               hipStream_t st);
// learned warm start (mlp.hip)
hipError_t launch_mlp_gemm(int at, int bt, int epi, const float* A, int lda, const float* B, int ldb,
                           float* C, int ldc, int M, int N, int K, const float* bias, const float* aux,
                           int ldaux, hipStream_t st);
hipError_t launch_scale_rows(const float* X, int64_t ldx, const int* idx, int64_t nsrc, int Bn, int k,
                             const float* T, int64_t ldt, int r, float* Xs, float* Ts, float* nrm, hipStream_t st);
size_t nnls_rows_lds_bytes(int k, int r);
hipError_t launch_nnls_rows(const float* Xr, int64_t ldx, int n, int k, const float* Wh, int r, int sweeps,
                            int warm, float* H, int64_t ldh, hipStream_t st);
hipError_t launch_loss_grad(const float* Z3, const float* Ts, int Bn, int r, float* dZ3, double* lpart,
                            double* loss_out, double* loss_acc, hipStream_t st);
hipError_t launch_colsum(const float* dZ, int Bn, int N, float* gb, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, int t,
                       hipStream_t st);
hipError_t launch_infer_out(const float* Z3, const float* nrm, int Bn, int r, float* out, int64_t ldo,
                            hipStream_t st);
// count[0] = number of nonzero flags (n flags)
hipError_t launch_count(const int* flags, int n, long long* count, hipStream_t st);
hipError_t launch_select(const float* Xh, int64_t ldx, int n, int k, const float* Wh, int r, const float* Hn,
                         const float* Hc, float* Hout, int* rejected, long long* count, hipStream_t st);

// host runtime glue shared by nmfrp.cpp and mlp_rt.cpp
struct nmf_mlp;
hipError_t mlp_infer_rows(nmf_mlp* net, const float* in, int64_t ld_in, int64_t n, float* out, int64_t ldo,
                          hipStream_t st);
void mlp_dims(const nmf_mlp* net, int* k, int* h, int* r);
void nmf_set_thread_error(const char* msg);


