// Tall-skinny QR of a sketch Y (rows x k, FP32) by CholeskyQR in FP64:
//   G = Y^T Y (FP64 MFMA, split over rows), G = R^T R (Cholesky), Q = Y R^{-1}
// (R^{-1} formed with the factorisation; Y R^{-1} on FP64 MFMA, written back
// as FP32 in place).
// CholeskyQR2 runs this twice; the second pass is skipped when the second Gram
// is already within 1e-6 of the identity (with FP64 Gram and R^{-1} on FP32 data
// the first pass is orthonormal to ~k u kappa^2).  On a non-positive or non-finite pivot the
// factorisation restarts with the shift s = 11 (rows k + k(k+1)) u tr(G)
// (shifted CholeskyQR, Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
// SIAM J. Sci. Comput. 2020), and a third pass is enabled (shifted CholeskyQR3).
//
// status[0]: 1 if a pass needed the shift (enables the third pass);
// status[1]: 1 if a pass failed even with the shift (sticky);
// status[2]: number of shifted factorisations (sticky);
// status[3]: 1 if the second pass was skipped (the first was orthonormal).
#include <algorithm>

#include "common.h"

namespace {

constexpr int GT = 64;        // Gram output block (GT x GT) per workgroup
constexpr int GROWS = 64;     // rows staged per chunk
constexpr int GPT = GROWS * GT / 256;   // staged elements per thread

// part[s] = Y[rows of split s]^T Y[rows of split s] restricted to the output
// block (bi, bj).  f64 16x16x4 MFMA: A[i][kk] = Y[kk][i], B[kk][j] = Y[kk][j];
// D[i][j] sits in lane j + 16 (i % 4), register i / 4.  The loads of the next
// chunk are issued before the MFMAs of the current one.
__global__ void __launch_bounds__(256)
gram_f64_kernel(const float* __restrict__ Y, int64_t ldy, int64_t rows, int k, int64_t rchunk,
                double* __restrict__ part, const int* __restrict__ skip_flag,
                const float* __restrict__ Yb, int64_t ldb, int kb) {
  // Yb == NULL: the Gram Y^T Y (k x k).  Otherwise the cross product Y^T Yb
  // (k x kb) over the same rows, partials of k x kb.
  if (skip_flag && skip_flag[0] == 0) return;
  __shared__ float Yi[GROWS][GT + 1];
  __shared__ float Yj[GROWS][GT + 1];
  const bool cross = Yb != nullptr;
  const int kc = cross ? kb : k;                     // columns of the right operand
  const int nbj = (kc + GT - 1) / GT;
  const int bi = blockIdx.x / nbj, bj = blockIdx.x % nbj;
  const bool diag = !cross && (bi == bj);
  const float* B = cross ? Yb : Y;
  const int64_t ldbb = cross ? ldb : ldy;
  const int64_t r0 = (int64_t)blockIdx.y * rchunk;
  const int64_t r1 = (r0 + rchunk < rows) ? r0 + rchunk : rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  f64x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f64x4){0, 0, 0, 0};

  float vi[GPT], vj[GPT];
  auto load = [&](int64_t c0) {
#pragma unroll
    for (int p = 0; p < GPT; ++p) {
      const int e = tid + 256 * p, rr = e / GT, cc = e % GT;
      const int64_t gr = c0 + rr;
      const int gi = bi * GT + cc, gj = bj * GT + cc;
      vi[p] = (gr < r1 && gi < k) ? Y[gr * ldy + gi] : 0.f;
      if (!diag) vj[p] = (gr < r1 && gj < kc) ? B[gr * ldbb + gj] : 0.f;
    }
  };
  if (r0 < r1) load(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += GROWS) {
#pragma unroll
    for (int p = 0; p < GPT; ++p) {
      const int e = tid + 256 * p, rr = e / GT, cc = e % GT;
      Yi[rr][cc] = vi[p];
      if (!diag) Yj[rr][cc] = vj[p];
    }
    __syncthreads();
    if (c0 + GROWS < r1) load(c0 + GROWS);
    float (*B)[GT + 1] = diag ? Yi : Yj;
#pragma unroll 4
    for (int kk = 0; kk < GROWS; kk += 4) {
      const int rr = kk + (lane >> 4);
      const double a = (double)Yi[rr][wave * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double b = (double)B[rr][t * 16 + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.y * k * kc;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = bi * GT + wave * 16 + 4 * q + (lane >> 4);
      const int j = bj * GT + t * 16 + (lane & 15);
      if (i < k && j < kc) P[(int64_t)i * kc + j] = acc[t][q];
    }
}

// G = Y^T Y for 128 < k <= 256 by 128 x 128 blocks: the three blocks (0, 0),
// (0, 1), (1, 1) of the symmetric result, the off-diagonal one written to both
// triangles of the split's partial (k x k).  Per 64-row chunk the two 128-column
// slices are staged in LDS (FP32, converted to FP64 as they enter the MFMA), the
// next chunk loaded into registers meanwhile.  Wave w owns row blocks 2 w, 2 w + 1
// and all eight column blocks of 16 (v_mfma_f64_16x16x4_f64; A[i][kk] =
// Y[kk][i], B[kk][j] = Y[kk][j]; D[i][j] in lane j + 16 (i % 4), register i / 4).
__global__ void __launch_bounds__(256)
gram_wide_kernel(const float* __restrict__ Y, int64_t ldy, int64_t rows, int k, int64_t rchunk,
                 double* __restrict__ part, const int* __restrict__ skip_flag) {
  if (skip_flag && skip_flag[0] == 0) return;
  constexpr int WB = 128, CR = 64, SROW = WB + 4, PE = CR * WB / 256;
  __shared__ float Yi[CR * SROW], Yj[CR * SROW];
  const int blk = blockIdx.x;                       // 0: (0, 0), 1: (0, 1), 2: (1, 1)
  const int bi = blk == 2 ? 1 : 0, bj = blk == 0 ? 0 : 1;
  const bool diag = bi == bj;
  const int64_t r0 = (int64_t)blockIdx.y * rchunk;
  const int64_t r1 = (r0 + rchunk < rows) ? r0 + rchunk : rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  f64x4 acc[2][8];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  float vi[PE], vj[PE];
  auto load = [&](int64_t c0) {
#pragma unroll
    for (int p = 0; p < PE; ++p) {
      const int e = tid + 256 * p, rr = e / WB, cc = e % WB;
      const int64_t gr = c0 + rr;
      const int gi = WB * bi + cc, gj = WB * bj + cc;
      vi[p] = (gr < r1 && gi < k) ? Y[gr * ldy + gi] : 0.f;
      if (!diag) vj[p] = (gr < r1 && gj < k) ? Y[gr * ldy + gj] : 0.f;
    }
  };
  if (r0 < r1) load(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += CR) {
#pragma unroll
    for (int p = 0; p < PE; ++p) {
      const int e = tid + 256 * p, rr = e / WB, cc = e % WB;
      Yi[rr * SROW + cc] = vi[p];
      if (!diag) Yj[rr * SROW + cc] = vj[p];
    }
    __syncthreads();
    if (c0 + CR < r1) load(c0 + CR);
    const float* B = diag ? Yi : Yj;
#pragma unroll 2
    for (int kk = 0; kk < CR; kk += 4) {
      const int rr = kk + g4;
      double av[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = (double)Yi[rr * SROW + 32 * wave + 16 * a + l16];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const double bv = (double)B[rr * SROW + 16 * b + l16];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv, acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.y * k * k;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int i = WB * bi + 32 * wave + 16 * a + 4 * x + g4, j = WB * bj + 16 * b + l16;
        if (i < k && j < k) {
          P[(int64_t)i * k + j] = acc[a][b][x];
          if (!diag) P[(int64_t)j * k + i] = acc[a][b][x];
        }
      }
}

// One workgroup factorises G = L L^T and inverts L, then writes
// R^{-1} = L^{-T} (upper, k x k).  TD x TD threads hold both matrices in
// registers, block-cyclically: thread (tx, ty) owns rows i = ty + TD a and
// columns l = tx + TD b (a, b < PB).  Column j (right-looking, pivot
// p = A[j][j], L[i][j] = A[i][j] / sqrt(p), A[i][l] -= L[i][j] L[l][j] for
// j < l <= i) is published through LDS together with row j of X, where X = L^{-1}
// is built by forward elimination on the identity in the same loop
// (X[j][:] /= L[j][j], then X[i][:] -= L[i][j] X[j][:] for i > j).
// attempt 0: first pass, resets the per-orthonormalisation flags.
// attempt 1: second pass; if G is already within 1e-6 of I (the first pass was
//            orthonormal to working precision) it only sets status[3] (skip).
// attempt 2: third pass, only after a shifted factorisation (status[0]).
// Factorisation of the k x k lower triangle of G (ld ldg) plus shift I, k <= KMAX,
// and R^{-1} written to Rinv (ld ldr; upper triangle, zeros below), visible to
// the whole workgroup on return.  Returns false (uniformly, nothing written) on
// a non-positive or non-finite pivot.  Called by every thread of a TD x TD
// workgroup.
template <int KMAX, int TD>
__device__ bool chol_factor_inverse(const double* __restrict__ G, int ldg, int k, double shift,
                                    double* __restrict__ Rinv, int ldr, double (*colj)[KMAX],
                                    double (*rowj)[KMAX], int* fail) {
  constexpr int PB = KMAX / TD;
  const int tid = threadIdx.x, tx = tid % TD, ty = tid / TD;
  double M[PB][PB], X[PB][PB];
#pragma unroll
  for (int a = 0; a < PB; ++a)
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int i = ty + TD * a, l = tx + TD * b;
      M[a][b] = (i < k && l <= i) ? G[i * ldg + l] + (i == l ? shift : 0.0) : 0.0;
      X[a][b] = (i < k && i == l) ? 1.0 : 0.0;
    }
  if (tid == 0) *fail = 0;
  __syncthreads();
  bool stop = false;
#pragma unroll
  for (int b0 = 0; b0 < PB; ++b0) {
    for (int jj = 0; jj < TD; ++jj) {
      const int j = b0 * TD + jj;
      if (j >= k || stop) break;
      // publish column j of A and row j of X (both unscaled) into buffer j % 2;
      // a thread writes buffer j % 2 again only after the barrier of step
      // j + 1, which every reader of step j has passed
      // (rows of blocks a < b0 lie above row j, columns of blocks b > b0 to the
      // right of column j: the updates below never touch or read them, which the
      // unrolled block indices let the compiler drop)
      const int bf = j & 1;
      if (tx == jj) {
#pragma unroll
        for (int a = b0; a < PB; ++a) colj[bf][ty + TD * a] = M[a][b0];
      }
      if (ty == jj) {
#pragma unroll
        for (int b = 0; b <= b0; ++b) rowj[bf][tx + TD * b] = X[b0][b];
      }
      __syncthreads();
      const double p = colj[bf][j];
      if (!(p > 0.0) || !isfinite(p)) {   // uniform: every thread reads the same p
        stop = true;
        if (tid == 0) *fail = 1;
        break;
      }
      // 1/sqrt(p): hardware estimate and one Newton step; d = p / sqrt(p)
      double id = __builtin_amdgcn_rsq(p);
      id = id * fma(-0.5 * p * id, id, 1.5);
      const double d = p * id;
      double lc[PB], lr[PB], xj[PB];
#pragma unroll
      for (int a = 0; a < PB; ++a) lc[a] = a >= b0 ? colj[bf][ty + TD * a] * id : 0.0;   // L[i][j]
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        lr[b] = b >= b0 ? colj[bf][tx + TD * b] * id : 0.0;                       // L[l][j]
        xj[b] = b <= b0 ? rowj[bf][tx + TD * b] * id : 0.0;                       // X[j][c] / L[j][j]
      }
#pragma unroll
      for (int a = b0; a < PB; ++a) {
        const int i = ty + TD * a;
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          const int l = tx + TD * b;
          if (b >= b0 && b <= a && j < l && l <= i) M[a][b] -= lc[a] * lr[b];
          if (b <= b0 && l <= j && j < i) X[a][b] -= lc[a] * xj[b];
        }
      }
      if (tx == jj) {
#pragma unroll
        for (int a = b0; a < PB; ++a) {
          const int i = ty + TD * a;
          if (i > j) M[a][b0] = lc[a];
          else if (i == j) M[a][b0] = d;
        }
      }
      if (ty == jj) {
#pragma unroll
        for (int b = 0; b <= b0; ++b)
          if (tx + TD * b <= j) X[b0][b] = xj[b];
      }
    }
  }
  __syncthreads();
  if (*fail) return false;
  // R^{-1}[c][i] = X[i][c] for c <= i, 0 below the diagonal
#pragma unroll
  for (int a = 0; a < PB; ++a)
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int i = ty + TD * a, c = tx + TD * b;
      if (i < k && c < k) Rinv[c * ldr + i] = (c <= i) ? X[a][b] : 0.0;
    }
  __syncthreads();   // R^{-1} is read by other threads of the workgroup next
  return true;
}

// Largest |G_il - delta_il| over the k x k matrix, reduced over the workgroup
// (wred: one slot per wave).
__device__ double gram_identity_dev(const double* __restrict__ G, int k, double* wred) {
  double dev = 0.0;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int i = e / k, l = e % k;
    dev = fmax(dev, fabs(G[e] - (i == l ? 1.0 : 0.0)));
  }
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off));
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = dev;
  __syncthreads();
  double mx = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = fmax(mx, wred[w]);
  return mx;
}

// One workgroup factorises G = L L^T and inverts L, then writes
// R^{-1} = L^{-T} (upper, k x k).  TD x TD threads hold both matrices in
// registers, block-cyclically: thread (tx, ty) owns rows i = ty + TD a and
// columns l = tx + TD b (a, b < PB).  Column j (right-looking, pivot
// p = A[j][j], L[i][j] = A[i][j] / sqrt(p), A[i][l] -= L[i][j] L[l][j] for
// j < l <= i) is published through LDS together with row j of X, where X = L^{-1}
// is built by forward elimination on the identity in the same loop
// (X[j][:] /= L[j][j], then X[i][:] -= L[i][j] X[j][:] for i > j).
// attempt 0: first pass, resets the per-orthonormalisation flags.
// attempt 1: second pass; if G is already within 1e-6 of I (the first pass was
//            orthonormal to working precision) it only sets status[3] (skip).
// attempt 2: third pass, only after a shifted factorisation (status[0]).
template <int KMAX, int TD>
__global__ void __launch_bounds__(TD * TD)
cholesky_kernel(const double* __restrict__ G, int k, int64_t rows, double* __restrict__ Rinv,
                int* __restrict__ status, int attempt) {
  constexpr int NW = TD * TD / 64;
  if (attempt == 2 && status[0] == 0) return;
  __shared__ double colj[2][KMAX], rowj[2][KMAX];   // double-buffered: one barrier per column
  __shared__ double wred[NW];
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (attempt == 1 && gram_identity_dev(G, k, wred) <= 1e-6) {   // uniform
    if (tid == 0) status[3] = 1;
    return;
  }
  if (attempt == 0 && tid == 0) {
    status[0] = 0;
    status[3] = 0;
  }
  for (int tryi = 0; tryi < 2; ++tryi) {
    double shift = 0.0;
    if (tryi == 1) {
      double trace = 0.0;
      for (int i = 0; i < k; ++i) trace += G[i * k + i];
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * k + (double)k * (k + 1)) * u * trace;
    }
    if (chol_factor_inverse<KMAX, TD>(G, k, k, shift, Rinv, k, colj, rowj, &fail)) return;
    if (tryi == 0 && tid == 0 && attempt < 2) {
      status[0] = 1;               // enables the third pass (shifted CholeskyQR3)
      atomicAdd(status + 2, 1);    // shifted orthonormalisations since compress
    }
    __syncthreads();
  }
  if (tid == 0) status[1] = 1;
}

// C = op(A) op(B), na x nb (each <= 128) over K <= 128, by the whole 1024-thread
// workgroup on v_mfma_f64_16x16x4_f64: element (i, c) of A is A[i ai + c ac],
// (c, j) of B is B[c bc + j bj], zero outside the ranges.  K is staged into LDS
// in chunks of 32 (A chunk na x 32, B chunk 32 x nb), every load of a chunk in
// flight together and coalesced along whichever stride is 1; wave w accumulates
// the 16 x 16 tiles t = w, w + 16, ... (row-major over the tile grid) over k in
// ascending steps of 4 and hands each to st(ti, tj, d), with D[i][j] in lane
// j + 16 (i % 4), register i / 4.  Called by every thread (it holds barriers).
constexpr int MMC = 32, MAS = MMC + 1, MBS = 128 + 1;
template <typename Store>
__device__ __attribute__((noinline)) void mm_lds_f64(const double* A, int ai, int ac, int na, const double* B, int bc, int bj, int nb,
                           int K, double* As, double* Bs, Store st) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l16 = lane & 15, g4 = lane >> 4;
  const int ntj = (nb + 15) / 16, nt = ((na + 15) / 16) * ntj;
  f64x4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += MMC) {
    double av[4], bv[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int e = tid + 1024 * p;
      const int i = ac == 1 ? e >> 5 : e & 127, c = ac == 1 ? e & 31 : e >> 7;
      av[p] = (i < na && k0 + c < K) ? A[(int64_t)i * ai + (int64_t)(k0 + c) * ac] : 0.0;
      const int jb = bj == 1 ? e & 127 : e >> 5, cb = bj == 1 ? e >> 7 : e & 31;
      bv[p] = (jb < nb && k0 + cb < K) ? B[(int64_t)(k0 + cb) * bc + (int64_t)jb * bj] : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int e = tid + 1024 * p;
      const int i = ac == 1 ? e >> 5 : e & 127, c = ac == 1 ? e & 31 : e >> 7;
      As[i * MAS + c] = av[p];
      const int jb = bj == 1 ? e & 127 : e >> 5, cb = bj == 1 ? e >> 7 : e & 31;
      Bs[cb * MBS + jb] = bv[p];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = wave + 16 * q;
      if (t >= nt) break;   // uniform
      const int ti = t / ntj, tj = t % ntj;
#pragma unroll
      for (int s4 = 0; s4 < MMC / 4; ++s4) {
        const double a = As[(16 * ti + l16) * MAS + 4 * s4 + g4];
        const double b = Bs[(4 * s4 + g4) * MBS + 16 * tj + l16];
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = wave + 16 * q;
    if (t < nt) st(t / ntj, t % ntj, acc[q]);
  }
}

// 128 < k <= 256: the same factorisation by 2 x 2 blocks of 128 (one workgroup
// of 32 x 32 threads).  With G = [G11 G12; G21 G22] and L = [L11 0; L21 L22]:
// L11 from G11 (R11^{-1} = L11^{-T}), L21 = G21 R11^{-1}, L22 from the Schur
// complement S = G22 - L21 L21^T, and
//   R^{-1} = [R11^{-1}, -R11^{-1} L21^T R22^{-1}; 0, R22^{-1}].
// Rinv (k x k) doubles as the scratch: L21 in its lower-left block, S and then
// R11^{-1} L21^T in its upper-right block, the transpose of R12 in the lower-left
// block before it is copied up; the lower-left block is zeroed last.
// The shift of a failed first try applies to the whole diagonal.
__global__ void __launch_bounds__(1024)
cholesky256_kernel(const double* __restrict__ G, int k, int64_t rows, double* __restrict__ Rinv,
                   int* __restrict__ status, int attempt) {
  constexpr int KB = 128, NWV = 16;
  if (attempt == 2 && status[0] == 0) return;
  __shared__ double colj[2][KB], rowj[2][KB];
  __shared__ double wred[NWV];
  __shared__ double mmA[KB * MAS], mmB[MMC * MBS];   // staged operand chunks of the block products
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int k2 = k - KB;
  if (attempt == 1 && gram_identity_dev(G, k, wred) <= 1e-6) {   // uniform
    if (tid == 0) status[3] = 1;
    return;
  }
  if (attempt == 0 && tid == 0) {
    status[0] = 0;
    status[3] = 0;
  }
  double* R11 = Rinv;                    // k x k, ld k
  double* R12 = Rinv + KB;               // KB x k2
  double* R21 = Rinv + (int64_t)KB * k;  // k2 x KB (scratch: L21, then T^T)
  double* R22 = R21 + KB;                // k2 x k2
  for (int tryi = 0; tryi < 2; ++tryi) {
    double shift = 0.0;
    if (tryi == 1) {
      double trace = 0.0;
      for (int i = 0; i < k; ++i) trace += G[i * k + i];
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * k + (double)k * (k + 1)) * u * trace;
    }
    bool ok = chol_factor_inverse<KB, 32>(G, k, KB, shift, R11, k, colj, rowj, &fail);
    if (ok) {
      // L21 = G21 R11^{-1} (k2 x KB) -> lower-left block
      mm_lds_f64(G + (int64_t)KB * k, k, 1, k2, R11, k, 1, KB, KB, mmA, mmB, [&](int ti, int tj, f64x4 d) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int i = 16 * ti + 4 * x + g4, j = 16 * tj + l16;
          if (i < k2) R21[i * k + j] = d[x];
        }
      });
      __syncthreads();
      // S = G22 + shift I - L21 L21^T (k2 x k2) -> upper-right block
      mm_lds_f64(R21, k, 1, k2, R21, 1, k, k2, KB, mmA, mmB, [&](int ti, int tj, f64x4 d) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int i = 16 * ti + 4 * x + g4, j = 16 * tj + l16;
          if (i < k2 && j < k2)
            R12[i * k + j] = G[(int64_t)(KB + i) * k + KB + j] + (i == j ? shift : 0.0) - d[x];
        }
      });
      __syncthreads();
      ok = chol_factor_inverse<KB, 32>(R12, k, k2, 0.0, R22, k, colj, rowj, &fail);
    }
    if (ok) {
      // U = R11^{-1} L21^T (KB x k2) -> upper-right block (S is consumed)
      mm_lds_f64(R11, k, 1, KB, R21, 1, k, k2, KB, mmA, mmB, [&](int ti, int tj, f64x4 d) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int i = 16 * ti + 4 * x + g4, j = 16 * tj + l16;
          if (j < k2) R12[i * k + j] = d[x];
        }
      });
      __syncthreads();
      // R12 = -U R22^{-1}, stored transposed over L21 (lower-left block, dead now)
      mm_lds_f64(R12, k, 1, KB, R22, k, 1, k2, k2, mmA, mmB, [&](int ti, int tj, f64x4 d) {
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          const int i = 16 * ti + 4 * x + g4, j = 16 * tj + l16;
          if (j < k2) R21[j * k + i] = -d[x];
        }
      });
      __syncthreads();
      for (int e = tid; e < k2 * KB; e += 1024) {   // back into the upper-right block, then zeros below
        const int j = e / KB, i = e % KB;
        R12[i * k + j] = R21[j * k + i];
      }
      __syncthreads();
      for (int e = tid; e < k2 * KB; e += 1024) R21[(e / KB) * k + e % KB] = 0.0;
      return;
    }
    if (tryi == 0 && tid == 0 && attempt < 2) {
      status[0] = 1;               // enables the third pass (shifted CholeskyQR3)
      atomicAdd(status + 2, 1);    // shifted orthonormalisations since compress
    }
    __syncthreads();
  }
  if (tid == 0) status[1] = 1;
}

// 64-bit value of lane `src` (uniform result).
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A_ij -= L_ip L_jp^T for 16 x 16 blocks of the LDS matrix (row stride LD):
// one wave, four v_mfma_f64_16x16x4_f64 steps over the 16 columns of panel p.
// A operand: lane (r, g) = (lane % 16, lane / 16) holds L[16i + r][16p + 4s + g];
// B operand: L[16j + r][16p + 4s + g]; D[row][col] in lane col + 16 (row % 4),
// register row / 4.
template <int LD>
__device__ __forceinline__ void chol_block_update(double* As, int i, int j, int p, int r, int g) {
  f64x4 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = As[(16 * i + 4 * q + g) * LD + 16 * j + r];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double a = -As[(16 * i + r) * LD + 16 * p + 4 * s + g];
    const double b = As[(16 * j + r) * LD + 16 * p + 4 * s + g];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) As[(16 * i + 4 * q + g) * LD + 16 * j + r] = acc[q];
}

// The value of lane (lane % 16) + 16 GO in every lane: rows of 16 lanes are
// exchanged by v_permlane16_swap (rows 0 1 2 3 of x become 0 0 2 2 and 1 1 3 3)
// and v_permlane32_swap (0 1 0 1 and 2 3 2 3), no LDS round trip.
template <int GO>
__device__ __forceinline__ double lane_group_bcast(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  uint32_t h[2] = {(uint32_t)u, (uint32_t)(u >> 32)};
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const auto a = __builtin_amdgcn_permlane16_swap(h[i], h[i], false, false);
    const uint32_t y = (GO & 1) ? a[1] : a[0];
    const auto b = __builtin_amdgcn_permlane32_swap(y, y, false, false);
    h[i] = (GO & 2) ? b[1] : b[0];
  }
  return __builtin_bit_cast(double, ((uint64_t)h[1] << 32) | h[0]);
}

// D = L_bb^{-1} for one 16 x 16 diagonal block (dense, zeros above the
// diagonal), by forward substitution for column c = lane % 16.  The four lane
// groups g = lane / 16 share the column: lane (c, g) holds rows 4 q + g (the
// MFMA output layout, q = 0..3).  Step t: the group holding row t finalises
// x_t (the division is the product with 1 / L[t][t]), passes it to the other
// groups (lane_group_bcast), and every row r > t takes x_r -= L[r][t] x_t.
// The entries of L are read from LDS one step ahead; an opaque zero added to
// their indices keeps the reads of a step from being hoisted above the step
// before it, so only a few are live at a time.
template <int DL>
__device__ __forceinline__ void chol_diag_inverse(const double* Ld, const double* inv_diag, double* D, int c,
                                                  int g) {
  double x[4], ln[4], dn;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[q] = (4 * q + g == c) ? 1.0 : 0.0;
    ln[q] = Ld[(4 * q + g) * 16];
  }
  dn = inv_diag[0];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    double lc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) lc[q] = ln[q];
    const double dc = dn;
    if (t < 15) {
      int z = 0;
      asm volatile("" : "+s"(z));
#pragma unroll
      for (int q = 0; q < 4; ++q) ln[q] = (4 * q + 3 > t + 1) ? Ld[(4 * q + g) * 16 + t + 1 + z] : 0.0;
      dn = inv_diag[t + 1 + z];
    }
    const int qt = t >> 2;
    x[qt] = (g == (t & 3)) ? x[qt] * dc : x[qt];
    double v;
    switch (t & 3) {
      case 0: v = lane_group_bcast<0>(x[qt]); break;
      case 1: v = lane_group_bcast<1>(x[qt]); break;
      case 2: v = lane_group_bcast<2>(x[qt]); break;
      default: v = lane_group_bcast<3>(x[qt]); break;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (4 * q + 3 <= t) continue;   // every row of this register is <= t
      const double nx = fma(-lc[q], v, x[q]);
      x[q] = (4 * q + g > t) ? nx : x[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) D[(4 * q + g) * DL + c] = x[q];
}

// Blocked form of the same factorisation for k <= 64 (four waves).  G is staged
// in LDS, padded to Kp = 16 ceil(k / 16) with the identity (the padding factors
// to itself and leaves the leading k x k block unchanged).  Right-looking over
// 16-column panels:
//  - wave 0 factors panel b over its whole height, one row per lane, with no
//    barrier or LDS round trip inside the panel.  Column t: with p its pivot and
//    v the column, the later columns u of the panel take a[u] -= (v / p) v[u],
//    where v[u] (the entry in the row of column u) is read from its lane before
//    the pivot is known; the column itself becomes v / sqrt(p).  The next pivot
//    is formed from the same uniform values (the operation its lane performs),
//    so the serial chain per column is 1/sqrt(p) (hardware estimate and one
//    Newton step, as above), 1/p and one FMA;
//  - the trailing update runs on FP64 MFMA with one step of lookahead: right
//    after panel b only column block b + 1 is updated; the other trailing blocks
//    take panel b's update while wave 0 factors panel b + 1.  The idle waves also
//    invert the diagonal block of the previous panel then.
// L^{-1} = X is formed blockwise: wave w builds column block w,
// X_ww = L_ww^{-1} = D_w, X_iw = -D_i (sum_{w <= c < i} L_ic X_cw); the last row
// block waits only for the last diagonal inverse, which another wave forms
// meanwhile.  Attempts, shift and status flags as in cholesky_kernel.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
cholesky_blocked_kernel(const double* __restrict__ G, int k, int64_t rows, double* __restrict__ Rinv,
                        int* __restrict__ status, int attempt) {
  if (attempt == 2 && status[0] == 0) return;
  constexpr int LD = 65, DL = 17;
  __shared__ double As[64 * LD];
  __shared__ __align__(16) double Ldg[4 * 256];   // diagonal blocks L_bb, dense, zeros above
  __shared__ double Ds[64 * DL];                  // D_b in rows 16 b .. 16 b + 15
  __shared__ double idv[64];                      // 1 / L[j][j]
  __shared__ __align__(16) double colb[128];      // the current panel column, two buffers
  __shared__ double wred[4];
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nb = (k + 15) >> 4, Kp = 16 * nb;

  if (attempt == 1) {
    double dev = 0.0;
    // unconditional loads from clamped (in-bounds) indices, all in flight together
    double gv[16];
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int e = tid + 256 * p, i = e >> 6, l = e & 63;
      gv[p] = G[min(i, k - 1) * k + min(l, k - 1)];
    }
#pragma unroll
    for (int p = 0; p < 16; ++p) asm volatile("" : "+v"(gv[p]));
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int e = tid + 256 * p, i = e >> 6, l = e & 63;
      if (i < k && l < k) dev = fmax(dev, fabs(gv[p] - (i == l ? 1.0 : 0.0)));
    }
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off));
    if (lane == 0) wred[wave] = dev;
    __syncthreads();
    const double mx = fmax(fmax(wred[0], wred[1]), fmax(wred[2], wred[3]));
    if (mx <= 1e-6) {                     // uniform
      if (tid == 0) status[3] = 1;
      return;
    }
  }
  if (attempt == 0 && tid == 0) {
    status[0] = 0;
    status[3] = 0;
  }

  for (int tryi = 0; tryi < 2; ++tryi) {
    double shift = 0.0;
    if (tryi == 1) {
      double trace = 0.0;
      for (int i = 0; i < k; ++i) trace += G[i * k + i];
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * k + (double)k * (k + 1)) * u * trace;
    }
    // the whole 64 x 64 tile from clamped (in-bounds) indices; the empty asm
    // consumes every loaded value, so the loads are not sunk into the selects
    // and all sixteen are in flight together.  Opaque copies of the base and
    // of the thread index keep the address arithmetic inside this loop (hoisted
    // out of it, it would stay live through the factorisation).
    {
      const double* Gp = G;
      int te = tid;
      asm volatile("" : "+s"(Gp), "+v"(te));
      double gv[16];
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int e = te + 256 * p, i = e >> 6, l = e & 63;
        gv[p] = Gp[min(i, k - 1) * k + min(l, k - 1)];
      }
#pragma unroll
      for (int p = 0; p < 16; ++p) asm volatile("" : "+v"(gv[p]));
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int e = te + 256 * p, i = e >> 6, l = e & 63;
        As[i * LD + l] = (i < k && l < k) ? gv[p] + (i == l ? shift : 0.0) : (i == l ? 1.0 : 0.0);
      }
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
      if (wave == 0) {
        const int c0 = 16 * b;
        double a[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) a[t] = (lane < Kp && lane >= c0 + t) ? As[lane * LD + c0 + t] : 0.0;
        // lanes above the diagonal only change entries above it, which are never read
        // Software-pipelined: the estimate for the next pivot is issued before
        // this column's updates, whose issue hides its latency.  The two values
        // the next pivot needs are read from their lanes (readlane); the rest of
        // the column goes through LDS (one store, uniform-address loads).
        // Scheduling fences keep that order.
        double idl = 0.0;
        bool bad = false;
        double p = readlane_f64(a[0], c0);
        double r0 = __builtin_amdgcn_rsq(p);
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          double* cb = colb + 64 * (t & 1);
          cb[lane] = a[t];
          double w[16];
          if (t < 15) w[t + 1] = readlane_f64(a[t], c0 + t + 1);
#pragma unroll
          for (int u = t + 2; u < 16; ++u) w[u] = cb[c0 + u];
          const double xn = readlane_f64(a[t < 15 ? t + 1 : 15], c0 + (t < 15 ? t + 1 : 15));
          __builtin_amdgcn_sched_barrier(0);
          bad = bad | !(p > 0.0) | !isfinite(p);
          const double id = r0 * fma(-0.5 * p * r0, r0, 1.5);
          const double rp = id * id;
          if (t < 15) {
            p = fma(-(w[t + 1] * rp), w[t + 1], xn);
            r0 = __builtin_amdgcn_rsq(p);
          }
          __builtin_amdgcn_sched_barrier(0);
          const double m = a[t] * rp;
          a[t] *= id;
          idl = (lane == c0 + t) ? id : idl;
#pragma unroll
          for (int u = t + 1; u < 16; ++u) a[u] = fma(-m, w[u], a[u]);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (bad) {
          if (lane == 0) fail = 1;
        } else {
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (lane < Kp && lane >= c0 + t) As[lane * LD + c0 + t] = a[t];
          if (lane >= c0 && lane < c0 + 16) {
            const int r = lane - c0;
            idv[lane] = idl;
#pragma unroll
            for (int t = 0; t < 16; ++t) Ldg[256 * b + 16 * r + t] = (t <= r) ? a[t] : 0.0;
          }
        }
      } else if (b >= 1) {
        // the rest of panel b - 1's trailing update: blocks (i, j), b < j <= i
        int q = 0;
        for (int j = b + 1; j < nb; ++j)
          for (int i = j; i < nb; ++i, ++q)
            if (q % 3 == wave - 1) chol_block_update<LD>(As, i, j, b - 1, lr, lg);
        if (wave == 1 + (b - 1) % 3)
          chol_diag_inverse<DL>(Ldg + 256 * (b - 1), idv + 16 * (b - 1), Ds + 16 * (b - 1) * DL, lr, lg);
      }
      __syncthreads();
      if (fail) break;
      // column block b + 1 takes panel b's update
      if (wave < nb - b - 1) chol_block_update<LD>(As, b + 1 + wave, b + 1, b, lr, lg);
      __syncthreads();
    }
    if (!fail) break;
    if (tryi == 0 && tid == 0 && attempt < 2) {
      status[0] = 1;               // enables the third pass (shifted CholeskyQR3)
      atomicAdd(status + 2, 1);    // shifted orthonormalisations since compress
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) status[1] = 1;
    return;
  }

  // column blocks w < nb - 1 up to the last row block, whose D wave 3 forms meanwhile
  const int last = nb - 1;
  f64x4 Xr[4], T = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i) Xr[i] = (f64x4){0.0, 0.0, 0.0, 0.0};
  if (wave == 3) chol_diag_inverse<DL>(Ldg + 256 * last, idv + 16 * last, Ds + 16 * last * DL, lr, lg);
  if (wave < last) {
    const int w = wave;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i == w)
#pragma unroll
        for (int q = 0; q < 4; ++q) Xr[i][q] = Ds[(16 * w + 4 * q + lg) * DL + lr];
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      if (i <= w || i >= last) continue;   // uniform
      f64x4 U = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < i; ++c) {
        if (c < w) continue;
#pragma unroll
        for (int s = 0; s < 4; ++s)
          U = __builtin_amdgcn_mfma_f64_16x16x4f64(As[(16 * i + lr) * LD + 16 * c + 4 * s + lg], Xr[c][s], U,
                                                   0, 0, 0);
      }
      f64x4 Y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        Y = __builtin_amdgcn_mfma_f64_16x16x4f64(-Ds[(16 * i + lr) * DL + 4 * s + lg], U[s], Y, 0, 0, 0);
      Xr[i] = Y;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c < w || c >= last) continue;
#pragma unroll
      for (int s = 0; s < 4; ++s)
        T = __builtin_amdgcn_mfma_f64_16x16x4f64(As[(16 * last + lr) * LD + 16 * c + 4 * s + lg], Xr[c][s], T,
                                                 0, 0, 0);
    }
  }
  __syncthreads();
  if (wave < nb) {
    const int w = wave;
    f64x4 Y = {0.0, 0.0, 0.0, 0.0};
    if (w == last) {
#pragma unroll
      for (int q = 0; q < 4; ++q) Y[q] = Ds[(16 * w + 4 * q + lg) * DL + lr];
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        Y = __builtin_amdgcn_mfma_f64_16x16x4f64(-Ds[(16 * last + lr) * DL + 4 * s + lg], T[s], Y, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i == last) Xr[i] = Y;
    // R^{-1}[c][i] = X[i][c] for c <= i, 0 below the diagonal
    const int cg = 16 * w + lr;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i >= nb) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ig = 16 * i + 4 * q + lg;
        if (ig < k && cg < k) Rinv[cg * k + ig] = (cg <= ig) ? Xr[i][q] : 0.0;
      }
    }
  }
}

// Q = Y R^{-1} in place on FP64 MFMA (v_mfma_f64_16x16x4_f64): a workgroup owns
// 64 rows (16 per wave) and all k columns; the tile is read into LDS before any
// write, so rows of other workgroups are never touched.  The tile is staged with
// batched float4 loads (ldy % 4 == 0); R^{-1} is staged in LDS too (row stride
// KMAX + 2 doubles).  (Wider bases: apply_rinv_wide_kernel.)
// BT = true: instead of Y, write the transposed BF16 copy Bt (k x ldbt, nearest
// even; the operand of the next low-precision product): the tile of Q goes
// through LDS (row stride KMAX + 2 halves) and out as 16-byte chunks of Bt's
// rows.  The grid then covers all ldbt columns, rows past `rows` giving zeros.
template <int KMAX, bool BT>
__global__ void __launch_bounds__(256)
apply_rinv_kernel(float* __restrict__ Y, int64_t ldy, int64_t rows, int k,
                  const double* __restrict__ Rinv, const int* __restrict__ status, int attempt,
                  uint16_t* __restrict__ Bt, int64_t ldbt) {
  if (status[1] != 0) return;
  if (attempt == 1 && status[3] != 0) return;   // second pass not needed
  if (attempt == 2 && status[0] == 0) return;
  constexpr int NT = KMAX / 16;
  constexpr bool RS = KMAX <= 64;
  constexpr int V4 = 64 * KMAX / 4 / 256;       // float4 per thread
  constexpr int RST = KMAX + 2;
  __shared__ float Ys[64][KMAX + 4];
  __shared__ double Rs[RS ? KMAX : 1][RS ? RST : 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  f32x4 v[V4];
#pragma unroll
  for (int p = 0; p < V4; ++p) {
    const int e = tid + 256 * p, i = e / (KMAX / 4), c = 4 * (e % (KMAX / 4));
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    v[p] = (row0 + i < rows && c < k) ? *(const f32x4*)(Y + (row0 + i) * ldy + c) : z;
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (c + d >= k) v[p][d] = 0.f;          // a partial last group (k % 4 != 0)
  }
  if (RS) {
    for (int e = tid; e < KMAX * KMAX; e += 256) {
      const int a = e / KMAX, b = e % KMAX;
      Rs[a][b] = (a < k && b < k) ? Rinv[a * k + b] : 0.0;
    }
  }
#pragma unroll
  for (int p = 0; p < V4; ++p) {
    const int e = tid + 256 * p, i = e / (KMAX / 4), c = 4 * (e % (KMAX / 4));
    *(f32x4*)(&Ys[i][c]) = v[p];
  }
  __syncthreads();
  f64x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (f64x4){0, 0, 0, 0};
  const int ar = wave * 16 + (lane & 15);
  for (int s = 0; s < KMAX / 4; ++s) {
    if (4 * s >= k) break;
    const int kr = 4 * s + (lane >> 4);
    const double a = (double)Ys[ar][kr];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (s >= 4 * (t + 1)) continue;   // R^{-1} is upper triangular: rows >= 16 (t + 1) of block t are 0
      const int j = t * 16 + (lane & 15);
      double b;
      if (RS) b = Rs[kr][j];
      else b = (kr < k && j < k) ? Rinv[kr * k + j] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  // D[i][j] in lane j + 16 (i % 4), register i / 4
  if (!BT) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = row0 + wave * 16 + 4 * q + (lane >> 4);
        const int j = t * 16 + (lane & 15);
        if (gi < rows && j < k) Y[gi * ldy + j] = (float)acc[t][q];
      }
  } else {
    // Tb[j][i] = bf16(Q[row0 + i][j]) in the (now free) Ys tile; row stride 66 halves
    constexpr int TS = 66;
    static_assert(KMAX * TS * 2 <= 64 * (KMAX + 4) * 4, "Tb must fit in Ys");
    uint16_t* Tb = reinterpret_cast<uint16_t*>(&Ys[0][0]);
    __syncthreads();   // every wave is done reading Ys
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = wave * 16 + 4 * q + (lane >> 4), j = t * 16 + (lane & 15);
        float v = (row0 + i < rows) ? (float)acc[t][q] : 0.f;
        // round to FP32 first, then to BF16, as the unfused path (FP32 basis, then
        // its BF16 copy) does; without the barrier the two roundings merge into one
        asm volatile("" : "+v"(v));
        Tb[j * TS + i] = __builtin_bit_cast(uint16_t, (__bf16)v);
      }
    __syncthreads();
    for (int e = tid; e < k * 8; e += 256) {       // row j of Bt: 64 halves = 8 chunks of 16 bytes
      const int j = e >> 3, c = e & 7;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(Tb + j * TS + 8 * c);
      const i32x4 o = {(int)src[0], (int)src[1], (int)src[2], (int)src[3]};
      *(i32x4*)(Bt + j * ldbt + row0 + 8 * c) = o;
    }
  }
}

// Q = Y R^{-1} in place for wide bases (64 < k <= KMAX): a workgroup owns 64
// rows and all k columns (the tile is read into LDS before any write, 66 KB:
// two workgroups per CU).  Each wave owns four (KMAX 256) or two (KMAX 128)
// 16-column blocks of the output, {w, 7 - w, 8 + w, 15 - w}, which balances
// the work of the upper-triangular R^{-1} over the waves, and all 64 rows:
// v_mfma_f64_16x16x4_f64 with A[i][kk] = Y[i][kk] from LDS and B[kk][j] =
// R^{-1}[kk][j] read by the wave straight from global memory (no other wave
// uses its columns; R^{-1} stays in L2), two k-steps ahead in registers.
// D[i][j] lies in lane j + 16 (i % 4), register i / 4.  A block b only takes
// the k-steps 4 s <= 16 b + 15 (R^{-1} is zero below its diagonal).  Loads are
// unconditional from clamped addresses, values outside k x k zeroed after.
template <int KMAX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))   // two workgroups per CU
apply_rinv_wide_kernel(float* __restrict__ Y, int64_t ldy, int64_t rows, int k, const double* __restrict__ Rinv,
                       const int* __restrict__ status, int attempt) {
  if (status[1] != 0) return;
  if (attempt == 1 && status[3] != 0) return;   // second pass not needed
  if (attempt == 2 && status[0] == 0) return;
  constexpr int YROW = KMAX + 4;
  constexpr int NBW = KMAX / 64;                 // 16-column blocks per wave
  constexpr int V4 = 64 * KMAX / 4 / 256;        // float4 of the Y tile per thread
  constexpr int SC = 2;                          // k-steps per chunk (8 rows of R^{-1})
  __shared__ __attribute__((aligned(16))) float Ys[64 * YROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  {
    f32x4 yv[V4];
#pragma unroll
    for (int p = 0; p < V4; ++p) {
      const int e = tid + 256 * p, i = e / (KMAX / 4), c = 4 * (e % (KMAX / 4));
      yv[p] = *(const f32x4*)(Y + ((row0 + i < rows && c < k) ? (row0 + i) * ldy + c : 0));
    }
#pragma unroll
    for (int p = 0; p < V4; ++p) {
      const int e = tid + 256 * p, i = e / (KMAX / 4), c = 4 * (e % (KMAX / 4));
      f32x4 v;
#pragma unroll
      for (int d = 0; d < 4; ++d) v[d] = (row0 + i < rows && c + d < k) ? yv[p][d] : 0.f;   // k % 4 != 0
      *(f32x4*)(Ys + i * YROW + c) = v;
    }
  }
  // this wave's blocks: b = w, 7 - w (and 8 + w, 15 - w)
  int blk[NBW];
  blk[0] = wave;
  blk[1] = 7 - wave;
  if (NBW == 4) {
    blk[NBW > 2 ? 2 : 0] = 8 + wave;
    blk[NBW > 3 ? 3 : 0] = 15 - wave;
  }
  f64x4 acc[4][NBW];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
  // B fragments of k-steps s0, s0 + 1: lane holds R^{-1}[4 s + g4][16 blk + l16]
  double bq0[SC][NBW], bq1[SC][NBW];
  auto loadb = [&](double (*bq)[NBW], int s0) {
#pragma unroll
    for (int u = 0; u < SC; ++u)
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        const int kr = 4 * (s0 + u) + g4, j = 16 * blk[b] + l16;
        bq[u][b] = Rinv[(kr < k && j < k) ? (int64_t)kr * k + j : 0];
      }
  };
  auto chunk = [&](double (*bq)[NBW], int s0) {
#pragma unroll
    for (int u = 0; u < SC; ++u) {
      const int s = s0 + u;
      double av[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = (double)Ys[(16 * a + l16) * YROW + 4 * s + g4];
#pragma unroll
      for (int b = 0; b < NBW; ++b) {
        if (s > 4 * blk[b] + 3) continue;        // rows below block b's diagonal (uniform)
        const int kr = 4 * s + g4, j = 16 * blk[b] + l16;
        const double bv = (kr < k && j < k) ? bq[u][b] : 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv, acc[a][b], 0, 0, 0);
      }
    }
  };
  // the last k-step any block of this wave needs
  int smax = 0;
#pragma unroll
  for (int b = 0; b < NBW; ++b) smax = max(smax, 4 * blk[b] + 4);
  loadb(bq0, 0);
  __syncthreads();                               // the Y tile is in LDS
  for (int s0 = 0; s0 < smax; s0 += 2 * SC) {
    if (s0 + SC < smax) loadb(bq1, s0 + SC);
    __builtin_amdgcn_sched_barrier(0);           // the next chunk's loads stay ahead of the MFMAs
    chunk(bq0, s0);
    if (s0 + SC < smax) {
      if (s0 + 2 * SC < smax) loadb(bq0, s0 + 2 * SC);
      __builtin_amdgcn_sched_barrier(0);
      chunk(bq1, s0 + SC);
    }
  }
  __syncthreads();                               // every wave has read the whole tile
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NBW; ++b)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t gi = row0 + 16 * a + 4 * x + g4;
        const int j = 16 * blk[b] + l16;
        if (gi < rows && j < k) Y[gi * ldy + j] = (float)acc[a][b][x];
      }
}

}  // namespace

int gram_pick_splits(int64_t rows, int k) {
  if (k > 128) {
    // three blocks per split, two workgroups resident per CU (LDS): 170 splits
    // give 510 workgroups, two per CU in one wave of residency (with 128 splits,
    // 384 workgroups left half the CUs with twice the rows of the others);
    // partials 170 k^2 FP64 (89 MB at k = 256)
    int64_t s = std::min<int64_t>(170, ceil_div(rows, 64));
    return (int)(s < 1 ? 1 : s);
  }
  // 256 rows per split, or down to 64 rows per split so that short bases still
  // spread over 256 workgroups; partials capped at 32 MB
  int64_t s = ceil_div(rows, 256);
  if (s < 256) s = std::min<int64_t>(256, ceil_div(rows, 64));
  const int64_t cap = (32ll << 20) / ((int64_t)k * k * 8);
  if (s > cap) s = cap;
  if (s > 1024) s = 1024;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t launch_gram_f64(const float* Y, int64_t ldy, int64_t rows, int k, double* part,
                           int splits, double* G, const int* skip_flag, hipStream_t st) {
  const int nb = (k + GT - 1) / GT;
  const int64_t rchunk = round_up(ceil_div(rows, splits), GROWS);
  if (k > 128 && k <= 256)
    hipLaunchKernelGGL(gram_wide_kernel, dim3(3, splits), dim3(256), 0, st, Y, ldy, rows, k, rchunk, part,
                       skip_flag);
  else
    hipLaunchKernelGGL(gram_f64_kernel, dim3(nb * nb, splits), dim3(256), 0, st, Y, ldy, rows, k,
                       rchunk, part, skip_flag, nullptr, 0, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials_f64(part, splits, (int64_t)k * k, G, skip_flag, st);
}

namespace {
__global__ void __launch_bounds__(256)
f64_to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
    b[e] = (float)a[e];
}
}  // namespace

hipError_t launch_atb_f32out(const float* A, int64_t lda, int ka, const float* B, int64_t ldb, int kb,
                             int64_t rows, double* part, int splits, double* C64, float* C, hipStream_t st) {
  const int nbi = (ka + GT - 1) / GT, nbj = (kb + GT - 1) / GT;
  const int64_t rchunk = round_up(ceil_div(rows, splits), GROWS);
  hipLaunchKernelGGL(gram_f64_kernel, dim3(nbi * nbj, splits), dim3(256), 0, st, A, lda, rows, ka, rchunk, part,
                     nullptr, B, ldb, kb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_sum_partials_f64(part, splits, (int64_t)ka * kb, C64, nullptr, st))) return e;
  const int64_t cnt = (int64_t)ka * kb;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, C64, C, cnt);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* G, int k, int64_t rows, double* Rinv, int* status,
                           int attempt, hipStream_t st) {
  if (k <= 64)
    hipLaunchKernelGGL(cholesky_blocked_kernel, dim3(1), dim3(256), 0, st, G, k, rows, Rinv, status,
                       attempt);
  else if (k <= 128)
    hipLaunchKernelGGL((cholesky_kernel<128, 32>), dim3(1), dim3(1024), 0, st, G, k, rows, Rinv,
                       status, attempt);
  else if (k <= 256)
    hipLaunchKernelGGL(cholesky256_kernel, dim3(1), dim3(1024), 0, st, G, k, rows, Rinv, status, attempt);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_apply_rinv(float* Y, int64_t ldy, int64_t rows, int k, const double* Rinv,
                             const int* status, int attempt, hipStream_t st, uint16_t* Bt, int64_t ldbt) {
  if (Bt) {   // transposed BF16 operand instead of Y: the grid covers ldbt columns (ldbt % 64 == 0)
    if (k > 64 || ldbt % 64 || ldbt < rows || ((uintptr_t)Bt & 15)) return hipErrorInvalidValue;
    const unsigned g = (unsigned)(ldbt / 64);
    if (g == 0) return hipSuccess;
    if (k <= 32)
      hipLaunchKernelGGL((apply_rinv_kernel<32, true>), dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                         attempt, Bt, ldbt);
    else
      hipLaunchKernelGGL((apply_rinv_kernel<64, true>), dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                         attempt, Bt, ldbt);
    return hipGetLastError();
  }
  const unsigned g = (unsigned)ceil_div(rows, 64);
  if (g == 0) return hipSuccess;
  if (k <= 32)
    hipLaunchKernelGGL((apply_rinv_kernel<32, false>), dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt, nullptr, 0);
  else if (k <= 64)
    hipLaunchKernelGGL((apply_rinv_kernel<64, false>), dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt, nullptr, 0);
  else if (k <= 128)
    hipLaunchKernelGGL(apply_rinv_wide_kernel<128>, dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt);
  else if (k <= 256)
    hipLaunchKernelGGL(apply_rinv_wide_kernel<256>, dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
