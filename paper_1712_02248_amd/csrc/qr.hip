// Tall-skinny QR of a sketch Y (rows x k, FP32) by CholeskyQR in FP64:
//   G = Y^T Y (FP64 MFMA, split over rows), G = R^T R (Cholesky), Q = Y R^{-1}
// (R^{-1} formed with the factorisation; Y R^{-1} on FP64 MFMA, written back
// as FP32 in place).
// CholeskyQR2 runs this twice.  On a non-positive or non-finite pivot the
// factorisation restarts with the shift s = 11 (rows k + k(k+1)) u tr(G)
// (shifted CholeskyQR, Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
// SIAM J. Sci. Comput. 2020), and a third pass is enabled (shifted CholeskyQR3).
//
// status[0]: 1 if the first pass needed the shift;  status[1]: 1 if a pass
// failed even with the shift (the factor is then unusable).
#include "common.h"

namespace {

constexpr int GT = 64;        // Gram output block (GT x GT) per workgroup
constexpr int GROWS = 64;     // rows staged per chunk

// part[s] = Y[rows of split s]^T Y[rows of split s] restricted to the output
// block (bi, bj).  f64 16x16x4 MFMA: A[i][kk] = Y[kk][i], B[kk][j] = Y[kk][j];
// D[i][j] sits in lane j + 16 (i % 4), register i / 4.
__global__ void __launch_bounds__(256)
gram_f64_kernel(const float* __restrict__ Y, int64_t ldy, int64_t rows, int k, int64_t rchunk,
                double* __restrict__ part, const int* __restrict__ skip_flag) {
  if (skip_flag && skip_flag[0] == 0) return;
  __shared__ float Yi[GROWS][GT + 1];
  __shared__ float Yj[GROWS][GT + 1];
  const int nb = (k + GT - 1) / GT;
  const int bi = blockIdx.x / nb, bj = blockIdx.x % nb;
  const int64_t r0 = (int64_t)blockIdx.y * rchunk;
  const int64_t r1 = (r0 + rchunk < rows) ? r0 + rchunk : rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  f64x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = (f64x4){0, 0, 0, 0};

  for (int64_t c0 = r0; c0 < r1; c0 += GROWS) {
    for (int e = tid; e < GROWS * GT; e += 256) {
      const int rr = e / GT, cc = e % GT;
      const int64_t gr = c0 + rr;
      const int gi = bi * GT + cc, gj = bj * GT + cc;
      Yi[rr][cc] = (gr < r1 && gi < k) ? Y[gr * ldy + gi] : 0.f;
      Yj[rr][cc] = (gr < r1 && gj < k) ? Y[gr * ldy + gj] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < GROWS; kk += 4) {
      const int rr = kk + (lane >> 4);
      const double a = (double)Yi[rr][wave * 16 + (lane & 15)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double b = (double)Yj[rr][t * 16 + (lane & 15)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.y * k * k;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = bi * GT + wave * 16 + 4 * q + (lane >> 4);
      const int j = bj * GT + t * 16 + (lane & 15);
      if (i < k && j < k) P[(int64_t)i * k + j] = acc[t][q];
    }
}

// One workgroup: sum the split partials (fixed order) into LDS, factorise
// G = L L^T and invert L, then write R^{-1} = L^{-T} (upper, k x k).
// Both live in one k x k LDS array M: the lower triangle holds A -> L
// (right-looking, column j: pivot p = A[j][j], L[i][j] = A[i][j]/sqrt(p),
// A[i][l] -= L[i][j] L[l][j] for j < l <= i), the strict upper triangle holds
// X = L^{-1} transposed (M[c][i] = X[i][c], c < i) and Xd its diagonal.  X is
// built in the same column loop by forward elimination on the identity:
// X[j][:] /= L[j][j], then X[i][:] -= L[i][j] X[j][:] for i > j.
template <int KMAX>
__global__ void __launch_bounds__(1024)
cholesky_kernel(const double* __restrict__ part, int splits, int k, int64_t rows,
                double* __restrict__ Rinv, int* __restrict__ status, int attempt) {
  if (attempt == 2 && status[0] == 0) return;   // third pass only after a shift
  __shared__ double M[KMAX * KMAX];
  __shared__ double Xd[KMAX];
  __shared__ double trace;
  __shared__ int fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int kk = k * k;

  for (int tryi = 0; tryi < 2; ++tryi) {
    double shift = 0.0;
    if (tryi == 1) {
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * k + (double)k * (k + 1)) * u * trace;
    }
    for (int e = tid; e < kk; e += nt) {
      const int i = e / k, l = e % k;
      double v = 0.0;
      if (l <= i) {
        for (int z = 0; z < splits; ++z) v += part[(int64_t)z * kk + e];
        if (i == l) v += shift;
      }
      M[e] = v;   // strict upper triangle: X = I off the diagonal
    }
    for (int i = tid; i < k; i += nt) Xd[i] = 1.0;
    if (tid == 0) fail = 0;
    __syncthreads();
    if (tryi == 0 && tid == 0) {
      double t = 0.0;
      for (int i = 0; i < k; ++i) t += M[i * k + i];
      trace = t;
    }
    for (int j = 0; j < k; ++j) {
      const double p = M[j * k + j];
      if (!(p > 0.0) || !isfinite(p)) {   // uniform: every thread reads the same p
        if (tid == 0) fail = 1;
        break;
      }
      const double d = sqrt(p), id = 1.0 / d;
      __syncthreads();                     // everyone has read p before it changes
      // phase 1: scale column j of L and row j of X
      for (int i = j + 1 + tid; i < k; i += nt) M[i * k + j] *= id;
      for (int c = tid; c < j; c += nt) M[c * k + j] *= id;   // X[j][c], c < j
      if (tid == 0) {
        M[j * k + j] = d;
        Xd[j] = Xd[j] * id;
      }
      __syncthreads();
      // phase 2: trailing update of A and elimination in X
      const int mt = k - j - 1;
      for (int e = tid; e < mt * mt; e += nt) {
        const int i = j + 1 + e / mt, l = j + 1 + e % mt;
        if (l <= i) M[i * k + l] -= M[i * k + j] * M[l * k + j];
      }
      const int w = j + 1;
      for (int e = tid; e < mt * w; e += nt) {
        const int i = j + 1 + e / w, c = e % w;
        const double xjc = (c == j) ? Xd[j] : M[c * k + j];
        M[c * k + i] -= M[i * k + j] * xjc;   // X[i][c]
      }
      __syncthreads();
    }
    __syncthreads();
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
  // R^{-1}[c][i] = X[i][c]: c < i from the upper triangle, c == i from Xd.
  for (int e = tid; e < kk; e += nt) {
    const int c = e / k, i = e % k;
    Rinv[e] = (c < i) ? M[c * k + i] : (c == i ? Xd[i] : 0.0);
  }
}

// Q = Y R^{-1} in place on FP64 MFMA (v_mfma_f64_16x16x4_f64): a workgroup owns
// 64 rows (16 per wave) and all k columns; the tile is read into LDS before any
// write, so rows of other workgroups are never touched.
template <int KMAX>
__global__ void __launch_bounds__(256)
apply_rinv_kernel(float* __restrict__ Y, int64_t ldy, int64_t rows, int k,
                  const double* __restrict__ Rinv, const int* __restrict__ status, int attempt) {
  if (status[1] != 0) return;
  if (attempt == 2 && status[0] == 0) return;
  constexpr int NT = KMAX / 16;
  __shared__ float Ys[64][KMAX + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < 64 * KMAX; e += 256) {
    const int i = e / KMAX, c = e % KMAX;
    Ys[i][c] = (row0 + i < rows && c < k) ? Y[(row0 + i) * ldy + c] : 0.f;
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
      const int j = t * 16 + (lane & 15);
      const double b = (kr < k && j < k) ? Rinv[kr * k + j] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  // D[i][j] in lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gi = row0 + wave * 16 + 4 * q + (lane >> 4);
      const int j = t * 16 + (lane & 15);
      if (gi < rows && j < k) Y[gi * ldy + j] = (float)acc[t][q];
    }
}

}  // namespace

int gram_pick_splits(int64_t rows, int k) {
  (void)k;
  int64_t s = ceil_div(rows, 2048);
  if (s < 1) s = 1;
  if (s > 128) s = 128;
  return (int)s;
}

hipError_t launch_gram_f64(const float* Y, int64_t ldy, int64_t rows, int k, double* part,
                           int splits, const int* skip_flag, hipStream_t st) {
  const int nb = (k + GT - 1) / GT;
  const int64_t rchunk = round_up(ceil_div(rows, splits), GROWS);
  hipLaunchKernelGGL(gram_f64_kernel, dim3(nb * nb, splits), dim3(256), 0, st, Y, ldy, rows, k,
                     rchunk, part, skip_flag);
  return hipGetLastError();
}

hipError_t launch_cholesky(const double* part, int splits, int k, int64_t rows, double* Rinv,
                           int* status, int attempt, hipStream_t st) {
  if (k <= 64)
    hipLaunchKernelGGL(cholesky_kernel<64>, dim3(1), dim3(1024), 0, st, part, splits, k, rows, Rinv,
                       status, attempt);
  else if (k <= 128)
    hipLaunchKernelGGL(cholesky_kernel<128>, dim3(1), dim3(1024), 0, st, part, splits, k, rows, Rinv,
                       status, attempt);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_apply_rinv(float* Y, int64_t ldy, int64_t rows, int k, const double* Rinv,
                             const int* status, int attempt, hipStream_t st) {
  const unsigned g = (unsigned)ceil_div(rows, 64);
  if (g == 0) return hipSuccess;
  if (k <= 32)
    hipLaunchKernelGGL(apply_rinv_kernel<32>, dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt);
  else if (k <= 64)
    hipLaunchKernelGGL(apply_rinv_kernel<64>, dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt);
  else if (k <= 128)
    hipLaunchKernelGGL(apply_rinv_kernel<128>, dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
