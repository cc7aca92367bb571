// Eigenvalues of a small symmetric FP64 matrix (k <= 128) by the cyclic Jacobi
// method in parallel (round-robin) order, one workgroup.  Used for the singular
// values of the compressed data X-hat = Q_L^T X (Sec 4): the eigenvalues of its
// Gram X-hat X-hat^T are sigma_j(X-hat)^2, and for the leading j these approach
// sigma_j(X) as the basis captures the dominant subspace (Sec 3.1).
//
// Method (Golub and Van Loan, Matrix Computations, Sec 8.5): a rotation in the
// (p, q) plane with
//   tau = (a_qq - a_pp) / (2 a_pq),  t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1 / sqrt(1 + t^2),  s = t c
// makes the (p, q) entry of J^T A J zero.  One sweep visits every pair once in
// k - 1 rounds of k / 2 disjoint pairs (the circle method of a round-robin
// tournament: index K-1 meets index r in round r, and i = 1 .. K/2 - 1 pairs
// (r + i) and (r - i) mod (K - 1), K = k rounded up to even; a pair holding
// the padding index K-1 = k is skipped).  Rotations on disjoint pairs commute,
// so a round applies all its row rotations, then all its column rotations.
// Sweeps stop when the off-diagonal Frobenius norm falls below 1e-13 of the
// matrix's (at most 40 sweeps); the eigenvalues are then within that bound.
#include "common.h"

namespace {

constexpr int EKMAX = 128;
constexpr int ELD = EKMAX + 1;

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup's 256 threads; every thread gets the total.
__device__ inline double block_sum_d(double v, double* red) {
  v = wave_sum_d(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// A: k x k (lower triangle read), w: k outputs, descending (sqrt of the
// clamped value when sqrt_out).  info[0] = sweeps, info[1] = 1 if A holds a
// non-finite entry (then w is not written).
__global__ __launch_bounds__(256) void sym_eig_jacobi_kernel(const double* __restrict__ A, int64_t lda, int k,
                                                             int sqrt_out, double* __restrict__ w,
                                                             int* __restrict__ info) {
  __shared__ double S[EKMAX * ELD];
  __shared__ double cs[EKMAX / 2], sn[EKMAX / 2];
  __shared__ int pp[EKMAX / 2], qq[EKMAX / 2];
  __shared__ double red[4];
  const int t = threadIdx.x;
  const int ld = k + 1;
  // whole-matrix passes: eight rows at a time, 32 columns per row (no division)
  const int ri = t >> 5, cj = t & 31;
  double fro = 0.0, off = 0.0;
  for (int i = ri; i < k; i += 8)
    for (int j = cj; j < k; j += 32) {
      const double v = i >= j ? A[(int64_t)i * lda + j] : A[(int64_t)j * lda + i];
      S[i * ld + j] = v;
      fro += v * v;
      if (i != j) off += v * v;
    }
  fro = block_sum_d(fro, red);
  off = block_sum_d(off, red);
  if (!isfinite(fro)) {
    if (t == 0) {
      info[0] = 0;
      info[1] = 1;
    }
    return;
  }
  const double thr = 1e-26 * fro;
  const int K = k + (k & 1), P = K / 2;
  int sweeps = 0;
  while (off > thr && sweeps < 40) {
    for (int rd = 0; rd < K - 1; ++rd) {
      if (t < P) {
        int p, q;
        if (t == 0) {
          p = rd;
          q = K - 1;
        } else {
          p = (rd + t) % (K - 1);
          q = (rd - t + (K - 1)) % (K - 1);
        }
        double c = 1.0, s = 0.0;
        if (p < k && q < k) {
          const double apq = S[p * ld + q];
          if (apq != 0.0) {
            const double tau = (S[q * ld + q] - S[p * ld + p]) / (2.0 * apq);
            const double at = fabs(tau);
            const double tt = at > 1e150 ? 0.5 / tau : (tau >= 0 ? 1.0 : -1.0) / (at + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        } else {
          p = q = -1;   // the padding index: no rotation
        }
        pp[t] = p;
        qq[t] = q;
        cs[t] = c;
        sn[t] = s;
      }
      __syncthreads();
      // four threads per pair (t / 4), each taking every fourth row or column
      const int i = t >> 2, j0 = t & 3;
      const int p = i < P ? pp[i] : -1, q = i < P ? qq[i] : -1;
      const double c = i < P ? cs[i] : 1.0, s = i < P ? sn[i] : 0.0;
      // rows p, q of J^T A
      if (p >= 0)
        for (int j = j0; j < k; j += 4) {
          const double a = S[p * ld + j], b = S[q * ld + j];
          S[p * ld + j] = c * a - s * b;
          S[q * ld + j] = s * a + c * b;
        }
      __syncthreads();
      // columns p, q of (J^T A) J
      if (p >= 0)
        for (int j = j0; j < k; j += 4) {
          const double a = S[j * ld + p], b = S[j * ld + q];
          S[j * ld + p] = c * a - s * b;
          S[j * ld + q] = s * a + c * b;
        }
      __syncthreads();
    }
    ++sweeps;
    double o = 0.0;
    for (int i = ri; i < k; i += 8)
      for (int j = cj; j < k; j += 32)
        if (i != j) o += S[i * ld + j] * S[i * ld + j];
    off = block_sum_d(o, red);
  }
  // descending order by rank (equal values keep index order)
  if (t < k) {
    const double v = S[t * ld + t];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double u = S[j * ld + j];
      rank += (u > v) || (u == v && j < t);
    }
    w[rank] = sqrt_out ? sqrt(fmax(v, 0.0)) : v;
  }
  if (t == 0) {
    info[0] = sweeps;
    info[1] = 0;
  }
}

}  // namespace

hipError_t launch_sym_eig(const double* A, int64_t lda, int k, int sqrt_out, double* w, int* info, hipStream_t st) {
  if (k <= 0 || k > EKMAX || lda < k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sym_eig_jacobi_kernel, dim3(1), dim3(256), 0, st, A, lda, k, sqrt_out, w, info);
  return hipGetLastError();
}
