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
  constexpr int PB = KMAX / TD;
  constexpr int NW = TD * TD / 64;
  if (attempt == 2 && status[0] == 0) return;
  __shared__ double colj[2][KMAX], rowj[2][KMAX];   // double-buffered: one barrier per column
  __shared__ double wred[NW];
  __shared__ int fail;
  const int tid = threadIdx.x, tx = tid % TD, ty = tid / TD;

  if (attempt == 1) {
    double dev = 0.0;
#pragma unroll
    for (int a = 0; a < PB; ++a)
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        const int i = ty + TD * a, l = tx + TD * b;
        if (i < k && l < k) dev = fmax(dev, fabs(G[i * k + l] - (i == l ? 1.0 : 0.0)));
      }
    for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off));
    if ((tid & 63) == 0) wred[tid >> 6] = dev;
    __syncthreads();
    double mx = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) mx = fmax(mx, wred[w]);
    if (mx <= 1e-6) {                     // uniform
      if (tid == 0) status[3] = 1;
      return;
    }
  }
  if (attempt == 0 && tid == 0) {
    status[0] = 0;
    status[3] = 0;
  }

  double M[PB][PB], X[PB][PB];
  for (int tryi = 0; tryi < 2; ++tryi) {
    double shift = 0.0;
    if (tryi == 1) {
      double trace = 0.0;
      for (int i = 0; i < k; ++i) trace += G[i * k + i];
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * k + (double)k * (k + 1)) * u * trace;
    }
#pragma unroll
    for (int a = 0; a < PB; ++a)
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        const int i = ty + TD * a, l = tx + TD * b;
        M[a][b] = (i < k && l <= i) ? G[i * k + l] + (i == l ? shift : 0.0) : 0.0;
        X[a][b] = (i < k && i == l) ? 1.0 : 0.0;
      }
    if (tid == 0) fail = 0;
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
        const int bf = j & 1;
        if (tx == jj) {
#pragma unroll
          for (int a = 0; a < PB; ++a) colj[bf][ty + TD * a] = M[a][b0];
        }
        if (ty == jj) {
#pragma unroll
          for (int b = 0; b < PB; ++b) rowj[bf][tx + TD * b] = X[b0][b];
        }
        __syncthreads();
        const double p = colj[bf][j];
        if (!(p > 0.0) || !isfinite(p)) {   // uniform: every thread reads the same p
          stop = true;
          if (tid == 0) fail = 1;
          break;
        }
        // 1/sqrt(p): hardware estimate and one Newton step; d = p / sqrt(p)
        double id = __builtin_amdgcn_rsq(p);
        id = id * fma(-0.5 * p * id, id, 1.5);
        const double d = p * id;
        double lc[PB], lr[PB], xj[PB];
#pragma unroll
        for (int a = 0; a < PB; ++a) lc[a] = colj[bf][ty + TD * a] * id;     // L[i][j]
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          lr[b] = colj[bf][tx + TD * b] * id;                                // L[l][j]
          xj[b] = rowj[bf][tx + TD * b] * id;                                // X[j][c] / L[j][j]
        }
#pragma unroll
        for (int a = 0; a < PB; ++a) {
          const int i = ty + TD * a;
#pragma unroll
          for (int b = 0; b < PB; ++b) {
            const int l = tx + TD * b;
            if (j < l && l <= i) M[a][b] -= lc[a] * lr[b];
            if (l <= j && j < i) X[a][b] -= lc[a] * xj[b];
          }
        }
        if (tx == jj) {
#pragma unroll
          for (int a = 0; a < PB; ++a) {
            const int i = ty + TD * a;
            if (i > j) M[a][b0] = lc[a];
            else if (i == j) M[a][b0] = d;
          }
        }
        if (ty == jj) {
#pragma unroll
          for (int b = 0; b < PB; ++b)
            if (tx + TD * b <= j) X[b0][b] = xj[b];
        }
      }
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
  // R^{-1}[c][i] = X[i][c] for c <= i, 0 below the diagonal
#pragma unroll
  for (int a = 0; a < PB; ++a)
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int i = ty + TD * a, c = tx + TD * b;
      if (i < k && c < k) {
        Rinv[c * k + i] = (c <= i) ? X[a][b] : 0.0;
      }
    }
}

// Q = Y R^{-1} in place on FP64 MFMA (v_mfma_f64_16x16x4_f64): a workgroup owns
// 64 rows (16 per wave) and all k columns; the tile is read into LDS before any
// write, so rows of other workgroups are never touched.  The tile is staged with
// batched float4 loads (ldy % 4 == 0); for k <= 64 R^{-1} is staged in LDS too
// (row stride KMAX + 2 doubles), larger k reads it from L2.
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

}  // namespace

int gram_pick_splits(int64_t rows, int k) {
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
  if (k <= 32)
    hipLaunchKernelGGL((cholesky_kernel<32, 8>), dim3(1), dim3(64), 0, st, G, k, rows, Rinv, status,
                       attempt);
  else if (k <= 64)
    hipLaunchKernelGGL((cholesky_kernel<64, 16>), dim3(1), dim3(256), 0, st, G, k, rows, Rinv, status,
                       attempt);
  else if (k <= 128)
    hipLaunchKernelGGL((cholesky_kernel<128, 32>), dim3(1), dim3(1024), 0, st, G, k, rows, Rinv,
                       status, attempt);
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
    hipLaunchKernelGGL((apply_rinv_kernel<128, false>), dim3(g), dim3(256), 0, st, Y, ldy, rows, k, Rinv, status,
                       attempt, nullptr, 0);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
