// Exact relative error e = ||X - W Ht^T||_F / ||X||_F (the objective of eq 2.2),
// evaluated directly (never through the Gram expansion, which cancels
// catastrophically at small e) with FP64 products and FP64 accumulation.
//
// A workgroup owns 64 rows of X and a range of 64-column tiles.  Each wave
// computes a 16 x 64 block of W diag(sw) Ht^T on v_mfma_f64_16x16x4_f64
// (D[i][j] in lane j + 16 (i % 4), register i / 4), subtracts X, and
// accumulates squares.  Workgroup partials are summed in fixed order by the
// last workgroup to finish (completion counter, reset afterwards).
#include "common.h"

namespace {

constexpr int RB = 64;       // rows per workgroup
constexpr int CT = 64;       // columns per tile
constexpr int CTILES = 8;    // tiles per workgroup
constexpr int RMAXR = 128;

__global__ void __launch_bounds__(256)
residual_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                const float* __restrict__ W, const float* __restrict__ sw,
                const float* __restrict__ Ht, int r, double* __restrict__ part,
                double* __restrict__ out, unsigned* __restrict__ counter) {
  __shared__ float Hs[CT][RMAXR + 1];
  __shared__ double red[2][256];
  __shared__ int last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * RB;
  const int64_t colblk = (int64_t)blockIdx.y * CT * CTILES;
  const int ksteps = (r + 3) / 4;

  // A fragments (W rows of this wave), FP64, kept for all column tiles.
  double afr[RMAXR / 4];
  {
    const int64_t gi = row0 + wave * 16 + (lane & 15);
#pragma unroll
    for (int s = 0; s < RMAXR / 4; ++s) {
      const int k = 4 * s + (lane >> 4);
      double v = 0.0;
      if (s < ksteps && gi < m && k < r) v = (double)W[gi * r + k] * (double)(sw ? sw[k] : 1.f);
      afr[s] = v;
    }
  }
  double res = 0.0, xx = 0.0;
  for (int t = 0; t < CTILES; ++t) {
    const int64_t c0 = colblk + (int64_t)t * CT;
    if (c0 >= n) break;
    __syncthreads();
    for (int e = tid; e < CT * r; e += 256) {
      const int jj = e / r, k = e % r;
      Hs[jj][k] = (c0 + jj < n) ? Ht[(c0 + jj) * r + k] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      f64x4 d = {0, 0, 0, 0};
      const int jl = sub * 16 + (lane & 15);
#pragma unroll
      for (int s = 0; s < RMAXR / 4; ++s) {
        if (s < ksteps) {
          const int k = 4 * s + (lane >> 4);
          const double b = (k < r) ? (double)Hs[jl][k] : 0.0;
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[s], b, d, 0, 0, 0);
        }
      }
      const int64_t gj = c0 + jl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t gi = row0 + wave * 16 + 4 * q + (lane >> 4);
        if (gi < m && gj < n) {
          const double x = (double)X[gi * ldx + gj];
          const double df = x - d[q];
          res = fma(df, df, res);
          xx = fma(x, x, xx);
        }
      }
    }
  }
  red[0][tid] = res;
  red[1][tid] = xx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  if (tid == 0) {
    part[2 * bid] = red[0][0];
    part[2 * bid + 1] = red[1][0];
    __threadfence();
    last = (atomicAdd(counter, 1u) == (unsigned)nblk - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const volatile double* vp = part;
  double a0 = 0.0, a1 = 0.0;
  for (int b = tid; b < nblk; b += 256) {
    a0 += vp[2 * b];
    a1 += vp[2 * b + 1];
  }
  red[0][tid] = a0;
  red[1][tid] = a1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
    *counter = 0u;
  }
}

}  // namespace

int residual_blocks(int64_t m, int64_t n) {
  return (int)(ceil_div(m, RB) * ceil_div(n, (int64_t)CT * CTILES));
}

hipError_t launch_residual(const float* X, int64_t ldx, int64_t m, int64_t n, const float* W,
                           const float* sw, const float* Ht, int r, double* part, double* out,
                           unsigned* counter, hipStream_t st) {
  if (r > RMAXR) return hipErrorInvalidValue;
  dim3 grid((unsigned)ceil_div(m, RB), (unsigned)ceil_div(n, (int64_t)CT * CTILES));
  hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, st, X, ldx, m, n, W, sw, Ht, r, part, out,
                     counter);
  return hipGetLastError();
}
