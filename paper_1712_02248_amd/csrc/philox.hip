// Gaussian test matrix Omega of Sec 3 (entries i.i.d. N(0,1)) and uniform
// initial factors, drawn on the device from Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC'11).
//
// Element layout for a rows x cols matrix on stream `sid` with 64-bit `seed`:
// flat index e = row*cols + col; counter (e/4 low, e/4 high, sid, 0),
// key (seed low, seed high); the element takes word e%4 of the block.
// Normal: words (0,1) and (2,3) are Box-Muller pairs, u = (x + 0.5) 2^-32,
// cos for the even word, sin for the odd word, in FP64, rounded to FP32.
// Uniform: (x >> 8) 2^-24, times `scale`.
#include "common.h"
#include <math.h>

namespace {

NMF_DEV void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                          uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
  c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
}

NMF_DEV void philox10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    philox_round(ctr[0], ctr[1], ctr[2], ctr[3], k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

template <bool NORMAL>
__global__ void __launch_bounds__(256) philox_fill(float* __restrict__ out, int64_t rows, int64_t cols,
                                                   int64_t ld, uint32_t sid, uint64_t seed, float scale) {
  const int64_t total = rows * cols;
  const int64_t nblk = (total + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk;
       b += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)b, (uint32_t)((uint64_t)b >> 32), sid, 0u};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    float v[4];
    if (NORMAL) {
      const double two32 = 2.3283064365386963e-10;  // 2^-32
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const double ua = ((double)c[2 * p] + 0.5) * two32;
        const double ub = ((double)c[2 * p + 1] + 0.5) * two32;
        const double rad = sqrt(-2.0 * log(ua));
        const double ang = 6.283185307179586 * ub;
        v[2 * p] = (float)(rad * cos(ang));
        v[2 * p + 1] = (float)(rad * sin(ang));
      }
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) v[w] = (float)(c[w] >> 8) * 5.9604644775390625e-08f * scale;
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int64_t e = 4 * b + w;
      if (e < total) {
        const int64_t row = e / cols, col = e - row * cols;
        out[row * ld + col] = v[w];
      }
    }
  }
}

}  // namespace

static int fill_grid(int64_t total) {
  int64_t nblk = (total + 3) / 4;
  int64_t g = (nblk + 255) / 256;
  return (int)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

hipError_t launch_philox_normal(float* out, int64_t rows, int64_t cols, int64_t ld,
                                uint32_t sid, uint64_t seed, hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_fill<true>, dim3(fill_grid(rows * cols)), dim3(256), 0, st, out, rows,
                     cols, ld, sid, seed, 1.0f);
  return hipGetLastError();
}

hipError_t launch_philox_uniform(float* out, int64_t rows, int64_t cols, int64_t ld,
                                 uint32_t sid, uint64_t seed, float scale, hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(philox_fill<false>, dim3(fill_grid(rows * cols)), dim3(256), 0, st, out, rows,
                     cols, ld, sid, seed, scale);
  return hipGetLastError();
}
