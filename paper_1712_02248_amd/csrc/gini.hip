// Gini coefficient of a matrix (Sec 5.1, the sparsity measure of B):
//   G = sum_i (2 i - N - 1) b_(i) / (N sum_i b_i),  i = 1..N,
// over all N entries sorted ascending.  The entries are sorted on the device by
// a least-significant-digit radix sort of 32-bit keys (four stable passes of
// eight bits), then the two sums are formed in FP64 over the sorted order.
//
// Keys: the FP32 bit pattern with the sign bit flipped for x >= +0 and all bits
// flipped for x < 0 (or -0), which orders the keys as the values (-0 and +0 are
// adjacent and equal in value, so their order does not change the sums).
//
// One pass over the keys:
//   hist     per tile of GTILE keys the count of each digit, stored digit-major
//            (hist[d * nt + tile]);
//   scan     exclusive prefix sum over that array (one workgroup): the first
//            output slot of digit d from tile t;
//   scatter  each tile places its keys in element order: per round of 256 keys
//            the lanes of a wave with equal digits find each other by ballots
//            over the digit's bits, the wave totals per digit are exchanged in
//            LDS, and a key goes to run[d] + (keys of digit d in earlier waves
//            of the round) + (its rank among equal digits in its wave), so the
//            pass is stable.
#include <algorithm>

#include "common.h"

namespace {

constexpr int GT = 256, GI = 16, GTILE = GT * GI;   // keys per tile: 4096

NMF_DEV uint32_t gini_key(float x) {
  const uint32_t b = __builtin_bit_cast(uint32_t, x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

NMF_DEV float gini_value(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __builtin_bit_cast(float, b);
}

__global__ void __launch_bounds__(256)
gini_keys_kernel(const float* __restrict__ B, int64_t ldb, int64_t rows, int64_t cols, uint32_t* __restrict__ keys) {
  const int64_t n = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / cols, j = e - i * cols;
    keys[e] = gini_key(B[i * ldb + j]);
  }
}

__global__ void __launch_bounds__(GT)
gini_hist_kernel(const uint32_t* __restrict__ keys, int64_t n, int shift, uint32_t* __restrict__ hist, int nt) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * GTILE;
#pragma unroll
  for (int q = 0; q < GI; ++q) {
    const int64_t e = base + q * GT + tid;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nt + blockIdx.x] = h[tid];
}

// Exclusive prefix sum of a[0..total) in place, one workgroup of 1024 threads:
// each thread sums a contiguous segment, the segment sums are scanned in LDS,
// then each thread rewrites its segment.
__global__ void __launch_bounds__(1024)
gini_scan_kernel(uint32_t* __restrict__ a, int64_t total) {
  __shared__ uint32_t s[1024];
  const int tid = threadIdx.x;
  const int64_t seg = (total + 1023) / 1024;
  const int64_t b0 = tid * seg, b1 = b0 + seg < total ? b0 + seg : total;
  uint32_t sum = 0u;
  for (int64_t e = b0; e < b1; ++e) sum += a[e];
  s[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
    const uint32_t v = tid >= off ? s[tid - off] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  uint32_t run = s[tid] - sum;
  for (int64_t e = b0; e < b1; ++e) {
    const uint32_t v = a[e];
    a[e] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(GT)
gini_scatter_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int64_t n, int shift,
                    const uint32_t* __restrict__ offs, int nt) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[4][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  run[tid] = offs[(int64_t)tid * nt + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));   // lanes below this one
  const int64_t base = (int64_t)blockIdx.x * GTILE;
  for (int q = 0; q < GI; ++q) {
#pragma unroll
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    const int64_t e = base + q * GT + tid;
    const bool valid = e < n;
    const uint32_t k = valid ? in[e] : 0u;
    const uint32_t d = (k >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t v = __ballot(valid && bit);
      m &= bit ? v : ~v;
    }
    const int rank = __popcll(m & lt);
    if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + (uint32_t)rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      out[pos] = k;
    }
    __syncthreads();
    run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
    __syncthreads();
  }
}

// Per workgroup: sum_e (2 e + 1 - N) b_(e) and sum_e b_(e) (e = 0..N-1, sorted),
// FP64, reduced in a fixed order -> part[2 blockIdx.x + {0, 1}].
__global__ void __launch_bounds__(256)
gini_sum_kernel(const uint32_t* __restrict__ keys, int64_t n, double* __restrict__ part) {
  __shared__ double red[2][256];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double x = gini_value(keys[e]);
    s1 += (double)(2 * e + 1 - n) * x;
    s2 += x;
  }
  red[0][threadIdx.x] = s1;
  red[1][threadIdx.x] = s2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

constexpr int GSUM_BLOCKS = 256;

int64_t gini_tiles(int64_t n) { return ceil_div(n, (int64_t)GTILE); }

}  // namespace

size_t gini_workspace_bytes(int64_t rows, int64_t cols) {
  const int64_t n = rows * cols;
  const int64_t nt = gini_tiles(n);
  // keys twice, the digit counts, the partial sums and the two results
  return (size_t)round_up(2 * n * 4, 256) + (size_t)round_up(256 * nt * 4, 256) +
         (size_t)round_up(GSUM_BLOCKS * 2 * 8, 256) + 256;
}

hipError_t launch_gini(const float* B, int64_t ldb, int64_t rows, int64_t cols, void* ws, double* out2,
                       hipStream_t st) {
  const int64_t n = rows * cols;
  if (n <= 0 || n > (int64_t)0xFFFFFFFFll || ldb < cols) return hipErrorInvalidValue;
  const int64_t nt = gini_tiles(n);
  char* p = (char*)ws;
  uint32_t* k0 = (uint32_t*)p;
  uint32_t* k1 = k0 + n;
  p += round_up(2 * n * 4, 256);
  uint32_t* hist = (uint32_t*)p;
  p += round_up(256 * nt * 4, 256);
  double* part = (double*)p;
  const unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 256), 4096);
  hipLaunchKernelGGL(gini_keys_kernel, dim3(g), dim3(256), 0, st, B, ldb, rows, cols, k0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 8 * pass;
    uint32_t* src = (pass & 1) ? k1 : k0;
    uint32_t* dst = (pass & 1) ? k0 : k1;
    hipLaunchKernelGGL(gini_hist_kernel, dim3((unsigned)nt), dim3(GT), 0, st, src, n, shift, hist, (int)nt);
    hipLaunchKernelGGL(gini_scan_kernel, dim3(1), dim3(1024), 0, st, hist, 256 * nt);
    hipLaunchKernelGGL(gini_scatter_kernel, dim3((unsigned)nt), dim3(GT), 0, st, src, dst, n, shift, hist, (int)nt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // four passes: the sorted keys are back in k0
  const int sb = (int)std::min<int64_t>(ceil_div(n, 256), GSUM_BLOCKS);
  hipLaunchKernelGGL(gini_sum_kernel, dim3(sb), dim3(256), 0, st, k0, n, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_sum_partials_f64(part, sb, 2, out2, nullptr, st);
}
