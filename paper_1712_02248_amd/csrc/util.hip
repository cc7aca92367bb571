// Small element-wise kernels: fills (used instead of hipMemsetAsync so that
// captured graphs replay correctly), strided copies, column scaling and the
// non-negativity / finiteness check on X (the problem of Sec 2 needs X >= 0).
#include "common.h"

namespace {

__global__ void fill_f32_kernel(float* p, int64_t count, float v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void fill_i32_kernel(int* p, int64_t count, int v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void copy2d_kernel(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows,
                              int64_t cols) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e - i * cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

__global__ void scale_cols_kernel(float* dst, int64_t ldd, const float* src, int64_t lds,
                                  int64_t rows, int cols, const float* scale) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols;
    const int j = (int)(e - i * cols);
    dst[i * ldd + j] = src[i * lds + j] * (scale ? scale[j] : 1.f);
  }
}

// flags[0] |= 1 if some element is negative, flags[1] |= 1 if some is not finite.
__global__ void check_nonneg_kernel(const float* X, int64_t ldx, int64_t m, int64_t n, int* flags) {
  const int64_t total = m * n;
  int neg = 0, bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / n, j = e - i * n;
    const float v = X[i * ldx + j];
    neg |= (v < 0.f);
    bad |= !isfinite(v);
  }
  if (neg) atomicOr(flags, 1);
  if (bad) atomicOr(flags + 1, 1);
}

// One thread copies what the host reads after a synchronisation into pinned,
// device-mapped host memory: out[0..2] = proxy sums (po), out[3..4] = residual
// sums (ro), out[5], out[6] = breakdown flags of the two range finders (status
// words 1 and 9 of qs).  Null sources leave their slots untouched.
__global__ void gather_host_kernel(const double* po, const double* ro, const int* qs, double* out) {
  if (threadIdx.x != 0) return;
  if (po) {
    out[0] = po[0];
    out[1] = po[1];
    out[2] = po[2];
  }
  if (ro) {
    out[3] = ro[0];
    out[4] = ro[1];
  }
  if (qs) {
    out[5] = (double)qs[1];
    out[6] = (double)qs[9];
  }
  __threadfence_system();
}

unsigned grid_for(int64_t count) {
  int64_t g = ceil_div(count, 256);
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_fill_f32(float* p, int64_t count, float v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(count)), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

hipError_t launch_gather_host(const double* po, const double* ro, const int* qs, double* out, hipStream_t st) {
  hipLaunchKernelGGL(gather_host_kernel, dim3(1), dim3(64), 0, st, po, ro, qs, out);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t count, int v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count)), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

hipError_t launch_copy2d(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows,
                         int64_t cols, hipStream_t st) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, dst, ldd, src,
                     lds, rows, cols);
  return hipGetLastError();
}

hipError_t launch_scale_cols(float* dst, int64_t ldd, const float* src, int64_t lds, int64_t rows,
                             int cols, const float* scale, hipStream_t st) {
  if (rows * cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, st, dst, ldd, src,
                     lds, rows, cols, scale);
  return hipGetLastError();
}

hipError_t launch_check_nonneg(const float* X, int64_t ldx, int64_t m, int64_t n, int* flags,
                               hipStream_t st) {
  if (m * n <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_nonneg_kernel, dim3(grid_for(m * n)), dim3(256), 0, st, X, ldx, m, n, flags);
  return hipGetLastError();
}
