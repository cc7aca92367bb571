// Allocation-free variant of the FP32 compression product (nmf_gemm): the
// split-K partials live in a file-scope device array instead of a caller
// workspace, so the call performs no device allocation of any kind.
//
// The array is one per GPU (each device holds its own copy from the first
// launch until the process ends).  Host code never uses its name as an address:
// the device address is looked up once per device with hipGetSymbolAddress,
// with that device current, and kept per device.  Every call on a GPU shares
// that GPU's array and leaves its last contents there; calls that overlap on
// one GPU (different streams, or threads) race on it.  Nothing in it has to
// start at zero: every split writes its full M x N slice before the fixed-order
// sum reads it.
#include <mutex>

#include "../../include/nmfrp.h"
#include "common.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // NMF_NOALLOC_SCRATCH_BYTES in the header
static_assert(SCRATCH_BYTES == NMF_NOALLOC_SCRATCH_BYTES, "header and library disagree");

__device__ __align__(256) float scratch[SCRATCH_BYTES / sizeof(float)];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
float* g_ptr[MAX_DEVICES] = {};

// Device address of this GPU's scratch (looked up on the first call per device).
hipError_t scratch_ptr(float** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" nmf_status nmf_gemm_noalloc(const float* A, int64_t lda, int32_t a_trans, const float* B, int64_t ldb,
                                       float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* hs) {
  if (M < 0 || N < 0 || K < 0 || N > 256 || ldc < N) {
    nmf_set_thread_error("bad arguments");
    return NMF_EINVAL;
  }
  if (M == 0 || N == 0) return NMF_OK;
  if (!A || !B || !C) {
    nmf_set_thread_error("null pointer");
    return NMF_EINVAL;
  }
  if (lda % 4 || ldb % 4 || !aligned16(A) || !aligned16(B)) {
    nmf_set_thread_error("lda, ldb % 4 and 16-byte alignment required");
    return NMF_EINVAL;
  }
  if ((!a_trans && K % 4) || (a_trans && M % 4)) {
    nmf_set_thread_error("K % 4 (a_trans=0) or M % 4 (a_trans=1) required");
    return NMF_EINVAL;
  }
  if ((!a_trans && lda < K) || (a_trans && lda < M) || ldb < N) {
    nmf_set_thread_error("leading dimension too small");
    return NMF_EINVAL;
  }
  // the same launch configuration as nmf_gemm, partials in the static array
  const int s = gemm_f32_pick_splits(M, N, K, a_trans);
  const size_t need = gemm_f32_part_floats(M, N, s) * sizeof(float);
  if (need > SCRATCH_BYTES) {
    nmf_set_thread_error("split-K partials of this product exceed the 64 MiB static scratch of nmf_gemm_noalloc "
                         "(use nmf_gemm with a workspace)");
    return NMF_EINVAL;
  }
  float* part = nullptr;
  hipError_t e = scratch_ptr(&part);
  if (e == hipSuccess) e = launch_gemm_f32(A, lda, a_trans, B, ldb, C, ldc, M, N, K, s, part, (hipStream_t)hs);
  if (e != hipSuccess) {
    nmf_set_thread_error(hipGetErrorString(e));
    return NMF_EHIP;
  }
  return NMF_OK;
}
