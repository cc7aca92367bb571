// FP32 MFMA GEMM for the compression products of Sec 3.1 / Sec 4:
// X Omega, X^T Omega, X^T Q, X Z (skinny: N = k' <= 256, M and K large).
//
// C[M x N] = op(A)[M x K] * B[K x N], FP32 in, FP32 accumulate, on
// v_mfma_f32_32x32x2_f32.  One 256-thread workgroup (4 waves) owns a BM x BN
// tile; BN covers all of k' so every element of X is read from HBM once.
// Tiles of A and B are staged through LDS.  Within each group of 8 k-values the
// contraction order is permuted so that a lane holding row i of A reads its 4
// k-values of one MFMA group as one 16-byte LDS load: in step s (0..3) lanes
// 0-31 contribute k = 8g + s and lanes 32-63 contribute k = 8g + 4 + s.
// Split-K writes FP32 partials that a second kernel sums in fixed order.
#include "common.h"

namespace {

constexpr int BK = 32;

template <int BM, int BN, int WM, int WN, bool AT>
__global__ void __launch_bounds__(256)
gemm_f32_kernel(const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb,
                float* __restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t K, int64_t kchunk,
                double* __restrict__ sq) {
  constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  static_assert(TM >= 1 && TN >= 1 && WM * WN == 4, "bad tiling");
  constexpr int AROW = AT ? (BM + 4) : (BK + 4);
  constexpr int A_ELEMS = AT ? BK * (BM + 4) : BM * (BK + 4);
  constexpr int BROW = BN + 4;
  constexpr int A_V4 = BM * BK / 4 / 256;  // float4 loads per thread
  constexpr int B_V4 = BK * BN / 4 / 256;
  static_assert(A_V4 >= 1 && B_V4 >= 1, "tile too small");
  __shared__ __attribute__((aligned(16))) float As[A_ELEMS];
  __shared__ __attribute__((aligned(16))) float Bs[BK * BROW];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  const int64_t n0 = (int64_t)blockIdx.y * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;

  f32x16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  // two K steps in flight in registers (R0, R1) while the LDS tile is consumed
  f32x4 ra0[A_V4], rb0[B_V4], ra1[A_V4], rb1[B_V4];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};

  auto load_tile = [&](f32x4* ra, f32x4* rb, int64_t k0) {
#pragma unroll
    for (int p = 0; p < A_V4; ++p) {
      const int f = tid + 256 * p;
      if (!AT) {
        const int row = f / (BK / 4), c4 = f % (BK / 4);
        const int64_t gi = i0 + row, gk = k0 + 4 * c4;
        ra[p] = (gi < M && gk < kend) ? *(const f32x4*)(A + gi * lda + gk) : z4;
      } else {
        const int kk = f / (BM / 4), c4 = f % (BM / 4);
        const int64_t gk = k0 + kk, gi = i0 + 4 * c4;
        ra[p] = (gk < kend && gi < M) ? *(const f32x4*)(A + gk * lda + gi) : z4;
      }
    }
#pragma unroll
    for (int p = 0; p < B_V4; ++p) {
      const int f = tid + 256 * p;
      const int kk = f / (BN / 4), c4 = f % (BN / 4);
      const int64_t gk = k0 + kk, gn = n0 + 4 * c4;
      f32x4 v = z4;
      if (gk < kend) {
        const float* src = B + gk * ldb + gn;
        if (gn + 3 < N) {
          v = *(const f32x4*)src;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (gn + e < N) ? src[e] : 0.f;
        }
      }
      rb[p] = v;
    }
  };
  // optional FP64 sum of squares of A (first column tile of the grid only, so
  // every element of A is counted once): ||X||^2 for free with X Q
  const bool want_sq = !AT && sq != nullptr && blockIdx.y == 0;
  double asq = 0.0;
  auto store_tile = [&](const f32x4* ra, const f32x4* rb) {
    if (want_sq) {
#pragma unroll
      for (int p = 0; p < A_V4; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) asq = fma((double)ra[p][e], (double)ra[p][e], asq);
    }
#pragma unroll
    for (int p = 0; p < A_V4; ++p) {
      const int f = tid + 256 * p;
      if (!AT) {
        const int row = f / (BK / 4), c4 = f % (BK / 4);
        *(f32x4*)(As + row * AROW + 4 * c4) = ra[p];
      } else {
        const int kk = f / (BM / 4), c4 = f % (BM / 4);
        *(f32x4*)(As + kk * AROW + 4 * c4) = ra[p];
      }
    }
#pragma unroll
    for (int p = 0; p < B_V4; ++p) {
      const int f = tid + 256 * p;
      const int kk = f / (BN / 4), c4 = f % (BN / 4);
      *(f32x4*)(Bs + kk * BROW + 4 * c4) = rb[p];
    }
  };

  const int half = lane >> 5, l32 = lane & 31;
  auto compute = [&]() {
#pragma unroll
    for (int g = 0; g < BK / 8; ++g) {
      const int kb = 8 * g + 4 * half;
      f32x4 af[TM], bf[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int il = wm * (BM / WM) + a * 32 + l32;
        if (!AT) {
          af[a] = *(const f32x4*)(As + il * AROW + kb);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) af[a][s] = As[(kb + s) * AROW + il];
        }
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jl = wn * (BN / WN) + b * 32 + l32;
#pragma unroll
        for (int s = 0; s < 4; ++s) bf[b][s] = Bs[(kb + s) * BROW + jl];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
          for (int b = 0; b < TN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a][s], bf[b][s], acc[a][b], 0, 0, 0);
    }
  };
  // steps t = 0 .. T-1 at k = kbeg + t BK; the LDS tile holds step t while
  // steps t + 1 and t + 2 load into the register sets
  const int64_t T = kend > kbeg ? ceil_div(kend - kbeg, (int64_t)BK) : 0;
  // natural K order: here the thin operand's tile is shared by all concurrent
  // workgroups through L2 (measured faster than a rotated order)
  auto kstep = [&](int64_t s) { return kbeg + s * BK; };
  if (T > 0) {
    load_tile(ra0, rb0, kstep(0));
    if (T > 1) load_tile(ra1, rb1, kstep(1));
    store_tile(ra0, rb0);
    __syncthreads();
    if (T > 2) load_tile(ra0, rb0, kstep(2));
    for (int64_t t = 0; t < T; t += 2) {
      compute();   // LDS: step t; R1: step t + 1; R0: step t + 2
      __syncthreads();
      if (t + 1 < T) {
        store_tile(ra1, rb1);
        __syncthreads();
        if (t + 3 < T) load_tile(ra1, rb1, kstep(t + 3));
        compute();   // LDS: step t + 1; R0: step t + 2; R1: step t + 3
        __syncthreads();
        if (t + 2 < T) {
          store_tile(ra0, rb0);
          __syncthreads();
          if (t + 4 < T) load_tile(ra0, rb0, kstep(t + 4));
        }
      }
    }
  }

  if (want_sq) {   // block sum in fixed order -> sq[blockIdx.x + gridDim.x blockIdx.z]
    __shared__ double red[256];
    red[tid] = asq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) sq[blockIdx.x + (int64_t)gridDim.x * blockIdx.z] = red[0];
  }
  // D[i][j] of a 32x32 tile: lane j + 32*((i/4)%2), register (i/8)*4 + i%4.
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);  // partial slice when split
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (BN / WN) + b * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int il = (r >> 2) * 8 + half * 4 + (r & 3);
        const int64_t gi = i0 + wm * (BM / WM) + a * 32 + il;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][r];
      }
    }
}

__global__ void __launch_bounds__(256)
splitk_reduce(const float* __restrict__ part, int splits, float* __restrict__ C, int64_t ldc,
              int64_t M, int64_t N) {
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / N, j = e - i * N;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(int64_t)z * total + e];
    C[i * ldc + j] = s;
  }
}

template <int BM, int BN, int WM, int WN>
hipError_t run(const float* A, int64_t lda, int a_trans, const float* B, int64_t ldb, float* C,
               int64_t ldc, int64_t M, int64_t N, int64_t K, int splits, double* sq, hipStream_t st) {
  const int64_t kchunk = round_up(ceil_div(K, splits), BK);
  dim3 grid((unsigned)ceil_div(M, BM), (unsigned)ceil_div(N, BN), (unsigned)splits);
  if (a_trans)
    hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, true>), grid, dim3(256), 0, st, A, lda, B,
                       ldb, C, ldc, M, N, K, kchunk, nullptr);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, false>), grid, dim3(256), 0, st, A, lda, B,
                       ldb, C, ldc, M, N, K, kchunk, sq);
  return hipGetLastError();
}

int bn_for(int64_t N) { return N <= 32 ? 32 : N <= 64 ? 64 : N <= 128 ? 128 : 256; }
// N <= 64 on large products: 256-row tiles, every wave owning 64 rows (two 32-row
// blocks), so each thin-operand fragment read from LDS feeds two MFMAs per column
// block.  Measured against 128-row tiles at 65536 x 4096: 10-20 % faster at N = 32
// (the update's r-wide products) and 12-19 % at N = 64 (the compression products).
// When they would leave fewer than 256 workgroups even with the deepest split-K
// (400 x 4096: 16), 128-row tiles are kept; there they were 35-40 % faster.
int bm_pick(int64_t M, int64_t N, int64_t K) {
  const int bn = bn_for(N);
  if (bn > 64) return bn <= 128 ? 128 : 64;
  int64_t kmax = K / 256;
  if (kmax > 64) kmax = 64;
  if (kmax < 1) kmax = 1;
  return ceil_div(M, 256) * kmax >= 256 ? 256 : 128;
}

}  // namespace

// Number of sum-of-squares partials launch_gemm_f32 writes for these sizes.
int gemm_f32_sq_parts(int64_t M, int64_t N, int64_t K, int splits) {
  return (int)(ceil_div(M, bm_pick(M, N, K)) * splits);
}

int gemm_f32_pick_splits(int64_t M, int64_t N, int64_t K, int a_trans) {
  (void)a_trans;
  const int bn = bn_for(N), bm = bm_pick(M, N, K);
  const int64_t tiles = ceil_div(M, bm) * ceil_div(N, bn);
  if (tiles <= 0) return 1;
  // about 1024 workgroups, 512 for the 256-row tiles (measured best for each)
  int64_t s = ceil_div(bm >= 256 ? 512 : 1024, tiles);
  const int64_t kmax = K / 256;  // keep at least 8 BK steps per split
  if (s > kmax) s = kmax;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

size_t gemm_f32_part_floats(int64_t M, int64_t N, int splits) {
  return splits > 1 ? (size_t)splits * M * N : 0;
}

hipError_t launch_gemm_f32(const float* A, int64_t lda, int a_trans, const float* B, int64_t ldb,
                           float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int splits,
                           float* part, hipStream_t st, double* sq) {
  if (M == 0 || N == 0) return hipSuccess;
  if (N > 256 || splits < 1) return hipErrorInvalidValue;
  if (lda % 4 || ldb % 4 || ((uintptr_t)A & 15) || ((uintptr_t)B & 15)) return hipErrorInvalidValue;
  if ((!a_trans && K % 4) || (a_trans && M % 4)) return hipErrorInvalidValue;
  if (splits > 1 && !part) return hipErrorInvalidValue;
  float* out = splits > 1 ? part : C;
  const int64_t ldo = splits > 1 ? N : ldc;
  hipError_t e;
  const bool tall = bm_pick(M, N, K) == 256;
  switch (bn_for(N)) {
    case 32:
      e = tall ? run<256, 32, 4, 1>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st)
               : run<128, 32, 4, 1>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st);
      break;
    case 64:
      e = tall ? run<256, 64, 4, 1>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st)
               : run<128, 64, 2, 2>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st);
      break;
    case 128: e = run<128, 128, 2, 2>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st); break;
    default: e = run<64, 256, 1, 4>(A, lda, a_trans, B, ldb, out, ldo, M, N, K, splits, sq, st); break;
  }
  if (e != hipSuccess || splits == 1) return e;
  int64_t g = ceil_div(M * N, 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)g), dim3(256), 0, st, part, splits, C, ldc, M, N);
  return hipGetLastError();
}
