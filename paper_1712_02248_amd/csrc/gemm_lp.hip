// Low-precision compression products (extension): C[M x N] = A[M x K] Bt[N x K]^T
// with both operands K-contiguous ("NT"), FP32 accumulation, FP32 output.
// A is the low-precision copy of X (for X B) or of X^T (for X^T B); Bt is the
// transposed low-precision copy of the thin operand (Omega or Q).  K is padded
// to the tile depth with zeros in both operands.  A is streamed once per
// product, so its loads are nontemporal (they do not displace the thin
// operand, which every workgroup re-reads, from L2).
//
// BF16: v_mfma_f32_32x32x16_bf16, lane l holds A[l % 32][16s + 8(l / 32) .. +7];
//       D[i][j] in lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4.
// FP8 (e4m3): v_mfma_scale_f32_16x16x128_f8f6f4, lane l holds
//       A[l % 16][32(l / 16) .. +31]; D[i][j] in lane j + 16 (i / 4), register i % 4.
//       Each 128-deep step multiplies by 2^(eA + eB) through the E8M0 scale
//       operands: eA is the exponent of X's 128 x 128 tile, eB that of the thin
//       operand's 128-row block.
#include "common.h"

namespace {

// ------------------------------------------------------------------------- BF16
// AT = false: A is M x Kpad (K-contiguous).  AT = true: A is K x lda (the copy
// of X itself, for X^T B): a thread loads rows 4 (t / 16) .. +3, columns
// 8 (t % 16) .. +7 of the 64 x 128 tile and writes their transpose, eight 4-value
// runs, into LDS; row i of the LDS tile keeps its 16-byte k chunks XOR-swizzled
// by (i / 8) % 8, which spreads those 8-byte stores over the banks while the
// MFMA fragment reads stay 16-byte aligned.  Rows at or past K and column
// chunks past lda read as zero.
template <int BM, int BN, int WM, int WN, bool AT>
__global__ void __launch_bounds__(256)
gemm_bf16_nt_kernel(const uint16_t* __restrict__ A, int64_t lda, const uint16_t* __restrict__ Bt,
                    int64_t ldbt, float* __restrict__ C, int64_t ldc, int64_t M, int64_t N,
                    int64_t Kpad, int64_t kchunk, int rot_xcd, int64_t K) {
  constexpr int BK = 64, ROW = BK + 8;                    // u16 per LDS row
  constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  constexpr int AV = BM * BK / 8 / 256, BV = BN * BK / 8 / 256;   // 16-byte loads per thread
  static_assert(AV >= 1 && BV >= 1 && WM * WN == 4, "tiling");
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * ROW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < Kpad ? kbeg + kchunk : Kpad;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[a][b][x] = 0.f;
  // two K steps in flight in registers (R0, R1) while the LDS tile is consumed
  i32x4 ra0[AV], rb0[BV], ra1[AV], rb1[BV];
  const i32x4 z4 = {0, 0, 0, 0};
  static_assert(!AT || (BM == 128 && AV == 4), "transposed A: 128-wide tiles, four rows per thread");
  auto load = [&](i32x4* ra, i32x4* rb, int64_t k0) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      if (!AT) {
        const int f = tid + 256 * p, row = f / (BK / 8), c8 = f % (BK / 8);
        const int64_t gi = i0 + row;
        ra[p] = gi < M ? __builtin_nontemporal_load((const i32x4*)(A + gi * lda + k0 + 8 * c8)) : z4;
      } else {
        const int64_t gk = k0 + 4 * (tid >> 4) + p, gi = i0 + 8 * (tid & 15);
        ra[p] = (gk < K && gi + 8 <= lda) ? __builtin_nontemporal_load((const i32x4*)(A + gk * lda + gi)) : z4;
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 8), c8 = f % (BK / 8);
      const int64_t gj = n0 + row;
      rb[p] = gj < N ? *(const i32x4*)(Bt + gj * ldbt + k0 + 8 * c8) : z4;
    }
  };
  auto store = [&](const i32x4* ra, const i32x4* rb) {
    if (!AT) {
#pragma unroll
      for (int p = 0; p < AV; ++p) {
        const int f = tid + 256 * p, row = f / (BK / 8), c8 = f % (BK / 8);
        *(i32x4*)(As + row * ROW + 8 * c8) = ra[p];
      }
    } else {
      // column c of the thread's chunk: tile row i = 8 (t % 16) + c gets k = 4 g .. 4 g + 3
      const int cl = tid & 15, g = tid >> 4;
      const int koff = 8 * ((g >> 1) ^ (cl & 7)) + 4 * (g & 1);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int sh = 16 * (c & 1);
        uint32_t v[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) v[p] = ((uint32_t)ra[p][c >> 1] >> sh) & 0xFFFFu;
        *(uint2*)(As + (8 * cl + c) * ROW + koff) = make_uint2(v[0] | (v[1] << 16), v[2] | (v[3] << 16));
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 8), c8 = f % (BK / 8);
      *(i32x4*)(Bs + row * ROW + 8 * c8) = rb[p];
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK / 16; ++ks) {
      bf16x8 af[TM], bf[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int il = wm * (BM / WM) + a * 32 + l32;
        const int kc = AT ? ((2 * ks + half) ^ ((il >> 3) & 7)) : (2 * ks + half);
        af[a] = *(const bf16x8*)(As + il * ROW + 8 * kc);
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jl = wn * (BN / WN) + b * 32 + l32;
        bf[b] = *(const bf16x8*)(Bs + jl * ROW + ks * 16 + 8 * half);
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };
  // steps t = 0 .. T-1 at k = kbeg + t BK; the LDS tile holds step t while
  // steps t + 1 and t + 2 load into the register sets
  const int64_t T = kend > kbeg ? (kend - kbeg) / BK : 0;
  // Rotated K order, which spreads concurrent loads of A over the HBM channels.
  // rot_xcd = 0: every workgroup starts at its own step.  rot_xcd = 1 (thin
  // operand too large to stay in L2 under arbitrary order): the workgroups of
  // one XCD (dispatch ids are dealt round-robin over the 8 XCDs) share a start
  // step and so read the thin operand in step from their L2, and the 8 XCDs
  // start 1/8 of the range apart.
  const int64_t wg = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t rot = T == 0 ? 0 : rot_xcd ? ((wg % 8) * T) / 8 : (int64_t)blockIdx.x % T;
  auto kstep = [&](int64_t s) { return kbeg + ((s + rot) % T) * BK; };
  if (T > 0) {
    load(ra0, rb0, kstep(0));
    if (T > 1) load(ra1, rb1, kstep(1));
    store(ra0, rb0);
    __syncthreads();
    if (T > 2) load(ra0, rb0, kstep(2));
    for (int64_t t = 0; t < T; t += 2) {
      // LDS: step t; R1: step t + 1; R0: step t + 2
      compute();
      __syncthreads();
      if (t + 1 < T) {
        store(ra1, rb1);
        __syncthreads();
        if (t + 3 < T) load(ra1, rb1, kstep(t + 3));
        // LDS: step t + 1; R0: step t + 2; R1: step t + 3
        compute();
        __syncthreads();
        if (t + 2 < T) {
          store(ra0, rb0);
          __syncthreads();
          if (t + 4 < T) load(ra0, rb0, kstep(t + 4));
        }
      }
    }
  }
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (BN / WN) + b * 32 + l32;
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int il = (x >> 2) * 8 + half * 4 + (x & 3);
        const int64_t gi = i0 + wm * (BM / WM) + a * 32 + il;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][x];
      }
    }
}

// -------------------------------------------------------------------------- FP8
// BM = 128 rows of A (one X tile row-block), BN columns, BK = 128 (one scale block).
template <int BN, int WN>
__global__ void __launch_bounds__(256)
gemm_fp8_nt_kernel(const uint8_t* __restrict__ A, int64_t lda, const int* __restrict__ EA,
                   int64_t ea_i, int64_t ea_k, const uint8_t* __restrict__ Bt, int64_t ldbt,
                   const int* __restrict__ EB, float* __restrict__ C, int64_t ldc, int64_t M,
                   int64_t N, int64_t Kpad, int64_t kchunk, int rot_xcd) {
  constexpr int BM = 128, BK = 128, ROW = BK + 16;         // bytes per LDS row
  constexpr int WM = 4 / WN;
  constexpr int TM = BM / WM / 16, TN = BN / WN / 16;      // 16x16 tiles per wave
  constexpr int AV = BM * BK / 16 / 256, BV = BN * BK / 16 / 256;
  static_assert(AV >= 1 && BV >= 1, "tiling");
  __shared__ __attribute__((aligned(16))) uint8_t As[BM * ROW];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[BN * ROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < Kpad ? kbeg + kchunk : Kpad;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  i32x4 ra[AV], rb[BV];
  const i32x4 z4 = {0, 0, 0, 0};
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 16), c16 = f % (BK / 16);
      const int64_t gi = i0 + row;
      ra[p] = gi < M ? __builtin_nontemporal_load((const i32x4*)(A + gi * lda + k0 + 16 * c16)) : z4;
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 16), c16 = f % (BK / 16);
      const int64_t gj = n0 + row;
      rb[p] = gj < N ? *(const i32x4*)(Bt + gj * ldbt + k0 + 16 * c16) : z4;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 16), c16 = f % (BK / 16);
      *(i32x4*)(As + row * ROW + 16 * c16) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, row = f / (BK / 16), c16 = f % (BK / 16);
      *(i32x4*)(Bs + row * ROW + 16 * c16) = rb[p];
    }
  };
  const int g4 = lane >> 4, l16 = lane & 15;
  const int64_t ti = i0 / 128;
  // rotated K-step order, as in the BF16 kernel
  const int64_t T = kend > kbeg ? (kend - kbeg) / BK : 0;
  const int64_t wg = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t rot = T == 0 ? 0 : rot_xcd ? ((wg % 8) * T) / 8 : (int64_t)blockIdx.x % T;
  auto kstep = [&](int64_t s) { return kbeg + ((s + rot) % T) * BK; };
  if (T > 0) {
    load(kstep(0));
    store();
    __syncthreads();
    for (int64_t t = 0; t < T; ++t) {
      const int64_t k0 = kstep(t);
      const bool more = t + 1 < T;
      if (more) load(kstep(t + 1));
      const int64_t kb = k0 / 128;
      const int sa = 127 + EA[ti * ea_i + kb * ea_k];
      const int sb = 127 + EB[kb];
      i32x8 af[TM], bf[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int il = wm * (BM / WM) + a * 16 + l16;
        const i32x4 lo = *(const i32x4*)(As + il * ROW + 32 * g4);
        const i32x4 hi = *(const i32x4*)(As + il * ROW + 32 * g4 + 16);
        af[a] = (i32x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jl = wn * (BN / WN) + b * 16 + l16;
        const i32x4 lo = *(const i32x4*)(Bs + jl * ROW + 32 * g4);
        const i32x4 hi = *(const i32x4*)(Bs + jl * ROW + 32 * g4 + 16);
        bf[b] = (i32x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[a], bf[b], acc[a][b], 0, 0, 0,
                                                                        sa, 0, sb);
      __syncthreads();
      if (more) {
        store();
        __syncthreads();
      }
    }
  }
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (BN / WN) + b * 16 + l16;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t gi = i0 + wm * (BM / WM) + a * 16 + 4 * g4 + x;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][x];
      }
    }
}

// Wide thin operands (128 < N <= 256): 512 threads over a 128 x 256 tile, eight
// waves of 64 x 64 (4 x 4 blocks of 16 x 16), two LDS stages (the tile of step
// t + 1 is stored while step t is read) with one barrier per step, and two
// register sets carrying the next two steps' loads.  Each output element
// accumulates the same MFMAs in the same K order as gemm_fp8_nt_kernel, so the
// results are identical.
__global__ void __launch_bounds__(512)
gemm_fp8_wide_kernel(const uint8_t* __restrict__ A, int64_t lda, const int* __restrict__ EA, int64_t ea_i,
                     int64_t ea_k, const uint8_t* __restrict__ Bt, int64_t ldbt, const int* __restrict__ EB,
                     float* __restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t Kpad, int64_t kchunk,
                     int rot_xcd) {
  constexpr int BM = 128, BN = 256, BK = 128, ROW = BK + 16, NT = 512;
  constexpr int WM = 2, WN = 4, TM = BM / WM / 16, TN = BN / WN / 16;   // 4 x 4 tiles per wave
  constexpr int AV = BM * BK / 16 / NT, BV = BN * BK / 16 / NT;          // 2, 4
  constexpr int STAGE = (BM + BN) * ROW;
  __shared__ __attribute__((aligned(16))) uint8_t lds[2 * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < Kpad ? kbeg + kchunk : Kpad;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  i32x4 ra0[AV], rb0[BV], ra1[AV], rb1[BV];
  const i32x4 z4 = {0, 0, 0, 0};
  auto load = [&](i32x4* ra, i32x4* rb, int64_t k0) {
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int f = tid + NT * p, row = f / (BK / 16), c16 = f % (BK / 16);
      const int64_t gi = i0 + row;
      ra[p] = gi < M ? __builtin_nontemporal_load((const i32x4*)(A + gi * lda + k0 + 16 * c16)) : z4;
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + NT * p, row = f / (BK / 16), c16 = f % (BK / 16);
      const int64_t gj = n0 + row;
      rb[p] = gj < N ? *(const i32x4*)(Bt + gj * ldbt + k0 + 16 * c16) : z4;
    }
  };
  auto store = [&](const i32x4* ra, const i32x4* rb, int stage) {
    uint8_t* As = lds + stage * STAGE;
    uint8_t* Bs = As + BM * ROW;
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const int f = tid + NT * p, row = f / (BK / 16), c16 = f % (BK / 16);
      *(i32x4*)(As + row * ROW + 16 * c16) = ra[p];
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + NT * p, row = f / (BK / 16), c16 = f % (BK / 16);
      *(i32x4*)(Bs + row * ROW + 16 * c16) = rb[p];
    }
  };
  const int g4 = lane >> 4, l16 = lane & 15;
  const int64_t ti = i0 / 128;
  const int64_t T = kend > kbeg ? (kend - kbeg) / BK : 0;
  const int64_t wg = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t rot = T == 0 ? 0 : rot_xcd ? ((wg % 8) * T) / 8 : (int64_t)blockIdx.x % T;
  auto kstep = [&](int64_t s) { return kbeg + ((s + rot) % T) * BK; };
  auto compute = [&](int64_t k0, int stage) {
    const uint8_t* As = lds + stage * STAGE;
    const uint8_t* Bs = As + BM * ROW;
    const int64_t kb = k0 / 128;
    const int sa = 127 + EA[ti * ea_i + kb * ea_k];
    const int sb = 127 + EB[kb];
    i32x8 af[TM], bf[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int il = wm * (BM / WM) + a * 16 + l16;
      const i32x4 lo = *(const i32x4*)(As + il * ROW + 32 * g4);
      const i32x4 hi = *(const i32x4*)(As + il * ROW + 32 * g4 + 16);
      af[a] = (i32x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int jl = wn * (BN / WN) + b * 16 + l16;
      const i32x4 lo = *(const i32x4*)(Bs + jl * ROW + 32 * g4);
      const i32x4 hi = *(const i32x4*)(Bs + jl * ROW + 32 * g4 + 16);
      bf[b] = (i32x8){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af[a], bf[b], acc[a][b], 0, 0, 0,
                                                                      sa, 0, sb);
  };
  // step s is staged in stage s % 2 from register set s % 2
  if (T > 0) {
    load(ra0, rb0, kstep(0));
    if (T > 1) load(ra1, rb1, kstep(1));
    store(ra0, rb0, 0);
    if (T > 2) load(ra0, rb0, kstep(2));
    __syncthreads();
    for (int64_t t = 0; t < T; t += 2) {
      // set 1: step t + 1, set 0: step t + 2
      if (t + 1 < T) store(ra1, rb1, 1);
      if (t + 3 < T) load(ra1, rb1, kstep(t + 3));
      __builtin_amdgcn_sched_barrier(0);
      compute(kstep(t), 0);
      __syncthreads();
      if (t + 1 < T) {
        if (t + 2 < T) store(ra0, rb0, 0);
        if (t + 4 < T) load(ra0, rb0, kstep(t + 4));
        __builtin_amdgcn_sched_barrier(0);
        compute(kstep(t + 1), 1);
        __syncthreads();
      }
    }
  }
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (BN / WN) + b * 16 + l16;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int64_t gi = i0 + wm * (BM / WM) + a * 16 + 4 * g4 + x;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][x];
      }
    }
}

__global__ void __launch_bounds__(256)
splitk_reduce_lp(const float* __restrict__ part, int splits, float* __restrict__ C, int64_t ldc,
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

int bn_lp(int64_t N) { return N <= 32 ? 32 : N <= 64 ? 64 : N <= 128 ? 128 : 256; }

hipError_t finish(float* part, int splits, float* C, int64_t ldc, int64_t M, int64_t N, hipStream_t st) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  return launch_splitk_reduce_lp(part, splits, C, ldc, M, N, st);
}

}  // namespace

// Per-XCD rotation when the thin-operand slices the grid streams (splits
// slices of N x kchunk elements) exceed a quarter of one XCD's 4 MiB L2.
int rot_per_xcd(int64_t N, int64_t kchunk, int splits, int elem_bytes) {
  return (double)N * kchunk * elem_bytes * splits > 1024.0 * 1024.0 ? 1 : 0;
}

hipError_t launch_splitk_reduce_lp(const float* part, int splits, float* C, int64_t ldc, int64_t M, int64_t N,
                                   hipStream_t st) {
  int64_t g = ceil_div(M * N, 256);
  if (g > 4096) g = 4096;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(splitk_reduce_lp, dim3((unsigned)g), dim3(256), 0, st, part, splits, C, ldc, M, N);
  return hipGetLastError();
}

int gemm_lp_pick_splits(int64_t M, int64_t N, int64_t Kpad, int bm) {
  const int64_t tiles = ceil_div(M, bm) * ceil_div(N, bn_lp(N));
  if (tiles <= 0) return 1;
  // about 512 workgroups: two per CU in a single dispatch wave (measured best
  // for both product shapes of the range finder)
  int64_t s = ceil_div(512, tiles);
  const int64_t kmax = Kpad / 512;  // at least 512 deep per split
  if (s > kmax) s = kmax;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

hipError_t launch_gemm_bf16_nt(const uint16_t* A, int64_t lda, const uint16_t* Bt, int64_t ldbt,
                               float* C, int64_t ldc, int64_t M, int64_t N, int64_t Kpad, int splits,
                               float* part, hipStream_t st, bool reduce, int a_trans, int64_t K) {
  if (M == 0 || N == 0) return hipSuccess;
  if (N > 256 || Kpad % 64 || lda % 8 || ldbt % 8) return hipErrorInvalidValue;
  if (a_trans && (N > 128 || K < 0 || K > Kpad)) return hipErrorInvalidValue;
  float* out = splits > 1 ? part : C;
  const int64_t ldo = splits > 1 ? N : ldc;
  const int64_t kchunk = round_up(ceil_div(Kpad, splits), 64);
  const int bn = bn_lp(N);
  const int bm = bn <= 128 ? 128 : 64;
  dim3 grid((unsigned)ceil_div(M, bm), (unsigned)ceil_div(N, bn), (unsigned)splits);
  const int rx = rot_per_xcd(N, kchunk, splits, 2);
  const int64_t kk = a_trans ? K : Kpad;
#define NMF_BF16_LAUNCH(BM_, BN_, WM_, WN_, AT_)                                                              \
  hipLaunchKernelGGL((gemm_bf16_nt_kernel<BM_, BN_, WM_, WN_, AT_>), grid, dim3(256), 0, st, A, lda, Bt, ldbt, \
                     out, ldo, M, N, Kpad, kchunk, rx, kk)
  if (a_trans) {
    switch (bn) {
      case 32: NMF_BF16_LAUNCH(128, 32, 4, 1, true); break;
      case 64: NMF_BF16_LAUNCH(128, 64, 2, 2, true); break;
      default: NMF_BF16_LAUNCH(128, 128, 2, 2, true); break;
    }
  } else {
    switch (bn) {
      case 32: NMF_BF16_LAUNCH(128, 32, 4, 1, false); break;
      case 64: NMF_BF16_LAUNCH(128, 64, 2, 2, false); break;
      case 128: NMF_BF16_LAUNCH(128, 128, 2, 2, false); break;
      default: NMF_BF16_LAUNCH(64, 256, 1, 4, false); break;
    }
  }
#undef NMF_BF16_LAUNCH
  if (!reduce) return hipGetLastError();
  return finish(part, splits, C, ldc, M, N, st);
}

hipError_t launch_gemm_fp8_nt(const uint8_t* A, int64_t lda, const int* EA, int64_t ea_i, int64_t ea_k,
                              const uint8_t* Bt, int64_t ldbt, const int* EB, float* C, int64_t ldc,
                              int64_t M, int64_t N, int64_t Kpad, int splits, float* part,
                              hipStream_t st, bool reduce) {
  if (M == 0 || N == 0) return hipSuccess;
  if (N > 256 || Kpad % 128 || lda % 16 || ldbt % 16) return hipErrorInvalidValue;
  float* out = splits > 1 ? part : C;
  const int64_t ldo = splits > 1 ? N : ldc;
  const int64_t kchunk = round_up(ceil_div(Kpad, splits), 128);
  const int bn = bn_lp(N);
  dim3 grid((unsigned)ceil_div(M, 128), (unsigned)ceil_div(N, bn), (unsigned)splits);
  const int rx = rot_per_xcd(N, kchunk, splits, 1);
  switch (bn) {
    case 32: hipLaunchKernelGGL((gemm_fp8_nt_kernel<32, 1>), grid, dim3(256), 0, st, A, lda, EA, ea_i, ea_k, Bt, ldbt, EB, out, ldo, M, N, Kpad, kchunk, rx); break;
    case 64: hipLaunchKernelGGL((gemm_fp8_nt_kernel<64, 2>), grid, dim3(256), 0, st, A, lda, EA, ea_i, ea_k, Bt, ldbt, EB, out, ldo, M, N, Kpad, kchunk, rx); break;
    case 128: hipLaunchKernelGGL((gemm_fp8_nt_kernel<128, 2>), grid, dim3(256), 0, st, A, lda, EA, ea_i, ea_k, Bt, ldbt, EB, out, ldo, M, N, Kpad, kchunk, rx); break;
    default: hipLaunchKernelGGL(gemm_fp8_wide_kernel, grid, dim3(512), 0, st, A, lda, EA, ea_i, ea_k, Bt, ldbt, EB, out, ldo, M, N, Kpad, kchunk, rx); break;
  }
  if (!reduce) return hipGetLastError();
  return finish(part, splits, C, ldc, M, N, st);
}
