// Split-BF16 products on the FP32 data matrix (extension, for the projected
// data of Sec 4, X^T Q_L and X Q_R), and the transposed BF16 copies of thin
// operands used by every BF16 product.
//
// Split-BF16: each FP32 value v is carried as hi + lo with hi = bf16(v) and
// lo = bf16(v - hi), both rounded to nearest even (v - hi is exact in FP32), so
// |v - hi - lo| <= 2^-16 |v|.  A product term is hi_a hi_b + hi_a lo_b + lo_a hi_b
// (lo_a lo_b, below 2^-16 |a b|, is dropped), three v_mfma_f32_32x32x16_bf16 per
// 16-deep step with FP32 accumulation: about 16 significant bits per term.
//
// C[M x N] = op(X)[M x K] B[K x N]:
//   at = 0: X is M x K (row i of C from row i of X)       -> X Q_R
//   at = 1: X is K x M (row i of C from column i of X)    -> X^T Q_L
// B arrives prepared as BtH, BtL (N x Kpad BF16, K-contiguous, zero padded).
// X is streamed from HBM with nontemporal loads, once per 64-column tile of C;
// the split (and for at = 1 the transposition, eight K values packed per
// 16-byte LDS store) happens while a tile is staged into LDS, so both cases
// read K-contiguous 16-byte MFMA fragments.  Two K steps are in flight in
// registers while the LDS tile is consumed; the K order is rotated per
// workgroup or per XCD as in the other products.  Split-K partials are summed
// by the caller in fixed order.
#include "common.h"

namespace {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// two FP32 values -> packed BF16 pair (a in the low half), nearest even
NMF_DEV uint32_t pk_bf16(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
// hi and lo pairs of (a, b)
NMF_DEV void split_pk(float a, float b, uint32_t& h, uint32_t& l) {
  h = pk_bf16(a, b);
  l = pk_bf16(a - __builtin_bit_cast(float, h << 16), b - __builtin_bit_cast(float, h & 0xFFFF0000u));
}

// B (K x N FP32, ldb) -> BtH (and BtL when SPLIT) (N x ldbt BF16), transposed,
// zero for k >= K.  64 x 64 tiles through LDS: coalesced reads along N,
// coalesced 32-byte writes along K.
template <bool SPLIT>
__global__ void __launch_bounds__(256)
prep_bt_kernel(const float* __restrict__ B, int64_t ldb, int64_t K, int64_t N, uint16_t* __restrict__ BtH,
               uint16_t* __restrict__ BtL, int64_t ldbt) {
  __shared__ float T[64][65];
  const int tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 64;
  {
    const int jj = tid & 63;
    const int64_t j = j0 + jj;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int kk = (tid >> 6) + 4 * r;
      const int64_t k = k0 + kk;
      T[jj][kk] = (k < K && j < N) ? B[k * ldb + j] : 0.f;
    }
  }
  __syncthreads();
  const int jj = tid >> 2, kq = (tid & 3) * 16;
  const int64_t j = j0 + jj;
  if (j >= N) return;
  uint32_t h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float a = T[jj][kq + 2 * e], b = T[jj][kq + 2 * e + 1];
    if (SPLIT) split_pk(a, b, h[e], l[e]);
    else h[e] = pk_bf16(a, b);
  }
  i32x4* dh = (i32x4*)(BtH + j * ldbt + k0 + kq);
  dh[0] = (i32x4){(int)h[0], (int)h[1], (int)h[2], (int)h[3]};
  dh[1] = (i32x4){(int)h[4], (int)h[5], (int)h[6], (int)h[7]};
  if (SPLIT) {
    i32x4* dl = (i32x4*)(BtL + j * ldbt + k0 + kq);
    dl[0] = (i32x4){(int)l[0], (int)l[1], (int)l[2], (int)l[3]};
    dl[1] = (i32x4){(int)l[4], (int)l[5], (int)l[6], (int)l[7]};
  }
}

constexpr int SBM = 128, SBK = 64, SROW = SBK + 8;   // u16 per LDS row

// SBN = 64 (N <= 64), 128 or 256 for wider thin operands (k' up to 256: one
// pass over X per product instead of one per 64 columns).
template <bool AT, int SBN>
__global__ void __launch_bounds__(256)
gemm_split_kernel(const float* __restrict__ X, int64_t ldx, const uint16_t* __restrict__ BtH,
                  const uint16_t* __restrict__ BtL, int64_t ldbt, float* __restrict__ C, int64_t ldc,
                  int64_t M, int64_t N, int64_t K, int64_t kchunk, int rot_xcd, double* __restrict__ sq) {
  constexpr int WM = 2, WN = 2;
  constexpr int TM = SBM / WM / 32, TN = SBN / WN / 32;
  constexpr int AV = SBM * SBK / 4 / 256;          // float4 loads of X per thread (8)
  constexpr int BV = SBN * SBK / 8 / 256;          // 16-byte loads per thread, each of hi and lo (2)
  __shared__ __attribute__((aligned(16))) uint16_t AsH[SBM * SROW];
  __shared__ __attribute__((aligned(16))) uint16_t AsL[SBM * SROW];
  __shared__ __attribute__((aligned(16))) uint16_t BsH[SBN * SROW];
  __shared__ __attribute__((aligned(16))) uint16_t BsL[SBN * SROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * SBM, n0 = (int64_t)blockIdx.y * SBN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[a][b][x] = 0.f;

  f32x4 ra0[AV], ra1[AV];
  i32x4 rh0[BV], rl0[BV], rh1[BV], rl1[BV];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  const i32x4 zi = {0, 0, 0, 0};
  // Per-lane element offsets inside a tile (32-bit: the launcher checks
  // SBM ldx < 2^30), added to a uniform tile base, so the loads use scalar-base
  // addressing.  at = 0: lane reads row (tid / 16) + 16 p, columns 4 (tid % 16) .. +3
  // of the tile; at = 1: columns 4 (tid % 32) .. +3 of tile rows 8 (tid / 32) + p.
  uint32_t aoff[AV];
#pragma unroll
  for (int p = 0; p < AV; ++p)
    aoff[p] = !AT ? (uint32_t)(((tid >> 4) + 16 * p) * ldx + 4 * (tid & 15))
                  : (uint32_t)((8 * (tid >> 5) + p) * ldx + 4 * (tid & 31));
  uint32_t boff[BV];
#pragma unroll
  for (int p = 0; p < BV; ++p) {
    const int f = tid + 256 * p;
    boff[p] = (uint32_t)((f >> 3) * ldbt + 8 * (f & 7));
  }
  const bool interior = i0 + SBM <= M && n0 + SBN <= N;   // uniform
  auto load = [&](f32x4* ra, i32x4* rh, i32x4* rl, int64_t k0) {
    const float* tile = !AT ? X + i0 * ldx + k0 : X + k0 * ldx + i0;
    const uint16_t* th = BtH + n0 * ldbt + k0;
    const uint16_t* tl = BtL + n0 * ldbt + k0;
    if (interior && k0 + SBK <= kend) {
#pragma unroll
      for (int p = 0; p < AV; ++p) ra[p] = __builtin_nontemporal_load((const f32x4*)(tile + aoff[p]));
#pragma unroll
      for (int p = 0; p < BV; ++p) {
        rh[p] = *(const i32x4*)(th + boff[p]);
        rl[p] = *(const i32x4*)(tl + boff[p]);
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      f32x4 v = z4;
      if (!AT) {
        const int64_t gi = i0 + (tid >> 4) + 16 * p, gk = k0 + 4 * (tid & 15);
        if (gi < M && gk < kend) {
          v = __builtin_nontemporal_load((const f32x4*)(tile + aoff[p]));
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (gk + d >= kend) v[d] = 0.f;               // K not a multiple of 4
        }
      } else {
        const int64_t gk = k0 + 8 * (tid >> 5) + p, gi = i0 + 4 * (tid & 31);
        if (gk < kend && gi < M) {
          v = __builtin_nontemporal_load((const f32x4*)(tile + aoff[p]));
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (gi + d >= M) v[d] = 0.f;                  // M not a multiple of 4
        }
      }
      ra[p] = v;
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int64_t gj = n0 + ((tid + 256 * p) >> 3);
      rh[p] = gj < N ? *(const i32x4*)(th + boff[p]) : zi;
      rl[p] = gj < N ? *(const i32x4*)(tl + boff[p]) : zi;
    }
  };
  // optional FP64 sum of squares of X (at = 0, first column tile only, so that
  // every element is counted once): ||X||^2 for free with X Q_R
  const bool want_sq = !AT && sq != nullptr && blockIdx.y == 0;
  double xsq = 0.0;
  auto store = [&](const f32x4* ra, const i32x4* rh, const i32x4* rl) {
    if (want_sq) {
#pragma unroll
      for (int p = 0; p < AV; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e) xsq = fma((double)ra[p][e], (double)ra[p][e], xsq);
    }
    if (!AT) {
#pragma unroll
      for (int p = 0; p < AV; ++p) {
        const int f = tid + 256 * p, row = f >> 4, c4 = f & 15;
        uint32_t h0, l0, h1, l1;
        split_pk(ra[p][0], ra[p][1], h0, l0);
        split_pk(ra[p][2], ra[p][3], h1, l1);
        *(uint2*)(AsH + row * SROW + 4 * c4) = make_uint2(h0, h1);
        *(uint2*)(AsL + row * SROW + 4 * c4) = make_uint2(l0, l1);
      }
    } else {
      // tile row k = 8 (tid / 32) + p, tile column i = 4 (tid % 32) + d: pack the
      // eight k values of column i into one 16-byte store at As[i][8 (tid / 32)]
      const int kb = 8 * (tid >> 5), ib = 4 * (tid & 31);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) split_pk(ra[2 * e][d], ra[2 * e + 1][d], h[e], l[e]);
        *(i32x4*)(AsH + (ib + d) * SROW + kb) = (i32x4){(int)h[0], (int)h[1], (int)h[2], (int)h[3]};
        *(i32x4*)(AsL + (ib + d) * SROW + kb) = (i32x4){(int)l[0], (int)l[1], (int)l[2], (int)l[3]};
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, row = f >> 3, c8 = f & 7;
      *(i32x4*)(BsH + row * SROW + 8 * c8) = rh[p];
      *(i32x4*)(BsL + row * SROW + 8 * c8) = rl[p];
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < SBK / 16; ++ks) {
      bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int il = wm * (SBM / WM) + a * 32 + l32;
        ah[a] = *(const bf16x8*)(AsH + il * SROW + ks * 16 + 8 * half);
        al[a] = *(const bf16x8*)(AsL + il * SROW + ks * 16 + 8 * half);
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jl = wn * (SBN / WN) + b * 32 + l32;
        bh[b] = *(const bf16x8*)(BsH + jl * SROW + ks * 16 + 8 * half);
        bl[b] = *(const bf16x8*)(BsL + jl * SROW + ks * 16 + 8 * half);
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {   // small terms first
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
  };
  const int T = kend > kbeg ? (int)ceil_div(kend - kbeg, (int64_t)SBK) : 0;
  const int wg = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int rot = T == 0 ? 0 : rot_xcd ? ((wg % 8) * T) / 8 : (int)(blockIdx.x % T);
  auto kstep = [&](int s) { return kbeg + (int64_t)((s + rot) % T) * SBK; };
  if (T > 0) {
    load(ra0, rh0, rl0, kstep(0));
    if (T > 1) load(ra1, rh1, rl1, kstep(1));
    store(ra0, rh0, rl0);
    __syncthreads();
    if (T > 2) load(ra0, rh0, rl0, kstep(2));
    for (int t = 0; t < T; t += 2) {
      compute();   // LDS: step t; set 1: step t + 1; set 0: step t + 2
      __syncthreads();
      if (t + 1 < T) {
        store(ra1, rh1, rl1);
        __syncthreads();
        if (t + 3 < T) load(ra1, rh1, rl1, kstep(t + 3));
        compute();   // LDS: step t + 1; set 0: step t + 2; set 1: step t + 3
        __syncthreads();
        if (t + 2 < T) {
          store(ra0, rh0, rl0);
          __syncthreads();
          if (t + 4 < T) load(ra0, rh0, rl0, kstep(t + 4));
        }
      }
    }
  }
  if (want_sq) {   // block sum in fixed order -> sq[blockIdx.x + gridDim.x blockIdx.z]
    __shared__ double red[256];
    red[tid] = xsq;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) sq[blockIdx.x + (int64_t)gridDim.x * blockIdx.z] = red[0];
  }
  // D[i][j] of a 32x32 tile: lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (SBN / WN) + b * 32 + l32;
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int il = (x >> 2) * 8 + half * 4 + (x & 3);
        const int64_t gi = i0 + wm * (SBM / WM) + a * 32 + il;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][x];
      }
    }
}

// Wide thin operands (64 < N <= 256): 512 threads over a 256 x 256 tile of C,
// eight waves of 64 x 128 (2 x 4 blocks of 32 x 32) sharing one B tile, 32-deep
// K steps, two waves per SIMD.  LDS holds two stages (2 x 64 KB): the split of
// step t + 1 is staged into one while step t is read from the other, with one
// barrier per step, so the staging work of a wave overlaps the MFMAs of the
// other wave on its SIMD.  Rows of 32 halves (64 bytes) carry no padding; the
// 16-byte chunk c of row i sits at chunk c ^ swz(i), swz(i) = ((i >> 2) ^
// (i >> 4)) & 3, which keeps the fragment reads (16 consecutive rows, one
// chunk) and the staging stores free of bank conflicts.  Two register sets
// carry the next two K steps (one step of lookahead does not cover the load
// latency at full HBM load).  Loads are unconditional from clamped addresses
// (guarded loads become exec-masked blocks whose waits serialise them);
// out-of-range elements are zeroed when a step is staged.  The split, the K
// rotation and the output are those of gemm_split_kernel.
constexpr int WBM = 256, WBN = 256, WNT = 512, WBK = 32;
NMF_DEV int swz(int i) { return ((i >> 2) ^ (i >> 4)) & 3; }
// halves offset of element (i, k) of a 32-wide swizzled tile
NMF_DEV int sw_at(int i, int k) { return i * WBK + ((((k >> 3) ^ swz(i)) << 3) | (k & 7)); }
template <bool AT>
__global__ void __launch_bounds__(WNT)
gemm_split_wide_kernel(const float* __restrict__ X, int64_t ldx, const uint16_t* __restrict__ BtH,
                       const uint16_t* __restrict__ BtL, int64_t ldbt, float* __restrict__ C, int64_t ldc,
                       int64_t M, int64_t N, int64_t K, int64_t kchunk, int rot_xcd, double* __restrict__ sq) {
  constexpr int WN = 2;
  constexpr int TM = 2, TN = WBN / WN / 32;        // 64 x 128 per wave
  constexpr int XE = WBM * WBK / WNT;              // X elements per thread (16)
  constexpr int AV = XE / 4;                       // float4 loads of X per thread
  constexpr int BV = WBN * WBK / 8 / WNT;          // 16-byte loads per thread, each of hi and lo (2)
  constexpr int STAGE = (WBM + WBN) * WBK * 2;     // halves per stage: A hi, A lo, B hi, B lo
  static_assert(XE == 16 && BV == 2, "tile shape");
  __shared__ __attribute__((aligned(16))) uint16_t lds[2 * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * WBM, n0 = (int64_t)blockIdx.y * WBN;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int x = 0; x < 16; ++x) acc[a][b][x] = 0.f;
  // at = 0: lane reads row (tid / 8) + 64 p, columns 4 (tid % 8) .. +3 of the
  // tile; at = 1: columns 4 (tid % 64) .. +3 of tile rows 4 (tid / 64) + p
  // (32-bit in-tile offsets, the launcher checks WBM ldx < 2^30)
  auto arow = [&](int p) { return !AT ? (tid >> 3) + 64 * p : 4 * (tid >> 6) + p; };
  const int acol = !AT ? 4 * (tid & 7) : 4 * (tid & 63);
  constexpr int AW = 4;                            // width of one load
  auto aoff = [&](int p) { return (uint32_t)(arow(p) * ldx + acol); };
  auto brow = [&](int p) { return (tid + WNT * p) >> 2; };
  const int bcol = 8 * (tid & 3);
  auto boff = [&](int p) {   // rows past N read row n0 (zeroed when staged)
    return (uint32_t)((n0 + brow(p) < N ? brow(p) : 0) * ldbt + bcol);
  };
  float rx0[XE], rx1[XE];   // element AW p + e: load p, lane e
  i32x4 rh0[BV], rl0[BV], rh1[BV], rl1[BV];
  auto aok = [&](int p, int e, int64_t k0) {
    return !AT ? (i0 + arow(p) < M && k0 + acol + e < kend) : (k0 + arow(p) < kend && i0 + acol + e < M);
  };
  // the tile base (uniform) lies inside X: i0 < M and k0 < kend
  auto load = [&](float* rx, i32x4* rh, i32x4* rl, int64_t k0) {
    const float* tile = !AT ? X + i0 * ldx + k0 : X + k0 * ldx + i0;
#pragma unroll
    for (int p = 0; p < AV; ++p) {
      const f32x4 v = __builtin_nontemporal_load((const f32x4*)(tile + (aok(p, 0, k0) ? aoff(p) : 0u)));
      rx[4 * p] = v[0]; rx[4 * p + 1] = v[1]; rx[4 * p + 2] = v[2]; rx[4 * p + 3] = v[3];
    }
    const uint16_t* th = BtH + n0 * ldbt + k0;   // K columns up to ldbt lie inside Bt
    const uint16_t* tl = BtL + n0 * ldbt + k0;
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      rh[p] = *(const i32x4*)(th + boff(p));
      rl[p] = *(const i32x4*)(tl + boff(p));
    }
  };
  // optional FP64 sum of squares of X (at = 0; the single column tile counts
  // every element once): ||X||^2 for free with X Q_R
  const bool want_sq = !AT && sq != nullptr;
  double xsq = 0.0;
  auto store = [&](float* rx, const i32x4* rh, const i32x4* rl, int64_t k0, int stage) {
    uint16_t* AsH = lds + stage * STAGE;
    uint16_t* AsL = AsH + WBM * WBK;
    uint16_t* BsH = AsL + WBM * WBK;
    uint16_t* BsL = BsH + WBN * WBK;
#pragma unroll
    for (int p = 0; p < AV; ++p)
#pragma unroll
      for (int e = 0; e < AW; ++e) rx[AW * p + e] = aok(p, e, k0) ? rx[AW * p + e] : 0.f;
    if (want_sq) {
#pragma unroll
      for (int x = 0; x < XE; ++x) xsq = fma((double)rx[x], (double)rx[x], xsq);
    }
    if (!AT) {
#pragma unroll
      for (int p = 0; p < AV; ++p) {
        uint32_t h0, l0, h1, l1;
        split_pk(rx[4 * p], rx[4 * p + 1], h0, l0);
        split_pk(rx[4 * p + 2], rx[4 * p + 3], h1, l1);
        *(uint2*)(AsH + sw_at(arow(p), acol)) = make_uint2(h0, h1);
        *(uint2*)(AsL + sw_at(arow(p), acol)) = make_uint2(l0, l1);
      }
    } else {
      // the four K values of tile column i = acol + d go to As[i][4 (tid / 64) ..]
      // as one 8-byte store
      const int kb = 4 * (tid >> 6);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        uint2 vh, vl;
        split_pk(rx[d], rx[4 + d], vh.x, vl.x);
        split_pk(rx[8 + d], rx[12 + d], vh.y, vl.y);
        *(uint2*)(AsH + sw_at(acol + d, kb)) = vh;
        *(uint2*)(AsL + sw_at(acol + d, kb)) = vl;
      }
    }
    const i32x4 zi = {0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const bool ok = n0 + brow(p) < N;
      *(i32x4*)(BsH + sw_at(brow(p), bcol)) = ok ? rh[p] : zi;
      *(i32x4*)(BsL + sw_at(brow(p), bcol)) = ok ? rl[p] : zi;
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  auto compute = [&](int stage) {
    const uint16_t* AsH = lds + stage * STAGE;
    const uint16_t* AsL = AsH + WBM * WBK;
    const uint16_t* BsH = AsL + WBM * WBK;
    const uint16_t* BsL = BsH + WBN * WBK;
#pragma unroll
    for (int ks = 0; ks < WBK / 16; ++ks) {
      bf16x8 ah[TM], al[TM];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int il = wm * 64 + a * 32 + l32;
        ah[a] = *(const bf16x8*)(AsH + sw_at(il, ks * 16 + 8 * half));
        al[a] = *(const bf16x8*)(AsL + sw_at(il, ks * 16 + 8 * half));
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int jl = wn * (WBN / WN) + b * 32 + l32;
        const bf16x8 bh = *(const bf16x8*)(BsH + sw_at(jl, ks * 16 + 8 * half));
        const bf16x8 bl = *(const bf16x8*)(BsL + sw_at(jl, ks * 16 + 8 * half));
#pragma unroll
        for (int a = 0; a < TM; ++a) {   // small terms first
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh, acc[a][b], 0, 0, 0);
        }
      }
    }
  };
  const int T = kend > kbeg ? (int)ceil_div(kend - kbeg, (int64_t)WBK) : 0;
  const int wg = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int rot = T == 0 ? 0 : rot_xcd ? ((wg % 8) * T) / 8 : (int)(blockIdx.x % T);
  auto kstep = [&](int s) { return kbeg + (int64_t)((s + rot) % T) * WBK; };
  // step s is staged in stage s % 2 from register set s % 2
  if (T > 0) {
    load(rx0, rh0, rl0, kstep(0));
    if (T > 1) load(rx1, rh1, rl1, kstep(1));
    store(rx0, rh0, rl0, kstep(0), 0);
    if (T > 2) load(rx0, rh0, rl0, kstep(2));
    __syncthreads();
    for (int t = 0; t < T; t += 2) {
      // set 1: step t + 1, set 0: step t + 2
      if (t + 1 < T) store(rx1, rh1, rl1, kstep(t + 1), 1);
      if (t + 3 < T) load(rx1, rh1, rl1, kstep(t + 3));
      __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the MFMAs
      compute(0);
      __syncthreads();
      if (t + 1 < T) {
        // set 0: step t + 2, set 1: step t + 3
        if (t + 2 < T) store(rx0, rh0, rl0, kstep(t + 2), 0);
        if (t + 4 < T) load(rx0, rh0, rl0, kstep(t + 4));
        __builtin_amdgcn_sched_barrier(0);
        compute(1);
        __syncthreads();
      }
    }
  }
  if (want_sq) {   // block sum in fixed order -> sq[blockIdx.x + gridDim.x blockIdx.z]
    __shared__ double red[WNT];
    red[tid] = xsq;
    __syncthreads();
    for (int w = WNT / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) sq[blockIdx.x + (int64_t)gridDim.x * blockIdx.z] = red[0];
  }
  // D[i][j] of a 32x32 tile: lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
  float* Cz = C + (int64_t)blockIdx.z * (M * ldc);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int64_t gj = n0 + wn * (WBN / WN) + b * 32 + l32;
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int il = (x >> 2) * 8 + half * 4 + (x & 3);
        const int64_t gi = i0 + wm * 64 + a * 32 + il;
        if (gi < M && gj < N) Cz[gi * ldc + gj] = acc[a][b][x];
      }
    }
}

}  // namespace

hipError_t launch_prep_bt(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* BtH, uint16_t* BtL,
                          int64_t ldbt, hipStream_t st) {
  if (K == 0 || N == 0) return hipSuccess;
  if (ldbt % 64 || ldbt < K) return hipErrorInvalidValue;
  dim3 grid((unsigned)(ldbt / 64), (unsigned)ceil_div(N, 64));
  if (BtL)
    hipLaunchKernelGGL(prep_bt_kernel<true>, grid, dim3(256), 0, st, B, ldb, K, N, BtH, BtL, ldbt);
  else
    hipLaunchKernelGGL(prep_bt_kernel<false>, grid, dim3(256), 0, st, B, ldb, K, N, BtH, BtL, ldbt);
  return hipGetLastError();
}

int gemm_split_pick_splits(int64_t M, int64_t N, int64_t K) {
  if (N <= 128) return gemm_lp_pick_splits(M, N, round_up(K, 64), 128);
  // wide kernel: one resident workgroup per CU, so about 256 workgroups in all
  // (each split at least 512 deep, at most 64 splits)
  int64_t s = ceil_div(256, ceil_div(M, WBM));
  const int64_t kmax = round_up(K, 64) / 512;
  if (s > kmax) s = kmax;
  if (s > 64) s = 64;
  if (s < 1) s = 1;
  return (int)s;
}

int gemm_split_sq_parts(int64_t M, int64_t N, int splits) {
  return (int)(ceil_div(M, N <= 128 ? SBM : WBM) * splits);
}

hipError_t launch_gemm_split(const float* X, int64_t ldx, int at, const uint16_t* BtH, const uint16_t* BtL,
                             int64_t ldbt, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, int splits,
                             float* part, hipStream_t st, double* sq) {
  hipError_t e = launch_gemm_split_kernel(X, ldx, at, BtH, BtL, ldbt, C, ldc, M, N, K, splits, part, st, sq);
  if (e != hipSuccess || splits == 1 || M == 0 || N == 0) return e;
  return launch_splitk_reduce_lp(part, splits, C, ldc, M, N, st);
}

hipError_t launch_gemm_split_kernel(const float* X, int64_t ldx, int at, const uint16_t* BtH, const uint16_t* BtL,
                                    int64_t ldbt, float* C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                    int splits, float* part, hipStream_t st, double* sq) {
  if (M == 0 || N == 0) return hipSuccess;
  if (ldx % 4 || ldbt % 64 || ldbt < round_up(K, 64) || splits < 1) return hipErrorInvalidValue;
  const int sbn = N <= 64 ? 64 : N <= 128 ? 128 : 256;
  // 32-bit in-tile offsets: SBM (WBM) rows of X (at = 0) or SBK rows (at = 1), and SBN rows of Bt
  if ((int64_t)WBM * ldx >= (1ll << 30) || (int64_t)sbn * ldbt >= (1ll << 30)) return hipErrorInvalidValue;
  float* out = splits > 1 ? part : C;
  const int64_t ldo = splits > 1 ? N : ldc;
  const int64_t kchunk = round_up(ceil_div(K, splits), 64);
  dim3 grid((unsigned)ceil_div(M, 128), (unsigned)ceil_div(N, sbn), (unsigned)splits);
  // thin operand per split: N x kchunk values of hi and lo (4 bytes per value)
  const int rx = rot_per_xcd(N, kchunk, splits, 4);
  if (sbn == 64) {
    if (at)
      hipLaunchKernelGGL((gemm_split_kernel<true, 64>), grid, dim3(256), 0, st, X, ldx, BtH, BtL, ldbt, out, ldo,
                         M, N, K, kchunk, rx, nullptr);
    else
      hipLaunchKernelGGL((gemm_split_kernel<false, 64>), grid, dim3(256), 0, st, X, ldx, BtH, BtL, ldbt, out, ldo,
                         M, N, K, kchunk, rx, sq);
  } else if (sbn == 128) {
    if (at)
      hipLaunchKernelGGL((gemm_split_kernel<true, 128>), grid, dim3(256), 0, st, X, ldx, BtH, BtL, ldbt, out,
                         ldo, M, N, K, kchunk, rx, nullptr);
    else
      hipLaunchKernelGGL((gemm_split_kernel<false, 128>), grid, dim3(256), 0, st, X, ldx, BtH, BtL, ldbt, out,
                         ldo, M, N, K, kchunk, rx, sq);
  } else {
    const dim3 wgrid((unsigned)ceil_div(M, WBM), 1, (unsigned)splits);
    if (at)
      hipLaunchKernelGGL((gemm_split_wide_kernel<true>), wgrid, dim3(WNT), 0, st, X, ldx, BtH, BtL, ldbt, out, ldo,
                         M, N, K, kchunk, rx, nullptr);
    else
      hipLaunchKernelGGL((gemm_split_wide_kernel<false>), wgrid, dim3(WNT), 0, st, X, ldx, BtH, BtL, ldbt, out, ldo,
                         M, N, K, kchunk, rx, sq);
  }
  return hipGetLastError();
}
