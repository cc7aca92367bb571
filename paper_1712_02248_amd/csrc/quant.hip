// Low-precision copies of X for the compression products (extension: BF16 and
// OCP FP8 e4m3 range-finder passes).  X (m x n FP32) is read once and written
// both as Xq (m x ldq) and as its transpose XqT (n x ldqt), so that X B and X^T B
// are both products with K-contiguous operands; padding columns are zero.
//
// BF16: round to nearest, ties to even, on the FP32 bit pattern.
// FP8 e4m3 (OCP "FN"): one power-of-two scale 2^e per 128 x 128 tile of X, e the
// smallest integer with amax(tile) <= 448 2^e (0 for an all-zero tile); codes are
// x 2^-e rounded to nearest even with saturation to +-448.  The scale is shared
// by the tile and its transpose.
#include "common.h"

namespace {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// (a, b) -> packed BF16 pair (a in the low half) by the hardware conversion,
// round to nearest even
NMF_DEV uint32_t bf16_pk_rne(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

NMF_DEV uint16_t bf16_rne(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// e4m3 code of y (|y| <= 448 after scaling), round to nearest even, saturating.
NMF_DEV uint8_t e4m3_rne(float y) {
  uint32_t u = __builtin_bit_cast(uint32_t, y);
  const uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  float a = fabsf(y);
  if (!(a == a)) return (uint8_t)(sign | 0x7F);          // NaN
  if (a >= 464.0f) return (uint8_t)(sign | 0x7E);        // beyond the rounding midpoint: saturate to 448
  // subnormal grid spacing 2^-9 below 2^-6; normal spacing 2^(e-3)
  int e;
  frexpf(a, &e);                                         // a = f 2^e, f in [0.5, 1)
  int ex = e - 1;                                        // a in [2^ex, 2^(ex+1))
  if (ex < -6) ex = -6;
  const float spacing = ldexpf(1.0f, ex - 3);
  float qv = rintf(a / spacing) * spacing;               // exact: power-of-two spacing
  if (qv > 448.0f) qv = 448.0f;
  if (qv == 0.0f) return sign;
  int qe;
  const float qf = frexpf(qv, &qe);                      // qv = qf 2^qe
  int E = qe - 1 + 7;                                    // biased exponent
  uint32_t mant;
  if (E <= 0) {                                          // subnormal: qv = m 2^-9
    E = 0;
    mant = (uint32_t)(qv * 512.0f);
  } else {
    mant = (uint32_t)((qf * 2.0f - 1.0f) * 8.0f);
  }
  return (uint8_t)(sign | (E << 3) | mant);
}


// FP64 block sum of a per-thread value into sq[blockIdx.x + gridDim.x blockIdx.y]
// (fixed order): the sum of squares of the elements of X a block reads.
NMF_DEV void block_sq(double v, double* __restrict__ sq) {
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sq[blockIdx.x + (int64_t)gridDim.x * blockIdx.y] = red[0];
}

constexpr int QT = 64;   // transpose tile

// BF16 copy and transposed copy, 64 x 64 tiles through LDS.
__global__ void __launch_bounds__(256)
quant_bf16_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                  uint16_t* __restrict__ Xq, int64_t ldq, uint16_t* __restrict__ XqT, int64_t ldqt,
                  double* __restrict__ sq) {
  __shared__ uint16_t T[QT][QT + 2];
  const int64_t i0 = (int64_t)blockIdx.y * QT, j0 = (int64_t)blockIdx.x * QT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  uint16_t v[16];
  double ssq = 0.0;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int ii = ty + 4 * p;
    const int64_t gi = i0 + ii, gj = j0 + tx;
    const float x = (gi < m && gj < n) ? X[gi * ldx + gj] : 0.f;
    ssq = fma((double)x, (double)x, ssq);
    v[p] = bf16_rne(x);
  }
  if (sq) block_sq(ssq, sq);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int ii = ty + 4 * p;
    const int64_t gi = i0 + ii, gj = j0 + tx;
    if (gi < m && gj < ldq) Xq[gi * ldq + gj] = v[p];
    T[ii][tx] = v[p];
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int jj = ty + 4 * p;
    const int64_t gj = j0 + jj, gi = i0 + tx;
    if (gj < n && gi < ldqt) XqT[gj * ldqt + gi] = T[tx][jj];
  }
}

// BF16 copy and transposed copy over 128 x 128 tiles (n % 4 == 0, ldx % 4 == 0,
// X 16-byte aligned).  Each thread converts two rows x four columns per pass
// (float4 loads, 8-byte stores of Xq); the pairs are packed into 32-bit LDS
// words of the transposed tile, which is written out as 8-byte runs of XqT.
constexpr int QV = 128;
__global__ void __launch_bounds__(256)
quant_bf16_v4_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                     uint16_t* __restrict__ Xq, int64_t ldq, uint16_t* __restrict__ XqT, int64_t ldqt,
                     double* __restrict__ sq) {
  __shared__ uint32_t T[QV][QV / 2 + 1];          // T[j][i/2] = (bf16 x[i][j], bf16 x[i+1][j])
  const int64_t i0 = (int64_t)blockIdx.y * QV, j0 = (int64_t)blockIdx.x * QV;
  const int l = threadIdx.x & 31, rp = threadIdx.x >> 5;
  const int64_t gj = j0 + 4 * l;
  const bool colok = gj < n;                       // n % 4 == 0: all four columns or none
  f32x4 v[16];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t gi = i0 + 2 * (rp + 8 * p) + h;
      f32x4 z = {0.f, 0.f, 0.f, 0.f};
      v[2 * p + h] = (colok && gi < m) ? *(const f32x4*)(X + gi * ldx + gj) : z;
    }
  }
  if (sq) {
    double ssq = 0.0;
#pragma unroll
    for (int p = 0; p < 16; ++p)
#pragma unroll
      for (int d = 0; d < 4; ++d) ssq = fma((double)v[p][d], (double)v[p][d], ssq);
    block_sq(ssq, sq);
  }
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int ip = rp + 8 * p;                      // row pair within the tile
    uint16_t b[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int d = 0; d < 4; ++d) b[h][d] = bf16_rne(v[2 * p + h][d]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t gi = i0 + 2 * ip + h;
      if (gi < m && gj < ldq) {
        uint2 w;
        w.x = (uint32_t)b[h][0] | ((uint32_t)b[h][1] << 16);
        w.y = (uint32_t)b[h][2] | ((uint32_t)b[h][3] << 16);
        *(uint2*)(Xq + gi * ldq + gj) = w;
      }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d) T[4 * l + d][ip] = (uint32_t)b[0][d] | ((uint32_t)b[1][d] << 16);
  }
  __syncthreads();
  // XqT row j0 + jj, columns i0 + 4 l .. i0 + 4 l + 3
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int jj = rp + 8 * p;
    const int64_t gjt = j0 + jj, gi = i0 + 4 * l;
    if (gjt < n && gi < ldqt) {
      uint2 w;
      w.x = T[jj][2 * l];
      w.y = T[jj][2 * l + 1];
      *(uint2*)(XqT + gjt * ldqt + gi) = w;
    }
  }
}

// Per-tile power-of-two exponents of X (128 x 128 tiles): one workgroup per tile.
__global__ void __launch_bounds__(256)
tile_exp_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, int* __restrict__ E,
                int tiles_n) {
  __shared__ float red[256];
  const int64_t i0 = (int64_t)blockIdx.y * 128, j0 = (int64_t)blockIdx.x * 128;
  float amax = 0.f;
  for (int e = threadIdx.x; e < 128 * 128; e += 256) {
    const int ii = e / 128, jj = e % 128;
    const int64_t gi = i0 + ii, gj = j0 + jj;
    if (gi < m && gj < n) amax = fmaxf(amax, fabsf(X[gi * ldx + gj]));
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float a = red[0];
    int e = 0;
    if (a > 0.f) {
      // smallest e with a <= 448 2^e (exact comparisons with power-of-two factors)
      int fe;
      frexpf(a / 448.0f, &fe);
      e = fe - 1;
      while (a > ldexpf(448.0f, e)) ++e;
      while (a <= ldexpf(448.0f, e - 1)) --e;
    }
    E[blockIdx.y * tiles_n + blockIdx.x] = e;
  }
}

// FP8 codes of X and of its transpose, with the tile exponents.
__global__ void __launch_bounds__(256)
quant_fp8_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                 const int* __restrict__ E, int tiles_n, uint8_t* __restrict__ Xq, int64_t ldq,
                 uint8_t* __restrict__ XqT, int64_t ldqt, double* __restrict__ sq) {
  __shared__ uint8_t T[QT][QT + 4];
  const int64_t i0 = (int64_t)blockIdx.y * QT, j0 = (int64_t)blockIdx.x * QT;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int e = E[(i0 / 128) * tiles_n + (j0 / 128)];    // 64-tiles nest inside 128-tiles
  const float s = ldexpf(1.0f, -e);
  uint8_t v[16];
  double ssq = 0.0;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int ii = ty + 4 * p;
    const int64_t gi = i0 + ii, gj = j0 + tx;
    const float x = (gi < m && gj < n) ? X[gi * ldx + gj] : 0.f;
    ssq = fma((double)x, (double)x, ssq);
    v[p] = (gi < m && gj < n) ? e4m3_rne(x * s) : (uint8_t)0;
  }
  if (sq) block_sq(ssq, sq);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int ii = ty + 4 * p;
    const int64_t gi = i0 + ii, gj = j0 + tx;
    if (gi < m && gj < ldq) Xq[gi * ldq + gj] = v[p];
    T[ii][tx] = v[p];
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int jj = ty + 4 * p;
    const int64_t gj = j0 + jj, gi = i0 + tx;
    if (gj < n && gi < ldqt) XqT[gj * ldqt + gi] = T[tx][jj];
  }
}


// B -> Bt in e4m3 with one power-of-two scale per 128-row block of B (shared by
// all columns): Ebt[kb] = smallest e with amax(B[128 kb .. 128 kb + 127, :]) <= 448 2^e.
__global__ void __launch_bounds__(256)
prep_b_fp8_exp_kernel(const float* __restrict__ B, int64_t ldb, int64_t K, int64_t N, int* __restrict__ Ebt) {
  __shared__ float red[256];
  const int64_t k0 = (int64_t)blockIdx.x * 128;
  float amax = 0.f;
  for (int64_t e = threadIdx.x; e < 128 * N; e += 256) {
    const int64_t k = k0 + e / N, j = e % N;
    if (k < K) amax = fmaxf(amax, fabsf(B[k * ldb + j]));
  }
  red[threadIdx.x] = amax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float a = red[0];
    int e = 0;
    if (a > 0.f) {
      int fe;
      frexpf(a / 448.0f, &fe);
      e = fe - 1;
      while (a > ldexpf(448.0f, e)) ++e;
      while (a <= ldexpf(448.0f, e - 1)) --e;
    }
    Ebt[blockIdx.x] = e;
  }
}

__global__ void __launch_bounds__(256)
prep_b_fp8_kernel(const float* __restrict__ B, int64_t ldb, int64_t K, int64_t N,
                  const int* __restrict__ Ebt, uint8_t* __restrict__ Bt, int64_t ldbt) {
  const int64_t total = N * ldbt;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ldbt, k = e - j * ldbt;
    uint8_t v = 0;
    if (k < K) v = e4m3_rne(B[k * ldb + j] * ldexpf(1.0f, -Ebt[k / 128]));
    Bt[e] = v;
  }
}

// Row-major BF16 copy of X only (Xq, m x ldq, zero padding columns), for runs
// whose X^T products read Xq through the transposing product kernel.  One
// workgroup per 128 x 128 tile: thread t converts columns 4 (t % 32) .. +3 of
// tile rows 16 (t / 32) .. +15, all sixteen float4 loads in flight at once;
// n % 4 == 0, X 16-byte aligned, ldq % 128 == 0.
__global__ void __launch_bounds__(256)
quant_bf16_rows_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, uint16_t* __restrict__ Xq,
                       int64_t ldq, double* __restrict__ sq) {
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 128 + 16 * (tid >> 5), gj = (int64_t)blockIdx.x * 128 + 4 * (tid & 31);
  const bool rows_in = i0 + 16 <= m;   // all sixteen rows of this thread exist
  f32x4 v[16];
  const float* src = X + i0 * ldx + gj;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    v[r] = ((rows_in || i0 + r < m) && gj < n) ? __builtin_nontemporal_load((const f32x4*)(src + r * ldx)) : z;
  }
  // all sixteen packed rows first (distinct registers), then the stores: a store
  // right after the conversion that reuses its registers waits for the one before
  uint2 o[16];
  double ssq = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int d = 0; d < 4; ++d) ssq = fma((double)v[r][d], (double)v[r][d], ssq);
    o[r] = make_uint2(bf16_pk_rne(v[r][0], v[r][1]), bf16_pk_rne(v[r][2], v[r][3]));
  }
  uint16_t* dst = Xq + i0 * ldq + gj;
  if (rows_in) {
#pragma unroll
    for (int r = 0; r < 16; ++r) *(uint2*)(dst + r * ldq) = o[r];
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r)
      if (i0 + r < m) *(uint2*)(dst + r * ldq) = o[r];
  }
  if (sq) block_sq(ssq, sq);
}

// smallest integer e with a <= 448 2^e (0 for a == 0); exact comparisons with
// power-of-two factors
NMF_DEV int e4m3_scale_exp(float a) {
  int e = 0;
  if (a > 0.f) {
    int fe;
    frexpf(a / 448.0f, &fe);
    e = fe - 1;
    while (a > ldexpf(448.0f, e)) ++e;
    while (a <= ldexpf(448.0f, e - 1)) --e;
  }
  return e;
}

// One pass over X for the FP8 copies: per 128 x 128 tile the exponent, the
// codes of X (Xq) and of X^T (XqT, through LDS), and optionally the FP64 sum
// of squares.  Grid (ldq / 128, ldqt / 128) also covers the zero padding.
// Thread t holds columns 4 (t % 32) .. +3 of tile rows 16 (t / 32) .. +15 in
// registers.  LDS word T[32 (c % 4) + c / 4][w] packs the codes of tile column c,
// rows 4 w .. 4 w + 3 (row stride 33 words: the 32 lanes of a half-wave write
// distinct banks).
__global__ void __launch_bounds__(256)
quant_fp8_fused_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, int* __restrict__ E,
                       int tiles_n, int tiles_m, uint8_t* __restrict__ Xq, int64_t ldq, uint8_t* __restrict__ XqT,
                       int64_t ldqt, double* __restrict__ sq) {
  __shared__ uint32_t T[128][33];
  __shared__ float wmax[4];
  __shared__ int sexp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c4 = tid & 31, g = tid >> 5;
  const int64_t i0 = (int64_t)blockIdx.y * 128, j0 = (int64_t)blockIdx.x * 128;
  const int64_t gj = j0 + 4 * c4;
  f32x4 v[16];
  float amax = 0.f;
  double ssq = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t gi = i0 + 16 * g + r;
    f32x4 x = {0.f, 0.f, 0.f, 0.f};
    if (gi < m && gj < n) x = __builtin_nontemporal_load((const f32x4*)(X + gi * ldx + gj));   // n % 4 == 0
    v[r] = x;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      amax = fmaxf(amax, fabsf(x[d]));
      ssq = fma((double)x[d], (double)x[d], ssq);
    }
  }
  for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
  if (lane == 0) wmax[wave] = amax;
  __syncthreads();
  if (tid == 0) {
    const int e = e4m3_scale_exp(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
    sexp = e;
    if ((int)blockIdx.y < tiles_m && (int)blockIdx.x < tiles_n) E[blockIdx.y * tiles_n + blockIdx.x] = e;
  }
  if (sq) block_sq(ssq, sq);
  __syncthreads();
  const float s = ldexpf(1.0f, -sexp);
  uint32_t code[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t gi = i0 + 16 * g + r;
    uint32_t w = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) w |= (uint32_t)e4m3_rne(v[r][d] * s) << (8 * d);   // padding: code of 0 is 0
    code[r] = w;
    if (gi < m) *(uint32_t*)(Xq + gi * ldq + gj) = w;
  }
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t w = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) w |= ((code[4 * b + k] >> (8 * d)) & 0xFFu) << (8 * k);
      T[32 * d + c4][4 * g + b] = w;
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jr = (tid >> 3) + 32 * q, w4 = 4 * (tid & 7);
    const int tr = 32 * (jr & 3) + (jr >> 2);
    if (j0 + jr < n) {
      const i32x4 o = {(int)T[tr][w4], (int)T[tr][w4 + 1], (int)T[tr][w4 + 2], (int)T[tr][w4 + 3]};
      *(i32x4*)(XqT + (j0 + jr) * ldqt + i0 + 4 * w4) = o;
    }
  }
}

// B -> Bt in e4m3 for N <= 256 in one launch: one workgroup per 128-row block of
// B (its exponent Ebt[block] as above from all N columns, then the transposed
// codes).  Wave w loads rows 32 w .. 32 w + 31 of the block, lane l columns
// 4 l .. 4 l + 3 (one 1 KB row segment per wave and load, all 32 loads in
// flight); the codes of four consecutive rows of a column are packed into one
// word of T[c][w4] (rows 4 w4 .. 4 w4 + 3; row stride 33 words), and eight
// threads per column store its 128 codes as 16-byte chunks.
template <bool VEC>
__global__ void __launch_bounds__(256)
prep_bt_fp8_kernel(const float* __restrict__ B, int64_t ldb, int64_t K, int64_t N, int* __restrict__ Ebt,
                   uint8_t* __restrict__ Bt, int64_t ldbt) {
  __shared__ uint32_t T[256 * 33];
  __shared__ float wmax[4];
  __shared__ int sexp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t k0 = (int64_t)blockIdx.x * 128 + 32 * wave;
  const int nn = (int)N, c0 = 4 * lane;
  f32x4 v[32];
  float amax = 0.f;
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int64_t k = k0 + i;
    f32x4 x = {0.f, 0.f, 0.f, 0.f};
    if (VEC) {
      if (k < K && c0 < nn) x = *(const f32x4*)(B + k * ldb + c0);   // N % 4 == 0
    } else {
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (k < K && c0 + d < nn) x[d] = B[k * ldb + c0 + d];
    }
    v[i] = x;
#pragma unroll
    for (int d = 0; d < 4; ++d) amax = fmaxf(amax, fabsf(x[d]));
  }
  for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
  if (lane == 0) wmax[wave] = amax;
  __syncthreads();
  if (tid == 0) {
    const int e = e4m3_scale_exp(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3])));
    sexp = e;
    Ebt[blockIdx.x] = e;
  }
  __syncthreads();
  const float s = ldexpf(1.0f, -sexp);
#pragma unroll
  for (int d = 0; d < 4; ++d)
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      uint32_t w = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) w |= (uint32_t)e4m3_rne(v[4 * a + b][d] * s) << (8 * b);   // padding: code 0
      T[(c0 + d) * 33 + 8 * wave + a] = w;
    }
  __syncthreads();
  const int w4 = 4 * (tid & 7);
  for (int j = tid >> 3; j < nn; j += 32) {
    const uint32_t* t = T + j * 33 + w4;
    const i32x4 o = {(int)t[0], (int)t[1], (int)t[2], (int)t[3]};
    *(i32x4*)(Bt + (int64_t)j * ldbt + (int64_t)blockIdx.x * 128 + 4 * w4) = o;
  }
}

unsigned grid1(int64_t total) {
  int64_t g = ceil_div(total, 256);
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (unsigned)g;
}

}  // namespace

int quant_sq_parts(int64_t m, int64_t n, int64_t ldq, int64_t ldqt) {
  (void)n;
  (void)m;
  return (int)(ceil_div(ldq, QT) * ceil_div(ldqt, QT));   // the largest grid (64 x 64 tiles)
}

hipError_t launch_quant_bf16_rows(const float* X, int64_t ldx, int64_t m, int64_t n, uint16_t* Xq, int64_t ldq,
                                  hipStream_t st, double* sq_part, double* sq_out) {
  if (m == 0) return hipSuccess;
  if (n % 4 || ldx % 4 || ((uintptr_t)X & 15) || ((uintptr_t)Xq & 15) || ldq % 128 || ldq < n)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(ldq / 128), (unsigned)ceil_div(m, 128));
  hipLaunchKernelGGL(quant_bf16_rows_kernel, grid, dim3(256), 0, st, X, ldx, m, n, Xq, ldq,
                     sq_out ? sq_part : nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sq_out) return e;
  return launch_sum_partials_f64(sq_part, (int)(grid.x * grid.y), 1, sq_out, nullptr, st);
}

hipError_t launch_quant_bf16(const float* X, int64_t ldx, int64_t m, int64_t n, uint16_t* Xq,
                             int64_t ldq, uint16_t* XqT, int64_t ldqt, hipStream_t st, double* sq_part,
                             double* sq_out) {
  const bool vec = n % 4 == 0 && ldx % 4 == 0 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)Xq & 7) == 0 &&
                   ((uintptr_t)XqT & 7) == 0 && ldq % QV == 0 && ldqt % QV == 0;
  dim3 grid;
  double* sq = sq_out ? sq_part : nullptr;
  if (vec) {
    grid = dim3((unsigned)(ldq / QV), (unsigned)(ldqt / QV));
    hipLaunchKernelGGL(quant_bf16_v4_kernel, grid, dim3(256), 0, st, X, ldx, m, n, Xq, ldq, XqT, ldqt, sq);
  } else {
    grid = dim3((unsigned)ceil_div(ldq, QT), (unsigned)ceil_div(ldqt, QT));
    hipLaunchKernelGGL(quant_bf16_kernel, grid, dim3(256), 0, st, X, ldx, m, n, Xq, ldq, XqT, ldqt, sq);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sq_out) return e;
  return launch_sum_partials_f64(sq_part, (int)(grid.x * grid.y), 1, sq_out, nullptr, st);
}

hipError_t launch_quant_fp8(const float* X, int64_t ldx, int64_t m, int64_t n, int* E, uint8_t* Xq,
                            int64_t ldq, uint8_t* XqT, int64_t ldqt, hipStream_t st, double* sq_part,
                            double* sq_out) {
  const int tn = (int)ceil_div(n, 128), tm = (int)ceil_div(m, 128);
  const bool fused = ldq % 128 == 0 && ldqt % 128 == 0 && n % 4 == 0 && ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
  dim3 grid;
  if (fused) {   // one pass over X
    grid = dim3((unsigned)(ldq / 128), (unsigned)(ldqt / 128));
    hipLaunchKernelGGL(quant_fp8_fused_kernel, grid, dim3(256), 0, st, X, ldx, m, n, E, tn, tm, Xq, ldq, XqT,
                       ldqt, sq_out ? sq_part : nullptr);
  } else {       // tile exponents first, then the codes
    hipLaunchKernelGGL(tile_exp_kernel, dim3(tn, tm), dim3(256), 0, st, X, ldx, m, n, E, tn);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    grid = dim3((unsigned)ceil_div(ldq, QT), (unsigned)ceil_div(ldqt, QT));
    hipLaunchKernelGGL(quant_fp8_kernel, grid, dim3(256), 0, st, X, ldx, m, n, E, tn, Xq, ldq, XqT, ldqt,
                       sq_out ? sq_part : nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !sq_out) return e;
  return launch_sum_partials_f64(sq_part, (int)(grid.x * grid.y), 1, sq_out, nullptr, st);
}

hipError_t launch_prep_b_bf16(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* Bt,
                              int64_t ldbt, hipStream_t st) {
  return launch_prep_bt(B, ldb, K, N, Bt, nullptr, ldbt, st);   // tiled transpose (gemm_split.hip)
}

hipError_t launch_prep_b_fp8(const float* B, int64_t ldb, int64_t K, int64_t N, int* Ebt, uint8_t* Bt,
                             int64_t ldbt, hipStream_t st) {
  if (N <= 256 && ldbt % 128 == 0 && ((uintptr_t)Bt & 15) == 0) {
    // one launch; also sets the exponents of the zero padding blocks (0)
    const dim3 grid((unsigned)(ldbt / 128));
    if (N % 4 == 0 && ldb % 4 == 0 && ((uintptr_t)B & 15) == 0)
      hipLaunchKernelGGL(prep_bt_fp8_kernel<true>, grid, dim3(256), 0, st, B, ldb, K, N, Ebt, Bt, ldbt);
    else
      hipLaunchKernelGGL(prep_bt_fp8_kernel<false>, grid, dim3(256), 0, st, B, ldb, K, N, Ebt, Bt, ldbt);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(prep_b_fp8_exp_kernel, dim3((unsigned)ceil_div(K, 128)), dim3(256), 0, st, B, ldb, K,
                     N, Ebt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_b_fp8_kernel, dim3(grid1(N * ldbt)), dim3(256), 0, st, B, ldb, K, N, Ebt, Bt, ldbt);
  return hipGetLastError();
}
