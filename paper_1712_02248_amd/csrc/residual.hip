// Exact relative error e = ||X - W Ht^T||_F / ||X||_F (the objective of eq 2.2),
// evaluated directly (never through the Gram expansion, which cancels
// catastrophically at small e) with FP64 products and FP64 accumulation; and a
// faster value for stopping tests from split-BF16 products (residual_split_kernel).
//
// A workgroup owns 4 RPW rows of X (RPW per wave) and walks all 64-column tiles,
// starting at tile (workgroup index mod tile count).  Per 16-column block the
// wave forms E = Htb (W diag(sw))^T on v_mfma_f64_16x16x4_f64 (A = Ht rows from
// LDS, already FP64; B = the wave's W rows, kept in registers), with the
// block's Ht rows taken in the order c(j) = 4 (j % 4) + j / 4: E[j][i] lands in
// lane i + 16 (j % 4), register j / 4, so lane l holds row l % 16 and the four
// adjacent columns 4 (l / 16) .. +3 of the block, one float4 of X.  It
// subtracts X and accumulates squares.  Workgroup partials are summed in fixed
// order by the last workgroup to finish (completion counter, reset afterwards).
#include <algorithm>

#include "common.h"

namespace {

constexpr int RBMIN = 64;    // fewest rows per workgroup of any instantiation
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
constexpr int CT = 64;       // columns per tile

template <int RMAX, int RPW>
__global__ void __launch_bounds__(256)
residual_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                const float* __restrict__ W, const float* __restrict__ sw,
                const float* __restrict__ Ht, int r, double* __restrict__ part,
                double* __restrict__ out, unsigned* __restrict__ counter, const double* __restrict__ gate,
                double gate_thr2) {
  // gate (optional): the proxy sums (sd, sx, ||X||^2); every workgroup returns at
  // once unless (||X||^2 - sx + sd) / ||X||^2 <= gate_thr2 (out is left untouched)
  if (gate) {
    const double e2 = (gate[2] - gate[1] + gate[0]) / gate[2];
    if (!(e2 <= gate_thr2)) return;
  }
  constexpr int RB = 4 * RPW, NB = RPW / 16;  // rows per workgroup, 16-row blocks per wave
  constexpr int KS = RMAX / 4;                // MFMA k-steps
  constexpr int HPT = CT * RMAX / 256;        // Ht tile elements per thread
  typedef double T;
  typedef f64x4 TV;
  __shared__ T Hs[CT][RMAX + 1];
  __shared__ double red[2][256];
  __shared__ int last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * RB;
  const int64_t ntile = ceil_div(n, CT);
  const bool vec = (ldx % 4 == 0) && (((uintptr_t)X & 15) == 0);   // float4 loads of X

  // B fragments (rows of W diag(sw) owned by this wave), kept for all tiles
  // (all loads issued first, unconditionally from clamped addresses, and
  // converted after: guarded loads serialise on their waits)
  T wfr[NB][KS];
  {
    float wv[NB][KS], sv[KS];
    const float* swp = sw ? sw : W;   // a valid address either way
#pragma unroll
    for (int s = 0; s < KS; ++s) sv[s] = swp[4 * s + (lane >> 4) < r ? 4 * s + (lane >> 4) : 0];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t gi = row0 + wave * RPW + nb * 16 + (lane & 15);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + (lane >> 4);
        wv[nb][s] = W[(gi < m && k < r) ? gi * r + k : 0];
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t gi = row0 + wave * RPW + nb * 16 + (lane & 15);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int k = 4 * s + (lane >> 4);
        wfr[nb][s] = (gi < m && k < r) ? (T)wv[nb][s] * (T)(sw ? sv[s] : 1.f) : (T)0;
      }
    }
  }
  // Ht rows in the order c(j) = 4 (j % 4) + j / 4
  const int hrow = 4 * (lane & 3) + ((lane & 15) >> 2);
  // Software pipeline over the 64-column tiles of this row strip: the loads of
  // tile t+1 are issued (Ht first, then X) before the MFMAs of tile t, so each
  // wait only covers loads issued one tile earlier.  n % 4 == 0, so a group of
  // four columns is either inside or outside.  Loads are unconditional from
  // clamped addresses and out-of-range values are zeroed when the tile is used
  // (guarded loads become exec-masked blocks whose waits serialise them).
  float hv[HPT];
  f32x4 xv[NB][4];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  auto load_h = [&](int64_t c0) {
#pragma unroll
    for (int p = 0; p < HPT; ++p) {
      const int e = tid + 256 * p, jj = e / RMAX, k = e % RMAX;
      hv[p] = Ht[(c0 + jj < n && k < r) ? (c0 + jj) * r + k : 0];
    }
  };
  auto load_x = [&](int64_t c0) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) {
        const int64_t gi = row0 + wave * RPW + nb * 16 + (lane & 15);
        const int64_t gj = c0 + sub * 16 + 4 * (lane >> 4);
        const float* src = X + ((gi < m && gj < n) ? gi * ldx + gj : 0);
        if (vec) xv[nb][sub] = *(const f32x4*)src;
        else xv[nb][sub] = (f32x4){src[0], src[1], src[2], src[3]};
      }
  };
  // workgroups start at different column tiles (rotated order) so that
  // concurrent loads of X spread over the HBM channels
  const int64_t rot = (int64_t)blockIdx.x % ntile;
  auto col0 = [&](int64_t t) { return ((t + rot) % ntile) * CT; };
  double res = 0.0, xx = 0.0;
  load_h(col0(0));
  load_x(col0(0));
  for (int64_t t = 0; t < ntile; ++t) {
    __syncthreads();   // readers of the previous Hs are done
    const int64_t c0 = col0(t);
#pragma unroll
    for (int p = 0; p < HPT; ++p) {
      const int e = tid + 256 * p, jj = e / RMAX, k = e % RMAX;
      Hs[jj][k] = (c0 + jj < n && k < r) ? (T)hv[p] : (T)0;
    }
    __syncthreads();
    f32x4 xc[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) {
        const int64_t gi = row0 + wave * RPW + nb * 16 + (lane & 15);
        const int64_t gj = c0 + sub * 16 + 4 * (lane >> 4);
        xc[nb][sub] = (gi < m && gj < n) ? xv[nb][sub] : z4;
      }
    if (t + 1 < ntile) {
      load_h(col0(t + 1));
      load_x(col0(t + 1));
    }
    TV d[NB][4];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) d[nb][sub] = (TV){0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + (lane >> 4);
#pragma unroll
      for (int sub = 0; sub < 4; ++sub) {
        const T h = Hs[sub * 16 + hrow][k];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          d[nb][sub] = __builtin_amdgcn_mfma_f64_16x16x4f64(h, wfr[nb][s], d[nb][sub], 0, 0, 0);
      }
    }
    // lane: row i = lane % 16 of block nb, tile columns 16 sub + 4 (lane / 16) + q in
    // register q; out-of-range entries are 0 - 0
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int sub = 0; sub < 4; ++sub)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double x = (double)xc[nb][sub][q];
          const double df = x - d[nb][sub][q];
          res = fma(df, df, res);
          xx = fma(x, x, xx);
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
  const int nblk = gridDim.x;
  const int bid = blockIdx.x;
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


// Sketch-only proxy of the residual (Sec 3: Q_L Q_L^T X approximates X):
//   e_p^2 = (||X||^2 - ||Xh||^2 + sum_j ||xh_j - Wh h_j||^2) / ||X||^2,
// exact when the columns of W lie in range(Q_L).  Per row j of Xh (n x k') and
// Ht (n x r): lane c (and c + 64, ... up to k') forms
// d_c = xh_jc - sum_l Wh[c][l] h_jl, l ascending, in FP64.  Wh is staged
// transposed (whs[l][c], row stride kpp = k' rounded up to 64, zero padded) so
// the lanes of a wave read consecutive words; a wave takes four rows at once
// (their rows of Ht staged in LDS), so each value of Wh read serves four rows.
// Block partials (two FP64 sums) go to part[2 blockIdx.x + {0, 1}].
__global__ void __launch_bounds__(256)
proxy_kernel(const float* __restrict__ Xh, int64_t ldx, const float* __restrict__ Ht, int r,
             const float* __restrict__ Wh, int kp, int64_t n, double* __restrict__ part) {
  constexpr int RW = 4;                          // rows per wave and pass
  extern __shared__ float whs[];                 // r x kpp
  __shared__ double red[2][256];
  __shared__ float hrow[4][RW][128];             // the wave's rows of Ht (r <= 128)
  const int kpp = (kp + 63) & ~63, nt = kpp >> 6;
  for (int e = threadIdx.x; e < kpp * r; e += 256) {
    const int l = e / kpp, c = e - l * kpp;
    whs[e] = c < kp ? Wh[c * r + l] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sd = 0.0, sx = 0.0;
  const int64_t step = (int64_t)gridDim.x * 4 * RW;
  for (int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * RW; row0 < n; row0 += step) {
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int64_t row = row0 + q < n ? row0 + q : n - 1;   // rows past n: a copy, not summed
      hrow[wave][q][lane] = lane < r ? Ht[row * r + lane] : 0.f;
      hrow[wave][q][lane + 64] = lane + 64 < r ? Ht[row * r + lane + 64] : 0.f;
    }
    double acc[RW][4];
#pragma unroll
    for (int q = 0; q < RW; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[q][t] = 0.0;
    for (int l = 0; l < r; ++l) {
      double w[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = t < nt ? (double)whs[l * kpp + 64 * t + lane] : 0.0;
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        const double hl = (double)hrow[wave][q][l];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[q][t] += w[t] * hl;
      }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      if (row0 + q >= n) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 64 * t + lane;
        if (c < kp) {
          const double x = Xh[(row0 + q) * ldx + c];
          const double d = x - acc[q][t];
          sd += d * d;
          sx += x * x;
        }
      }
    }
  }
  red[0][threadIdx.x] = sd;
  red[1][threadIdx.x] = sx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
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

// ------------------------------------------------------------------- split
// Residual for a stopping test on split-BF16 products: P = (W diag(sw)) Ht^T
// from hi hi + hi lo + lo hi of the BF16 splits (v = hi + lo, hi = bf16(v),
// lo = bf16(v - hi)), FP32 accumulation on v_mfma_f32_32x32x16_bf16, E = X - P
// in FP32, squares summed in FP64.  For W, Ht >= 0 the result lies within
// g (1 + e) + u' e of the exact e (g from the representation, 3.03 2^-16 per
// product, the scaling of W, and 3 KR FP32 additions per element; the host
// states the bound).  The splits are formed once per call (split_rows_kernel).
//
// A workgroup of 512 threads owns 256 rows of X (32 per wave) and walks all
// 64-column tiles from a rotated start; each wave keeps the A fragments of its
// rows (W splits, all KR columns) in registers.  The hi and lo splits of the
// tile's 64 rows of Ht go through LDS (two stages, rows padded by 8 halves: the
// 16-byte fragment reads are free of bank conflicts), the next tile's splits
// and X values are loaded while the current tile is consumed, one barrier per
// tile.  Loads are unconditional from clamped addresses, values outside the
// matrices zeroed after.

// hi and lo BF16 splits of A diag(scale) (rows x r, lda), zero from column r
// to KR (ld KR).
__global__ void __launch_bounds__(256)
split_rows_kernel(const float* __restrict__ A, int64_t lda, const float* __restrict__ scale, int64_t rows, int r,
                  int KR, uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const int64_t total = rows * (KR / 2);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / (KR / 2);
    const int k = 2 * (int)(e % (KR / 2));
    float v[2];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const bool ok = k + d < r;
      const float a = A[ok ? i * lda + k + d : 0];
      const float sc = scale ? scale[ok ? k + d : 0] : 1.f;
      v[d] = ok ? a * sc : 0.f;
    }
    const f32x2 pv = {v[0], v[1]};
    const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(pv, bf16x2));
    const f32x2 rv = {v[0] - __builtin_bit_cast(float, h << 16), v[1] - __builtin_bit_cast(float, h & 0xFFFF0000u)};
    const uint32_t l = __builtin_bit_cast(uint32_t, __builtin_convertvector(rv, bf16x2));
    *(uint32_t*)(hi + i * KR + k) = h;
    *(uint32_t*)(lo + i * KR + k) = l;
  }
}

template <int KR>
__global__ void __launch_bounds__(512)
residual_split_kernel(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                      const uint16_t* __restrict__ Wh, const uint16_t* __restrict__ Wl,
                      const uint16_t* __restrict__ Hh, const uint16_t* __restrict__ Hl, double* __restrict__ part,
                      double* __restrict__ out, unsigned* __restrict__ counter, const double* __restrict__ gate,
                      double gate_thr2, int64_t sstep) {
  if (gate) {   // as in residual_kernel: every workgroup returns unless the proxy is within the gate
    const double e2 = (gate[2] - gate[1] + gate[0]) / gate[2];
    if (!(e2 <= gate_thr2)) return;
  }
  constexpr int CT = 64, HROW = KR + 8, KS = KR / 16;
  constexpr int HV = CT * KR / 8 / 512;          // 16-byte loads of each split per thread
  static_assert(HV >= 1, "KR >= 64");
  __shared__ __attribute__((aligned(16))) uint16_t Hs[2][2][CT * HROW];
  __shared__ double red[2][512];
  __shared__ int last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  // this wave's 32 rows of strip blockIdx.x * sstep (every sstep-th 256-row strip)
  const int64_t row0 = (int64_t)blockIdx.x * sstep * 256 + 32 * wave;
  const int64_t ntile = ceil_div(n, CT);
  // A fragments: lane holds W[row0 + l32][16 ks + 8 half .. +7] (hi, lo)
  bf16x8 ah[KS], al[KS];
  {
    const int64_t wr = row0 + l32 < m ? row0 + l32 : 0;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      ah[ks] = *(const bf16x8*)(Wh + wr * KR + 16 * ks + 8 * half);
      al[ks] = *(const bf16x8*)(Wl + wr * KR + 16 * ks + 8 * half);
    }
    if (row0 + l32 >= m) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ah[ks] = al[ks] = (bf16x8){};
    }
  }
  // Ht splits of a tile: thread loads 16 bytes at row (tid + 512 p) / (KR / 8),
  // chunk (tid + 512 p) % (KR / 8) of each split (rows past n read row 0)
  i32x4 hh[HV], hl[HV];
  auto loadH = [&](int64_t c0) {
#pragma unroll
    for (int p = 0; p < HV; ++p) {
      const int f = tid + 512 * p, jr = f / (KR / 8), ch = f % (KR / 8);
      const int64_t j = c0 + jr < n ? c0 + jr : 0;
      hh[p] = *(const i32x4*)(Hh + j * KR + 8 * ch);
      hl[p] = *(const i32x4*)(Hl + j * KR + 8 * ch);
    }
  };
  auto storeH = [&](int64_t c0, int b) {
    const i32x4 zi = {0, 0, 0, 0};
#pragma unroll
    for (int p = 0; p < HV; ++p) {
      const int f = tid + 512 * p, jr = f / (KR / 8), ch = f % (KR / 8);
      const bool ok = c0 + jr < n;
      *(i32x4*)(&Hs[b][0][jr * HROW + 8 * ch]) = ok ? hh[p] : zi;
      *(i32x4*)(&Hs[b][1][jr * HROW + 8 * ch]) = ok ? hl[p] : zi;
    }
  };
  // X in the output layout of a 32 x 32 block: register x holds row
  // 8 (x / 4) + 4 half + x % 4, column l32 (two column blocks per tile)
  float xv[2][16];
  auto xrow = [&](int x) { return row0 + 8 * (x >> 2) + 4 * half + (x & 3); };
  auto loadX = [&](int64_t c0) {
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int64_t i = xrow(x), j = c0 + 32 * cb + l32;
        xv[cb][x] = X[(i < m && j < n) ? i * ldx + j : 0];
      }
  };
  // column part blockIdx.y of gridDim.y: tiles tbeg .. tbeg + nt - 1, from a rotated start
  const int tbeg = (int)((int64_t)blockIdx.y * ntile / gridDim.y);
  const int nt = (int)(((int64_t)blockIdx.y + 1) * ntile / gridDim.y) - tbeg;
  const int rot = nt > 0 ? (int)(blockIdx.x % (unsigned)nt) : 0;
  auto col0 = [&](int t) { return (int64_t)(tbeg + (t + rot) % nt) * CT; };
  double res = 0.0, xx = 0.0;
  if (nt > 0) {
    loadH(col0(0));
    loadX(col0(0));
    storeH(col0(0), 0);
  }
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int64_t c0 = col0(t);
    float xc[2][16];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        const int64_t i = xrow(x), j = c0 + 32 * cb + l32;
        xc[cb][x] = (i < m && j < n) ? xv[cb][x] : 0.f;
      }
    if (t + 1 < nt) {
      loadH(col0(t + 1));
      loadX(col0(t + 1));
    }
    __builtin_amdgcn_sched_barrier(0);   // the next tile's loads stay ahead of the MFMAs
    const int b = (int)(t & 1);
    f32x16 d[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) d[cb][e] = 0.f;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int jl = 32 * cb + l32;
        const bf16x8 bh = *(const bf16x8*)(&Hs[b][0][jl * HROW + 16 * ks + 8 * half]);
        const bf16x8 bl = *(const bf16x8*)(&Hs[b][1][jl * HROW + 16 * ks + 8 * half]);
        d[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ks], bh, d[cb], 0, 0, 0);   // small terms first
        d[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ks], bl, d[cb], 0, 0, 0);
        d[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ks], bh, d[cb], 0, 0, 0);
      }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int x = 0; x < 16; ++x) {   // out-of-range entries are 0 - 0
        const double df = (double)(xc[cb][x] - d[cb][x]);
        res = fma(df, df, res);
        xx = fma((double)xc[cb][x], (double)xc[cb][x], xx);
      }
    if (t + 1 < nt) storeH(col0(t + 1), b ^ 1);   // that stage was last read before the previous barrier
    __syncthreads();
  }
  red[0][tid] = res;
  red[1][tid] = xx;
  __syncthreads();
  for (int w = 256; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  const int nblk = gridDim.x * gridDim.y;
  const int bid = blockIdx.x + gridDim.x * blockIdx.y;
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
  for (int q = tid; q < nblk; q += 512) {
    a0 += vp[2 * q];
    a1 += vp[2 * q + 1];
  }
  red[0][tid] = a0;
  red[1][tid] = a1;
  __syncthreads();
  for (int w = 256; w > 0; w >>= 1) {
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

int residual_blocks(int64_t m, int64_t n) {   // upper bound over the instantiations
  (void)n;
  return (int)ceil_div(m, RBMIN);
}

hipError_t launch_residual(const float* X, int64_t ldx, int64_t m, int64_t n, const float* W,
                           const float* sw, const float* Ht, int r, double* part, double* out,
                           unsigned* counter, hipStream_t st, const double* gate, double gate_thr2) {
  if (n % 4) return hipErrorInvalidValue;
  // 32 rows per wave (each Ht fragment feeds two MFMA row blocks) while the W
  // fragments fit; 16 for larger r
#define NMF_RES_LAUNCH(RM_, RPW_)                                                                              \
  hipLaunchKernelGGL((residual_kernel<RM_, RPW_>), dim3((unsigned)ceil_div(m, 4 * RPW_)), dim3(256), 0, st, X, ldx, \
                     m, n, W, sw, Ht, r, part, out, counter, gate, gate_thr2)
  if (r <= 16) NMF_RES_LAUNCH(16, 32);
  else if (r <= 32) NMF_RES_LAUNCH(32, 32);
  else if (r <= 64) NMF_RES_LAUNCH(64, 16);
  else if (r <= 128) NMF_RES_LAUNCH(128, 16);
  else return hipErrorInvalidValue;
#undef NMF_RES_LAUNCH
  return hipGetLastError();
}

int proxy_blocks(int64_t n) {
  int64_t b = ceil_div(n, 16);   // four waves of four rows
  return (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
}

hipError_t launch_proxy(const float* Xh, int64_t ldx, const float* Ht, int r, const float* Wh, int kp, int64_t n,
                        double* part, hipStream_t st) {
  if (kp > 256 || r > 128) return hipErrorInvalidValue;
  const size_t lds = (size_t)((kp + 63) & ~63) * r * sizeof(float);
  hipLaunchKernelGGL(proxy_kernel, dim3(proxy_blocks(n)), dim3(256), lds, st, Xh, ldx, Ht, r, Wh, kp, n, part);
  return hipGetLastError();
}

int residual_split_kr(int r) { return r <= 64 ? 64 : r <= 128 ? 128 : 0; }

size_t residual_split_halves(int64_t m, int64_t n, int r) {
  const int KR = residual_split_kr(r);
  return KR ? (size_t)2 * (m + n) * KR : 0;
}

hipError_t launch_residual_split(const float* X, int64_t ldx, int64_t m, int64_t n, const float* W, const float* sw,
                                 const float* Ht, int r, uint16_t* ws, double* part, double* out, unsigned* counter,
                                 hipStream_t st, const double* gate, double gate_thr2, int64_t sstep) {
  const int KR = residual_split_kr(r);
  if (sstep < 1) return hipErrorInvalidValue;
  if (!KR || m == 0 || n == 0) return hipErrorInvalidValue;
  uint16_t* Wh = ws;
  uint16_t* Wl = Wh + m * KR;
  uint16_t* Hh = Wl + m * KR;
  uint16_t* Hl = Hh + n * KR;
  auto grid = [&](int64_t rows) { return dim3((unsigned)std::min<int64_t>(ceil_div(rows * (KR / 2), 256), 8192)); };
  hipLaunchKernelGGL(split_rows_kernel, grid(m), dim3(256), 0, st, W, (int64_t)r, sw, m, r, KR, Wh, Wl);
  hipLaunchKernelGGL(split_rows_kernel, grid(n), dim3(256), 0, st, Ht, (int64_t)r, nullptr, n, r, KR, Hh, Hl);
  // the sample: every sstep-th strip, each split into up to sstep column parts
  // (as many workgroups as the full pass, each with a share of the columns)
  const int64_t parts = std::min<int64_t>(sstep, std::max<int64_t>(1, ceil_div(n, 64)));
  const dim3 g((unsigned)ceil_div(ceil_div(m, 256), sstep), (unsigned)parts);
  if (KR == 64)
    hipLaunchKernelGGL(residual_split_kernel<64>, g, dim3(512), 0, st, X, ldx, m, n, Wh, Wl, Hh, Hl, part, out,
                       counter, gate, gate_thr2, sstep);
  else
    hipLaunchKernelGGL(residual_split_kernel<128>, g, dim3(512), 0, st, X, ldx, m, n, Wh, Wl, Hh, Hl, part, out,
                       counter, gate, gate_thr2, sstep);
  return hipGetLastError();
}

