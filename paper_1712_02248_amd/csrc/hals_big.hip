// FastHALS-RP half-steps (eq fastHALS_a) for wide factors: r up to 128 and k'
// up to 256, where the compressed factor C (k' x r) and its Gram G (r x r) no
// longer fit beside the row tiles in one workgroup's LDS.  The half-step is
// four launches (plus the fixed-order sum of the partials):
//
//   prep   C = (the other side's Qb'^T F') / its column norms when they come
//          from the W side (the normalisation at the end of Sec 4), G = C^T C
//          on FP64 MFMA, 1/(G_jj + beta), the column scales of F;
//   grad   g = S C - (F diag(scl)) G for every row (the row of X-check B-check
//          or X-hat^T A-hat minus f G), one FP32 MFMA product with the two
//          operand pairs concatenated along K;
//   sweep  the Gauss-Seidel sweep j = 1..r of each row in gradient form:
//          f_j <- [f_j + g_j / G_jj]_+ (Sec 4.1: [(f_j G_jj + g_j - alpha) /
//          (G_jj + beta)]_+), then g_l -= d G_jl with d the change of f_j;
//   qtf    this side's partials Qb^T F (the other side's compressed factor)
//          and the column sums of F^2, per workgroup, on FP32 MFMA.
//
// Semantics (scales, published C / G / 1/||a_j||, alpha, beta, normalisation
// modes) are those of the fused kernel for narrower factors.
#include "common.h"

namespace {

constexpr int BR = 128;              // factor width of this path (columns padded with zeros)
constexpr int BNB = BR / 16;         // 16-column blocks of G

// ------------------------------------------------------------------- prep
// Block (bi, bj) of G = C^T C on v_mfma_f64_16x16x4_f64: the two 16-column
// slices of C are staged in LDS with all loads in flight, the four waves take
// a quarter of k' each (A[i][k] = C[k][16 bi + i], B[k][j] = C[k][16 bj + j];
// D[i][j] in lane j + 16 (i % 4), register i / 4), and the four partial blocks
// are added in wave order.  Blocks with bj == 0 also write their 16 columns of
// C and of the scales; diagonal blocks write 1/(G_jj + beta).
constexpr int PKMAX = 256;
__global__ void __launch_bounds__(256)
hs_prep_kernel(HalfStepArgs a, float* __restrict__ Cp, float* __restrict__ Gp, float* __restrict__ rdiag,
               float* __restrict__ scl) {
  __shared__ double Ci[PKMAX][17], Cj[PKMAX][17];
  __shared__ double sf[2][16];
  __shared__ f64x4 part[4][64];
  const int bi = blockIdx.x, bj = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = lane & 15, g = lane >> 4;
  const int kp = a.kp, r = a.r;
  if (tid < 32) {   // the column normalisation of C when the sum comes from the W side (end of Sec 4)
    const int jj = 16 * (tid < 16 ? bi : bj) + (tid & 15);
    double sj = 1.0;
    if (a.norm_in && a.normalize && jj < r) {
      const double nrm = sqrt(a.acc_in[(int64_t)kp * r + jj]);
      sj = nrm > 0.0 ? nrm : 1.0;
    }
    sf[tid >> 4][tid & 15] = sj;
  }
  // raw slices: thread t loads columns (t % 16) of rows t / 16, t / 16 + 16, ...
  constexpr int PR = PKMAX / 16;
  double vi[PR], vj[PR];
#pragma unroll
  for (int p = 0; p < PR; ++p) {
    const int c = tid / 16 + 16 * p, jl = tid % 16;
    const int ji = 16 * bi + jl, jjj = 16 * bj + jl;
    vi[p] = (c < kp && ji < r) ? a.acc_in[(int64_t)c * r + ji] : 0.0;
    vj[p] = (c < kp && jjj < r) ? a.acc_in[(int64_t)c * r + jjj] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PR; ++p) {
    const int c = tid / 16 + 16 * p, jl = tid % 16;
    Ci[c][jl] = vi[p] / sf[0][jl];
    Cj[c][jl] = vj[p] / sf[1][jl];
  }
  __syncthreads();
  f64x4 d = {0.0, 0.0, 0.0, 0.0};
  const int kq = (kp + 15) / 16 * 4;            // k range per wave, a multiple of 4
  for (int k0 = wave * kq; k0 < (wave + 1) * kq && k0 < kp; k0 += 4) {
    const int kk = k0 + g;
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(Ci[kk][l], Cj[kk][l], d, 0, 0, 0);   // rows >= kp are zero
  }
  part[wave][lane] = d;
  __syncthreads();
  if (wave == 0) {
    const f64x4 t = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      const int i = 16 * bi + 4 * x + g, j = 16 * bj + l;
      const float gv = (float)t[x];
      Gp[i * BR + j] = gv;
      if (a.G_pub && i < r && j < r) a.G_pub[i * r + j] = gv;
      if (bi == bj && i == j) {
        const float den = (j < r) ? gv + a.beta : 0.f;
        rdiag[j] = den > 0.f ? 1.f / den : 0.f;
      }
    }
  }
  if (bj == 0) {
    for (int e = tid; e < kp * 16; e += 256) {
      const int c = e / 16, jl = e % 16, ji = 16 * bi + jl;
      const float cv = (float)Ci[c][jl];
      Cp[c * BR + ji] = cv;
      if (a.C_pub && ji < r) a.C_pub[c * r + ji] = cv;
    }
    if (tid < 16) {
      const int ji = 16 * bi + tid;
      const double si = sf[0][tid];
      float sc = 1.f;
      if (a.norm_in) sc = (a.normalize == 1) ? (float)si : 1.f;   // compensation b_j *= ||a_j||
      else if (a.scale) sc = (ji < r) ? a.scale[ji] : 1.f;
      scl[ji] = (ji < r) ? sc : 0.f;
      if (a.scale_pub && ji < r) a.scale_pub[ji] = (float)(1.0 / si);
    }
  }
}

// ------------------------------------------------------------------- grad
// g (N x r, ld r) = [S | F diag(scl)] [C ; -G]: K runs over the kp columns of S
// (padded to a multiple of 32 with zeros), then over the BR columns of F.
// 256 threads, 2 x 2 waves over a BM x 128 tile; v_mfma_f32_32x32x2_f32 with
// the k order permuted within groups of 8 so that a lane reads its four A values
// of a group as one 16-byte LDS load (lanes 0-31 take k = 8 g + s, lanes 32-63
// k = 8 g + 4 + s in step s).  The next K step is loaded into registers while
// the LDS tile is consumed.
template <int BM>
__global__ void __launch_bounds__(256)
hs_grad_kernel(const float* __restrict__ S, int64_t lds, const float* __restrict__ F, const float* __restrict__ scl,
               const float* __restrict__ Cp, const float* __restrict__ Gp, float* __restrict__ gout, int64_t N,
               int kp, int r) {
  constexpr int BK = 32, BN = BR, WM = 2, WN = 2;
  constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  constexpr int AROW = BK + 4, BROW = BN + 4;
  constexpr int AE = BM * BK / 256;        // A elements per thread
  constexpr int BV = BK * BN / 4 / 256;    // B float4 per thread
  __shared__ __attribute__((aligned(16))) float As[BM * AROW];
  __shared__ __attribute__((aligned(16))) float Bs[BK * BROW];
  __shared__ float sc[BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  if (tid < BR) sc[tid] = scl[tid];
  const int ks = (kp + BK - 1) / BK;       // K steps over S
  const int T = ks + BR / BK;              // then over F
  f32x16 acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.f;
  float ra[AE];
  f32x4 rb[BV];
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  __syncthreads();
  // A: thread t loads row (t / 8) + 32 p, columns 4 (t % 8) .. +3 of the 32-wide step
  auto load = [&](int t) {
    const bool fs = t >= ks;                // F part
    const int k0 = fs ? (t - ks) * BK : t * BK;
#pragma unroll
    for (int p = 0; p < AE / 4; ++p) {
      const int row = (tid >> 3) + 32 * p, c = 4 * (tid & 7);
      const int64_t gi = i0 + row;
      if (!fs) {
        f32x4 v = z4;
        if (gi < N && k0 + c < kp) v = *(const f32x4*)(S + gi * lds + k0 + c);   // padding columns are zero
        ra[4 * p] = v[0]; ra[4 * p + 1] = v[1]; ra[4 * p + 2] = v[2]; ra[4 * p + 3] = v[3];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int l = k0 + c + e;
          ra[4 * p + e] = (gi < N && l < r) ? F[gi * r + l] * sc[l] : 0.f;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, kk = f / (BN / 4), c4 = f % (BN / 4);
      f32x4 v = z4;
      if (!fs) {
        if (k0 + kk < kp) v = *(const f32x4*)(Cp + (int64_t)(k0 + kk) * BR + 4 * c4);
      } else {
        v = *(const f32x4*)(Gp + (int64_t)(k0 + kk) * BR + 4 * c4);
        v = -v;
      }
      rb[p] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int p = 0; p < AE / 4; ++p) {
      const int row = (tid >> 3) + 32 * p, c = 4 * (tid & 7);
      *(f32x4*)(As + row * AROW + c) = (f32x4){ra[4 * p], ra[4 * p + 1], ra[4 * p + 2], ra[4 * p + 3]};
    }
#pragma unroll
    for (int p = 0; p < BV; ++p) {
      const int f = tid + 256 * p, kk = f / (BN / 4), c4 = f % (BN / 4);
      *(f32x4*)(Bs + kk * BROW + 4 * c4) = rb[p];
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  load(0);
  for (int t = 0; t < T; ++t) {
    store();
    __syncthreads();
    if (t + 1 < T) load(t + 1);
#pragma unroll
    for (int gq = 0; gq < BK / 8; ++gq) {
      const int kb = 8 * gq + 4 * half;
      f32x4 af[TM];
      float bf[TN][4];
#pragma unroll
      for (int x = 0; x < TM; ++x) af[x] = *(const f32x4*)(As + (wm * (BM / WM) + 32 * x + l32) * AROW + kb);
#pragma unroll
      for (int y = 0; y < TN; ++y)
#pragma unroll
        for (int s = 0; s < 4; ++s) bf[y][s] = Bs[(kb + s) * BROW + wn * (BN / WN) + 32 * y + l32];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
          for (int y = 0; y < TN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[x][s], bf[y][s], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  // D[i][j] of a 32 x 32 tile: lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      const int j = wn * (BN / WN) + 32 * y + l32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int il = (e >> 2) * 8 + half * 4 + (e & 3);
        const int64_t gi = i0 + wm * (BM / WM) + 32 * x + il;
        if (gi < N && j < r) gout[gi * r + j] = acc[x][y][e];
      }
    }
}

// Broadcast of lane src of each quad to the quad (DPP quad permute).
__device__ __forceinline__ float quad_bcast_b(float v, int src) {
  const int x = __builtin_bit_cast(int, v);
  int y;
  switch (src) {
    case 0: y = __builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, false); break;
    case 1: y = __builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, false); break;
    case 2: y = __builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, false); break;
    default: y = __builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, false); break;
  }
  return __builtin_bit_cast(float, y);
}

// ------------------------------------------------------------------- sweep
// One quad of lanes per row, components interleaved over the quad: lane q owns
// components 4 u + q (u = 0..31), so that after component j the components
// still to come (> j) are spread over all four lanes.  At step j the owner lane
// (j % 4) forms the new f_j and the change d goes to the quad; every lane then
// takes g -= d G[j][.] for its slots u >= 4 floor(j / 16) (the slots below hold
// components <= j, whose gradients are never read again).  G is staged in LDS
// permuted, Gq[j][q][u] = G[j][4 u + q], so those reads are 16-byte loads.  A
// workgroup sweeps the 64-row tiles blockIdx.x, blockIdx.x + gridDim.x, ...;
// the rows of its next tile are loaded while the current one is swept.
template <bool PLAIN>   // alpha = beta = 0: the plain rule
__global__ void __launch_bounds__(256)
hs_sweep_kernel(const float* __restrict__ gin, const float* __restrict__ Gp, const float* __restrict__ rdiag,
                const float* __restrict__ scl, float* __restrict__ F, int64_t N, int r, float alpha, float beta) {
  constexpr int RQ = BR / 4;
  __shared__ __attribute__((aligned(16))) float Gq[BR * BR];
  __shared__ float rd[BR], gjj[BR], sc[BR];
  for (int e = threadIdx.x; e < BR * BR; e += 256) {
    const int j = e / BR, c = e % BR;          // c = 4 u + q  ->  Gq[j][q][u]
    Gq[j * BR + (c & 3) * RQ + (c >> 2)] = Gp[e];
  }
  if (threadIdx.x < BR) {
    rd[threadIdx.x] = rdiag[threadIdx.x];
    gjj[threadIdx.x] = Gp[threadIdx.x * BR + threadIdx.x];
    sc[threadIdx.x] = scl[threadIdx.x];
  }
  __syncthreads();
  const int q = threadIdx.x & 3, rl = threadIdx.x >> 2;
  const int64_t ntiles = ceil_div(N, 64);
  float f[RQ], g[RQ], fx[RQ], gx[RQ];
  auto load = [&](int64_t tile, float* fo, float* go) {
    const int64_t row = tile * 64 + rl;
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      fo[u] = 0.f;
      go[u] = 0.f;
    }
    if (tile < ntiles && row < N) {
      const float* fr = F + row * r;
      const float* gr = gin + row * r;
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const int c = 4 * u + q;
        if (c < r) {
          fo[u] = fr[c];
          go[u] = gr[c];
        }
      }
    }
  };
  load(blockIdx.x, fx, gx);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row = tile * 64 + rl;
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      f[u] = fx[u] * sc[4 * u + q];
      g[u] = gx[u];
    }
    load(tile + gridDim.x, fx, gx);            // in flight during the sweep
    // fully unrolled: every register index below is a compile-time constant
#pragma clang loop unroll(full)
    for (int j = 0; j < BR; ++j) {
      // no branch: a component with 1/(G_jj + beta) = 0 keeps f_j, so its d is 0
      const float rdj = rd[j];
      const int t = j >> 2;
      const float v = PLAIN ? f[t] + g[t] * rdj : (f[t] * gjj[j] + g[t] - alpha) * rdj;
      const float fn = rdj > 0.f ? (v > 0.f ? v : 0.f) : f[t];
      const float d = quad_bcast_b(fn - f[t], j & 3);
      if (q == (j & 3)) f[t] = fn;
      const float* gr = Gq + j * BR + q * RQ;
#pragma unroll
      for (int u = 4 * (j >> 4); u < RQ; u += 4) {
        const f32x4 gv = *(const f32x4*)(gr + u);
        g[u] -= d * gv[0];
        g[u + 1] -= d * gv[1];
        g[u + 2] -= d * gv[2];
        g[u + 3] -= d * gv[3];
      }
      __builtin_amdgcn_sched_barrier(0);   // keep each step's loads with it (register pressure)
    }
    if (row < N) {
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const int c = 4 * u + q;
        if (c < r) F[row * r + c] = f[u];
      }
    }
  }
}

// ------------------------------------------------------------------- qtf
// Workgroup partial Qb^T (F diag(sc)) (kp x r) and column sums of its squares,
// over the 64-row tiles blockIdx.x, blockIdx.x + gridDim.x, ...  The tiles of
// Qb and F are staged in LDS; v_mfma_f32_32x32x2_f32 with A[c][i] = Qb[i][c] and
// B[i][j] = F[i][j], contraction over the tile's rows.  Wave w owns the 32-row
// blocks c of its quarter and all four 32-column blocks j.
template <int KPMAX>
__global__ void __launch_bounds__(256)
hs_qtf_kernel(const float* __restrict__ Qb, int64_t ldq, const float* __restrict__ F, const float* __restrict__ scale,
              int64_t N, int kp, int r, float* __restrict__ part) {
  constexpr int TRW = 64, QROW = KPMAX + 4, FROW = BR + 4;
  constexpr int NTM = KPMAX / 32 / 4;       // 32-row blocks of the output per wave
  constexpr int QV = TRW * KPMAX / 4 / 256; // float4 of Qb per thread
  constexpr int FE = TRW * BR / 256;        // F elements per thread
  __shared__ __attribute__((aligned(16))) float Qs[TRW * QROW];
  __shared__ __attribute__((aligned(16))) float Fs[TRW * FROW];
  __shared__ float sc[BR];
  __shared__ float csum[2][BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < BR) sc[tid] = (scale && tid < r) ? scale[tid] : 1.f;
  f32x16 acc[NTM][4];
#pragma unroll
  for (int x = 0; x < NTM; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.f;
  float colsq = 0.f;
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  const int64_t ntiles = ceil_div(N, TRW);
  const int half = lane >> 5, l32 = lane & 31;
  // the next tile is loaded into registers while the current one is used
  f32x4 qv[QV];
  float fv[FE];
  auto load = [&](int64_t tile) {
    const int64_t row0 = tile * TRW;
#pragma unroll
    for (int p = 0; p < QV; ++p) {
      const int e = tid + 256 * p, i = e / (KPMAX / 4), c4 = e % (KPMAX / 4);
      qv[p] = (tile < ntiles && row0 + i < N && 4 * c4 < kp) ? *(const f32x4*)(Qb + (row0 + i) * ldq + 4 * c4) : z4;
    }
#pragma unroll
    for (int p = 0; p < FE; ++p) {
      const int e = tid + 256 * p, i = e / BR, j = e % BR;
      fv[p] = (tile < ntiles && row0 + i < N && j < r) ? F[(row0 + i) * r + j] : 0.f;   // padding is zero
    }
  };
  __syncthreads();
  load(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
    for (int p = 0; p < QV; ++p) {
      const int e = tid + 256 * p, i = e / (KPMAX / 4), c4 = e % (KPMAX / 4);
      *(f32x4*)(Qs + i * QROW + 4 * c4) = qv[p];
    }
#pragma unroll
    for (int p = 0; p < FE; ++p) {
      const int e = tid + 256 * p, i = e / BR, j = e % BR;
      Fs[i * FROW + j] = fv[p] * sc[j];
    }
    __syncthreads();
    load(tile + gridDim.x);
    {   // column sums of squares: two threads per column, fixed order
      const int j = tid % BR, pr = tid / BR;
      float sq = 0.f;
      for (int i = pr; i < TRW; i += 2) {
        const float v = Fs[i * FROW + j];
        sq += v * v;
      }
      colsq += sq;
    }
#pragma unroll 2
    for (int k = 0; k < TRW; k += 2) {
      const int i = k + half;
      float av[NTM], bv[4];
#pragma unroll
      for (int x = 0; x < NTM; ++x) av[x] = Qs[i * QROW + 32 * (wave * NTM + x) + l32];
#pragma unroll
      for (int y = 0; y < 4; ++y) bv[y] = Fs[i * FROW + 32 * y + l32];
#pragma unroll
      for (int x = 0; x < NTM; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  float* P = part + (int64_t)blockIdx.x * (kp * r + r);
#pragma unroll
  for (int x = 0; x < NTM; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int j = 32 * y + l32;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int c = 32 * (wave * NTM + x) + (e >> 2) * 8 + half * 4 + (e & 3);
        if (c < kp && j < r) P[c * r + j] = acc[x][y][e];
      }
    }
  csum[tid / BR][tid % BR] = colsq;
  __syncthreads();
  if (tid < r) P[kp * r + tid] = csum[0][tid] + csum[1][tid];
}

}  // namespace

// Floats of the auxiliary buffer of this path: C (256 x 128), G (128 x 128),
// 1/(G_jj + beta) and the column scales.
size_t halfstep_big_aux_floats() { return (size_t)256 * BR + BR * BR + 2 * BR; }

bool halfstep_big(int kp, int r) { return r <= 128 && kp <= 256 && (r > 64 || kp > 128); }

hipError_t launch_halfstep_big(const HalfStepArgs& a, int do_sweep, hipStream_t st) {
  if (!a.aux || (do_sweep && !a.gbuf)) return hipErrorInvalidValue;
  float* Cp = a.aux;
  float* Gp = Cp + 256 * BR;
  float* rdiag = Gp + BR * BR;
  float* scl = rdiag + BR;
  const int nblk = halfstep_blocks(a.N);
  if (do_sweep) {
    if (a.kp > PKMAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(hs_prep_kernel, dim3(BNB, BNB), dim3(256), 0, st, a, Cp, Gp, rdiag, scl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.N >= 128 * 512)
      hipLaunchKernelGGL(hs_grad_kernel<128>, dim3((unsigned)ceil_div(a.N, 128)), dim3(256), 0, st, a.S, a.lds, a.F,
                         scl, Cp, Gp, a.gbuf, a.N, a.kp, a.r);
    else
      hipLaunchKernelGGL(hs_grad_kernel<64>, dim3((unsigned)ceil_div(a.N, 64)), dim3(256), 0, st, a.S, a.lds, a.F,
                         scl, Cp, Gp, a.gbuf, a.N, a.kp, a.r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.alpha == 0.f && a.beta == 0.f)
      hipLaunchKernelGGL(hs_sweep_kernel<true>, dim3((unsigned)nblk), dim3(256), 0, st, a.gbuf, Gp, rdiag, scl, a.F,
                         a.N, a.r, a.alpha, a.beta);
    else
      hipLaunchKernelGGL(hs_sweep_kernel<false>, dim3((unsigned)nblk), dim3(256), 0, st, a.gbuf, Gp, rdiag, scl,
                         a.F, a.N, a.r, a.alpha, a.beta);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // after a sweep F is final; without one its pending column scales apply on load
  const float* qscale = do_sweep ? nullptr : a.scale;
  if (a.kp <= 128)
    hipLaunchKernelGGL(hs_qtf_kernel<128>, dim3((unsigned)nblk), dim3(256), 0, st, a.Qb, a.ldq, a.F, qscale, a.N,
                       a.kp, a.r, a.part);
  else
    hipLaunchKernelGGL(hs_qtf_kernel<256>, dim3((unsigned)nblk), dim3(256), 0, st, a.Qb, a.ldq, a.F, qscale, a.N,
                       a.kp, a.r, a.part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials_f32(a.part, nblk, (int64_t)a.kp * a.r + a.r, a.acc_out, st);
}
