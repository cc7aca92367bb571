// FastHALS-RP half-steps (eq fastHALS_a) on the compressed data.
//
// One kernel serves both halves of an iteration:
//   W side:  S = Xc (m x k'), C = Hc = Q_R^T Ht, G = Hc^T Hc, F = W,  Qb = Q_L
//   H side:  S = Xh (n x k'), C = Wh = Q_L^T W,  G = Wh^T Wh, F = Ht, Qb = Q_R
// For each row f of F (rows are independent):
//   h = s C                       (the row of X-check B-check or X-hat^T A-hat)
//   for j = 1..r:  f_j <- [f_j + (h_j - f G_j) / G_jj]_+      (skip if G_jj <= 0)
// (with sparsity alpha and smoothness beta: f_j <- [(f_j G_jj + h_j - f G_j - alpha)
//  / (G_jj + beta)]_+ , Sec 4.1).  The swept rows are written back and every
// workgroup emits its partial Qb^T F (the other side's compressed factor, Sec 4)
// and the column sums of F^2 (for a_j / ||a_j||, end of Sec 4).
//
// The partials of one half-step are summed in FP64 and fixed order by a small
// kernel; the next half-step's prologue turns that sum into its C and G (with
// the column normalisation when the sum comes from the W side), G = C^T C on
// FP64 MFMA.  No workgroup waits on another inside a kernel.
//
// A workgroup of 256 threads owns 64 rows at a time, four threads (a quad) per
// row, and loops over row tiles (bounded number of partials).  The loads of the
// next tile are issued before the sweep of the current one.
#include "common.h"

namespace {

constexpr int NTHR = 256;          // threads per workgroup
constexpr int TPR = 4;             // threads per row (one quad)
constexpr int TRW = NTHR / TPR;    // rows per tile
constexpr int MAXBLK = 512;        // cap on workgroups (and partials)

// Broadcast of a float from quad lane src to the four lanes of every quad (DPP;
// src is a constant after unrolling, so the switch folds to one move).
__device__ __forceinline__ float quad_bcast(float v, int src) {
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

template <int RMAX, int KPMAX>
struct Tile {
  static constexpr int RQ = RMAX / TPR;                    // components per thread
  static constexpr int SROW = KPMAX + 4;                   // LDS row stride of S / Qb tiles
  static constexpr int FROW = RMAX + 4;                    // LDS row stride of the F tile
  static constexpr int NV = KPMAX / 4;                     // float4 per row of S / Qb
  static constexpr int VPT = TRW * NV / NTHR;              // S or Qb float4 per thread
  static constexpr int FPT = TRW * RMAX / NTHR;            // F elements per thread
  static constexpr int NTM = KPMAX / 32, NTN = (RMAX + 31) / 32;
  static constexpr int NT = NTM * NTN;                     // 32x32 tiles of the partial
  static constexpr int KSPLIT = NT >= 4 ? 1 : 4 / NT;      // waves sharing one tile
  static constexpr int TPW = KSPLIT == 1 ? (NT + 3) / 4 : 1;
  static constexpr int SEG = TRW / KSPLIT;                 // rows per wave per tile
  static constexpr int NSUB = NTHR / RMAX;                 // threads per column (sums)
  static constexpr int U_TILES = 2 * TRW * SROW * 4;      // Ss + Qs bytes
  static constexpr int U_CD = KPMAX * RMAX * 8;            // FP64 C in the prologue
  static constexpr int U_MIN = 16384;                      // 4 waves x 1024 floats (wave sums)
  static constexpr int U_A = U_TILES > U_CD ? U_TILES : U_CD;
  static constexpr int U_BYTES = U_A > U_MIN ? U_A : U_MIN;
};

template <int RMAX, int KPMAX>
__global__ void __launch_bounds__(NTHR)
halfstep_kernel(HalfStepArgs a, int do_sweep) {
  using T = Tile<RMAX, KPMAX>;
  constexpr int RQ = T::RQ, SROW = T::SROW, FROW = T::FROW, NV = T::NV, VPT = T::VPT;
  constexpr int FPT = T::FPT, NT = T::NT, NTN = T::NTN, KSPLIT = T::KSPLIT, TPW = T::TPW;
  constexpr int SEG = T::SEG, NSUB = T::NSUB;
  static_assert(RQ % 4 == 0, "RMAX must be a multiple of 16");
  __shared__ __attribute__((aligned(16))) char U[T::U_BYTES];
  __shared__ __attribute__((aligned(16))) float Fs[TRW * FROW];
  __shared__ __attribute__((aligned(16))) float Cs[KPMAX * RMAX];
  __shared__ __attribute__((aligned(16))) float Gs[RMAX * RMAX];
  __shared__ __attribute__((aligned(16))) float Gu[RMAX * RMAX];   // G_jl for l > j, else 0
  __shared__ float scl[RMAX];            // column scale applied to F on load
  __shared__ __attribute__((aligned(16))) float rdiag[RMAX];   // 1/(G_jj + beta), 0 = skip
  __shared__ double sfac[RMAX];          // normalisation factors of C
  __shared__ float csum[NSUB][RMAX];
  float* Ss = reinterpret_cast<float*>(U);
  float* Qs = Ss + TRW * SROW;
  double* Cd = reinterpret_cast<double*>(U);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = tid / TPR, q = tid % TPR;
  const int kp = a.kp, r = a.r;
  const bool plain = (a.alpha == 0.f && a.beta == 0.f);

  f32x16 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int x = 0; x < 16; ++x) acc[t][x] = 0.f;
  float colsq = 0.f;   // thread (part, j): running sum of F[:, j]^2 over its rows

  const int64_t ntiles = ceil_div(a.N, TRW);
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  float fv[FPT];
  f32x4 sv[VPT], qv[VPT];
  auto issue = [&](int64_t tile) {
    const int64_t row0 = tile * TRW;
    const int rows = (int)((a.N - row0) < TRW ? (a.N - row0) : TRW);
#pragma unroll
    for (int p = 0; p < FPT; ++p) {
      const int e = tid + NTHR * p, i = e / RMAX, j = e % RMAX;
      fv[p] = (i < rows && j < r) ? a.F[(row0 + i) * r + j] : 0.f;
    }
#pragma unroll
    for (int p = 0; p < VPT; ++p) {
      const int e = tid + NTHR * p, i = e / NV, c4 = e % NV;
      const bool ok = i < rows && 4 * c4 < kp;
      sv[p] = (do_sweep && ok) ? *(const f32x4*)(a.S + (row0 + i) * a.lds + 4 * c4) : z4;
      qv[p] = ok ? *(const f32x4*)(a.Qb + (row0 + i) * a.ldq + 4 * c4) : z4;
    }
  };
  if ((int64_t)blockIdx.x < ntiles) issue(blockIdx.x);   // first tile in flight during the prologue

  // ---- prologue: C and G of this half-step from the other side's summed partials
  for (int j = tid; j < RMAX; j += NTHR) {
    double sj = 1.0;
    if (a.norm_in && a.normalize && j < r) {
      const double nrm = sqrt(a.acc_in[kp * r + j]);
      sj = nrm > 0.0 ? nrm : 1.0;
    }
    sfac[j] = sj;
    float sc = 1.f;
    if (a.norm_in) sc = (a.normalize == 1) ? (float)sj : 1.f;   // compensation b_j *= ||a_j||
    else if (a.scale) sc = (j < r) ? a.scale[j] : 1.f;
    scl[j] = (j < r) ? sc : 0.f;
    if (a.scale_pub && blockIdx.x == 0 && j < r) a.scale_pub[j] = (float)(1.0 / sj);
  }
  __syncthreads();
  if (do_sweep) {
    for (int e = tid; e < KPMAX * RMAX; e += NTHR) {
      const int c = e / RMAX, j = e % RMAX;
      const double v = (c < kp && j < r) ? a.acc_in[c * r + j] / sfac[j] : 0.0;
      Cd[e] = v;
      Cs[e] = (float)v;
      if (a.C_pub && blockIdx.x == 0 && c < kp && j < r) a.C_pub[c * r + j] = (float)v;
    }
    __syncthreads();
    // G = C^T C on v_mfma_f64_16x16x4_f64: A[i][k] = C[k][i], B[k][j] = C[k][j];
    // D[i][j] in lane j + 16 (i % 4), register i / 4.
    constexpr int nt = RMAX / 16;
    for (int t = wave; t < nt * nt; t += 4) {
      const int ti = t / nt, tj = t % nt;
      f64x4 d = {0, 0, 0, 0};
      for (int k0 = 0; k0 < KPMAX; k0 += 4) {
        const int kk = k0 + (lane >> 4);
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(Cd[kk * RMAX + ti * 16 + (lane & 15)],
                                                 Cd[kk * RMAX + tj * 16 + (lane & 15)], d, 0, 0, 0);
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int i = ti * 16 + 4 * x + (lane >> 4), j = tj * 16 + (lane & 15);
        Gs[i * RMAX + j] = (float)d[x];
        Gu[i * RMAX + j] = j > i ? (float)d[x] : 0.f;
        if (a.G_pub && blockIdx.x == 0 && i < r && j < r) a.G_pub[i * r + j] = (float)d[x];
      }
    }
    __syncthreads();
    for (int j = tid; j < RMAX; j += NTHR) {
      const float den = (j < r) ? Gs[j * RMAX + j] + a.beta : 0.f;
      rdiag[j] = den > 0.f ? 1.f / den : 0.f;
    }
  }


  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * TRW;
    const int rows = (int)((a.N - row0) < TRW ? (a.N - row0) : TRW);
    __syncthreads();   // readers of the previous tile are done
#pragma unroll
    for (int p = 0; p < FPT; ++p) {
      const int e = tid + NTHR * p, i = e / RMAX, j = e % RMAX;
      Fs[i * FROW + j] = fv[p] * scl[j];
    }
#pragma unroll
    for (int p = 0; p < VPT; ++p) {
      const int e = tid + NTHR * p, i = e / NV, c4 = e % NV;
      *(f32x4*)(Ss + i * SROW + 4 * c4) = sv[p];
      *(f32x4*)(Qs + i * SROW + 4 * c4) = qv[p];
    }
    __syncthreads();
    if (tile + gridDim.x < ntiles) issue(tile + gridDim.x);
    // ---- sweep.  The quad of a row holds the whole row f (replicated) and each
    // thread the gradient g = h - f G for its RQ components; after component j
    // moves by d, g_l -= d G_jl for l > j (G is symmetric; Gu holds those G_jl).
    if (do_sweep) {
      // g = S C - F G = [S | -F] [C ; G] on v_mfma_f32_16x16x4_f32.  Wave w owns
      // rows 16w..16w+15 of the tile (the rows of its own quads), so it reads and
      // then overwrites only its own rows of Ss: no workgroup barrier is needed.
      // In k-step s lane l holds A[l % 16][4s + l / 16] and B[4s + l / 16][l % 16];
      // D[i][j] sits in lane j + 16 (i / 4), register i % 4.
      {
        constexpr int NJ = RMAX / 16;
        f32x4 gd[NJ];
#pragma unroll
        for (int t = 0; t < NJ; ++t) gd[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
        const int ar = wave * 16 + (lane & 15), kq = lane >> 4;
#pragma unroll 4
        for (int k0 = 0; k0 < KPMAX; k0 += 4) {
          const float av = Ss[ar * SROW + k0 + kq];
#pragma unroll
          for (int t = 0; t < NJ; ++t)
            gd[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Cs[(k0 + kq) * RMAX + t * 16 + (lane & 15)],
                                                         gd[t], 0, 0, 0);
        }
#pragma unroll 4
        for (int k0 = 0; k0 < RMAX; k0 += 4) {
          const float av = -Fs[ar * FROW + k0 + kq];
#pragma unroll
          for (int t = 0; t < NJ; ++t)
            gd[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, Gs[(k0 + kq) * RMAX + t * 16 + (lane & 15)],
                                                         gd[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NJ; ++t)
#pragma unroll
          for (int x = 0; x < 4; ++x) Ss[(wave * 16 + 4 * kq + x) * SROW + t * 16 + (lane & 15)] = gd[t][x];
      }
      float f[RMAX], g[RQ];
#pragma unroll
      for (int j = 0; j < RMAX; j += 4) {
        const f32x4 v = *(const f32x4*)(Fs + row * FROW + j);
        f[j] = v[0]; f[j + 1] = v[1]; f[j + 2] = v[2]; f[j + 3] = v[3];
      }
      const int c0 = q * RQ;
#pragma unroll
      for (int l = 0; l < RQ; l += 4) {
        const f32x4 v = *(const f32x4*)(Ss + row * SROW + c0 + l);
        g[l] = v[0]; g[l + 1] = v[1]; g[l + 2] = v[2]; g[l + 3] = v[3];
      }
#pragma unroll
      for (int j = 0; j < RMAX; ++j) {
        const float gj = quad_bcast(g[j % RQ], j / RQ);
        const float rd = rdiag[j];
        if (rd > 0.f) {
          const float gjj = Gs[j * RMAX + j];
          const float v = plain ? f[j] + gj * rd : (f[j] * gjj + gj - a.alpha) * rd;
          const float fn = v > 0.f ? v : 0.f;
          const float d = fn - f[j];
          f[j] = fn;
#pragma unroll
          for (int l = 0; l < RQ; l += 4) {
            const f32x4 g4 = *(const f32x4*)(Gu + j * RMAX + c0 + l);
            g[l] -= d * g4[0];
            g[l + 1] -= d * g4[1];
            g[l + 2] -= d * g4[2];
            g[l + 3] -= d * g4[3];
          }
        }
      }
      if (q == 0) {
#pragma unroll
        for (int j = 0; j < RMAX; j += 4) {
          f32x4 v;
          v[0] = row < rows ? f[j] : 0.f;
          v[1] = row < rows ? f[j + 1] : 0.f;
          v[2] = row < rows ? f[j + 2] : 0.f;
          v[3] = row < rows ? f[j + 3] : 0.f;
          *(f32x4*)(Fs + row * FROW + j) = v;
        }
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < FPT; ++p) {
        const int e = tid + NTHR * p, i = e / RMAX, j = e % RMAX;
        if (i < rows && j < r) a.F[(row0 + i) * r + j] = Fs[i * FROW + j];
      }
    }
    // ---- column sums of squares (NSUB threads per column, fixed order)
    {
      const int j = tid % RMAX, part = tid / RMAX;
      float s = 0.f;
#pragma unroll
      for (int i = part; i < TRW; i += NSUB) {
        const float v = Fs[i * FROW + j];
        s += v * v;
      }
      colsq += s;
    }
    // ---- partial Qb^T F on MFMA: A[c][i] = Qb[i][c], B[i][j] = F[i][j], contraction
    // over the tile's rows (split over KSPLIT waves when there are few tiles)
    const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = KSPLIT == 1 ? wave + 4 * t : wave % NT;
      const int rs = KSPLIT == 1 ? 0 : (wave / NT) * SEG;
      if (tt < NT) {
        const int tm = tt / NTN, tn = tt % NTN;
        const int c = tm * 32 + l32, j = tn * 32 + l32;
#pragma unroll 4
        for (int kb = 0; kb < SEG; kb += 8) {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int i = rs + kb + 4 * half + s4;
            const float av = Qs[i * SROW + c];
            const float bv = (j < RMAX) ? Fs[i * FROW + j] : 0.f;
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[t], 0, 0, 0);
          }
        }
      }
    }
  }
  // ---- combine and write this workgroup's partial: [kp x r] then [r]
  csum[tid / RMAX][tid % RMAX] = colsq;
  float* P = a.part + (int64_t)blockIdx.x * (kp * r + r);
  const int half = lane >> 5, l32 = lane & 31;
  if (KSPLIT == 1) {
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = wave + 4 * t;
      if (tt < NT) {
        const int tm = tt / NTN, tn = tt % NTN;
        const int j = tn * 32 + l32;
#pragma unroll
        for (int x = 0; x < 16; ++x) {
          const int c = tm * 32 + (x >> 2) * 8 + half * 4 + (x & 3);
          if (c < kp && j < r) P[c * r + j] = acc[t][x];
        }
      }
    }
    __syncthreads();
  } else {
    // waves w, w + NT, ... hold partial sums of the same tile: add in wave order
    __syncthreads();
    float* buf = Ss;   // 4 waves x 1024 floats
#pragma unroll
    for (int x = 0; x < 16; ++x) buf[wave * 1024 + x * 64 + lane] = acc[0][x];
    __syncthreads();
    if (wave < NT) {
      const int tm = wave / NTN, tn = wave % NTN;
      const int j = tn * 32 + l32;
#pragma unroll
      for (int x = 0; x < 16; ++x) {
        float v = buf[wave * 1024 + x * 64 + lane];
#pragma unroll
        for (int sp = 1; sp < KSPLIT; ++sp) v += buf[(wave + sp * NT) * 1024 + x * 64 + lane];
        const int c = tm * 32 + (x >> 2) * 8 + half * 4 + (x & 3);
        if (c < kp && j < r) P[c * r + j] = v;
      }
    }
  }
  if (tid < r) {
    float s = 0.f;
#pragma unroll
    for (int p = 0; p < NSUB; ++p) s += csum[p][tid];
    P[kp * r + tid] = s;
  }
}

// Deterministic sum of split partials: out[e] = sum_s part[s*ne + e] in FP64,
// each of 16 thread groups summing a fixed stride of splits, combined in order.
template <typename T>
__global__ void __launch_bounds__(256)
sum_partials_kernel(const T* __restrict__ part, int nparts, int64_t ne, double* __restrict__ out,
                    const int* __restrict__ skip) {
  if (skip && skip[0] == 0) return;
  __shared__ double red[16][17];
  const int el = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t e = (int64_t)blockIdx.x * 16 + el;
  // partials g, g + 16, g + 32, ... in eight fixed accumulators; the eight
  // loads of a round are issued together (latency-bound for few elements)
  double s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  if (e < ne) {
    int b = g;
    for (; b + 112 < nparts; b += 128) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + 16 * u) * ne + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += (double)v[u];
    }
    for (; b < nparts; b += 16) s[0] += (double)part[(int64_t)b * ne + e];
  }
  red[g][el] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  if (g == 0 && e < ne) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][el];
    out[e] = t;
  }
}

template <int RMAX, int KPMAX>
hipError_t run(const HalfStepArgs& a, int do_sweep, hipStream_t st) {
  hipLaunchKernelGGL((halfstep_kernel<RMAX, KPMAX>), dim3(halfstep_blocks(a.N)), dim3(NTHR), 0, st, a,
                     do_sweep);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials_f32(a.part, halfstep_blocks(a.N), (int64_t)a.kp * a.r + a.r, a.acc_out,
                                 st);
}

// Few elements, many partials (sums of squares, proxy sums): one workgroup per
// element, thread t sums partials t, t + 256, ... (eight loads per round), then
// a fixed-order tree over the 256 threads.
template <typename T>
__global__ void __launch_bounds__(256)
sum_partials_few_kernel(const T* __restrict__ part, int nparts, int64_t ne, double* __restrict__ out,
                        const int* __restrict__ skip) {
  if (skip && skip[0] == 0) return;
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  double s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * 256 < nparts; b += 8 * 256) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(b + 256 * u) * ne + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += (double)v[u];
  }
  for (; b < nparts; b += 256) s[0] += (double)part[(int64_t)b * ne + e];
  red[threadIdx.x] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = red[0];
}


// ------------------------------------------------- uncompressed FastHALS (Sec 2.2)
// One sweep of the textbook rule over the rows of F (N x r, ld ldf) against the
// full-data targets: F = W with P = X Ht and G = Ht^T Ht, or F = Ht with P = X^T W
// and G = W^T W:  f_j <- [f_j + (p_j - (f G)_j) / G_jj]_+ , j ascending (G_jj <= 0:
// f_j unchanged).  A quad of lanes per row, lane q owning components
// q RMAX/4 .. +RMAX/4 - 1; gradient form as in the column NNLS (g = p - G f once,
// then g -= G[:, j] d after component j changes by d).  G (FP64) is staged in
// LDS as FP32.  sq (optional): per-workgroup column sums of F^2 after the sweep
// (nblk x r), for the normalisation a_j / ||a_j|| (end of Sec 4).
template <int RMAX>
__global__ void __launch_bounds__(256)
hals_rows_kernel(const float* __restrict__ P, int64_t ldp, const double* __restrict__ G, int64_t N, int r,
                 float* __restrict__ F, int64_t ldf, float* __restrict__ sq) {
  constexpr int RQ = RMAX / 4;
  __shared__ __attribute__((aligned(16))) float gs[RMAX * RMAX];
  __shared__ float rd[RMAX];
  __shared__ float csum[4][RMAX];
  for (int e = threadIdx.x; e < RMAX * RMAX; e += 256) {
    const int a = e / RMAX, b = e % RMAX;
    const double v = (a < r && b < r) ? G[a * r + b] : 0.0;
    gs[e] = (float)v;
    if (a == b) rd[a] = v > 0.0 ? (float)(1.0 / v) : 0.f;
  }
  __syncthreads();
  const int q = threadIdx.x & 3, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2);
  const bool valid = row < N;
  const int c0 = q * RQ;
  float f[RQ], g[RQ];
#pragma unroll
  for (int t = 0; t < RQ; ++t) {
    const bool in = valid && c0 + t < r;
    f[t] = in ? F[row * ldf + c0 + t] : 0.f;
    g[t] = in ? P[row * ldp + c0 + t] : 0.f;
  }
  // g = p - G f, with f of every component taken from its lane
#pragma unroll
  for (int qq = 0; qq < 4; ++qq)
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const float hv = quad_bcast(f[u], qq);
      const int col = qq * RQ + u;
#pragma unroll
      for (int t = 0; t < RQ; ++t) g[t] = fmaf(-gs[col * RMAX + c0 + t], hv, g[t]);
    }
#pragma unroll
  for (int j = 0; j < RMAX; ++j) {
    const float rdj = rd[j];
    if (rdj > 0.f) {                      // uniform over the block
      const int t = j % RQ;
      const float fn = fmaxf(fmaf(g[t], rdj, f[t]), 0.f);
      const float d = quad_bcast(fn - f[t], j / RQ);
      if (q == j / RQ) f[t] = fn;
#pragma unroll
      for (int u = 0; u < RQ; ++u) g[u] = fmaf(-gs[j * RMAX + c0 + u], d, g[u]);
    }
  }
  if (valid) {
#pragma unroll
    for (int t = 0; t < RQ; ++t)
      if (c0 + t < r) F[row * ldf + c0 + t] = f[t];
  }
  if (!sq) return;                        // uniform
  // column sums of f^2 over the block's 64 rows: the 16 rows of a wave by lane
  // moves (xor over the row bits of the lane index), then the four waves in LDS
#pragma unroll
  for (int t = 0; t < RQ; ++t) {
    float v = f[t] * f[t];
#pragma unroll
    for (int off = 4; off < 64; off <<= 1) v += __shfl_xor(v, off);
    if (lane < 4 && c0 + t < RMAX) csum[wave][c0 + t] = v;   // lanes 0..3 are quads' lane q
  }
  __syncthreads();
  if (threadIdx.x < r)
    sq[(int64_t)blockIdx.x * r + threadIdx.x] =
        (csum[0][threadIdx.x] + csum[1][threadIdx.x]) + (csum[2][threadIdx.x] + csum[3][threadIdx.x]);
}

// a_j <- a_j / ||a_j|| for the columns of W (M x r, ld ld) with ||a_j||^2 = sumsq[j]
// (FP64); mode 1 (compensated) also b_j <- b_j ||a_j|| in Ht (N x r, ld ld); zero
// columns stay.
__global__ void __launch_bounds__(256)
col_normalise_kernel(float* __restrict__ W, int64_t M, float* __restrict__ Ht, int64_t N, int r, int64_t ld,
                     const double* __restrict__ sumsq, int mode) {
  const int64_t tw = M * r, total = tw + (mode == 1 ? N * r : 0);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t f = e < tw ? e : e - tw;
    const int64_t i = f / r;
    const int j = (int)(f - i * r);
    const double s = sqrt(sumsq[j]);
    if (!(s > 0.0)) continue;
    if (e < tw) W[i * ld + j] = (float)((double)W[i * ld + j] / s);
    else Ht[i * ld + j] = (float)((double)Ht[i * ld + j] * s);
  }
}
}  // namespace

int halfstep_blocks(int64_t N) {
  int64_t t = ceil_div(N, TRW);
  if (t < 1) t = 1;
  return (int)(t < MAXBLK ? t : MAXBLK);
}

size_t halfstep_part_floats(int64_t N, int kp, int r) {
  return (size_t)halfstep_blocks(N) * (kp * r + r);
}

hipError_t launch_halfstep(const HalfStepArgs& a, int do_sweep, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  if (a.kp % 4 || a.lds % 4 || a.ldq % 4) return hipErrorInvalidValue;
  if (halfstep_big(a.kp, a.r)) return launch_halfstep_big(a, do_sweep, st);
  if (a.kp <= 32) {
    if (a.r <= 16) return run<16, 32>(a, do_sweep, st);
    if (a.r <= 32) return run<32, 32>(a, do_sweep, st);
  } else if (a.kp <= 64) {
    if (a.r <= 32) return run<32, 64>(a, do_sweep, st);
    if (a.r <= 64) return run<64, 64>(a, do_sweep, st);
  } else if (a.kp <= 128) {
    if (a.r <= 64) return run<64, 128>(a, do_sweep, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sum_partials_f32(const float* part, int nparts, int64_t ne, double* out,
                                   hipStream_t st) {
  if (ne <= 8 && nparts > 64) {
    hipLaunchKernelGGL(sum_partials_few_kernel<float>, dim3((unsigned)ne), dim3(256), 0, st, part, nparts, ne, out,
                       nullptr);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sum_partials_kernel<float>, dim3((unsigned)ceil_div(ne, 16)), dim3(256), 0, st,
                     part, nparts, ne, out, nullptr);
  return hipGetLastError();
}

hipError_t launch_sum_partials_f64(const double* part, int nparts, int64_t ne, double* out,
                                   const int* skip, hipStream_t st) {
  if (ne <= 8 && nparts > 64) {
    hipLaunchKernelGGL(sum_partials_few_kernel<double>, dim3((unsigned)ne), dim3(256), 0, st, part, nparts, ne, out,
                       skip);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(sum_partials_kernel<double>, dim3((unsigned)ceil_div(ne, 16)), dim3(256), 0, st,
                     part, nparts, ne, out, skip);
  return hipGetLastError();
}

int hals_rows_blocks(int64_t N) { return (int)ceil_div(N, 64); }

hipError_t launch_hals_rows(const float* P, int64_t ldp, const double* G, int64_t N, int r, float* F, int64_t ldf,
                            float* sq, hipStream_t st) {
  if (N == 0) return hipSuccess;
  const dim3 grid((unsigned)hals_rows_blocks(N));
  if (r <= 16)
    hipLaunchKernelGGL(hals_rows_kernel<16>, grid, dim3(256), 0, st, P, ldp, G, N, r, F, ldf, sq);
  else if (r <= 32)
    hipLaunchKernelGGL(hals_rows_kernel<32>, grid, dim3(256), 0, st, P, ldp, G, N, r, F, ldf, sq);
  else if (r <= 64)
    hipLaunchKernelGGL(hals_rows_kernel<64>, grid, dim3(256), 0, st, P, ldp, G, N, r, F, ldf, sq);
  else if (r <= 128)
    hipLaunchKernelGGL(hals_rows_kernel<128>, grid, dim3(256), 0, st, P, ldp, G, N, r, F, ldf, sq);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_col_normalise(float* W, int64_t M, float* Ht, int64_t N, int r, int64_t ld, const double* sumsq,
                                int mode, hipStream_t st) {
  if (mode == 0) return hipSuccess;
  int64_t g = ceil_div((M + N) * r, 256);
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(col_normalise_kernel, dim3((unsigned)g), dim3(256), 0, st, W, M, Ht, N, r, ld, sumsq, mode);
  return hipGetLastError();
}
