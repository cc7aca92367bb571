// FastHALS-RP half-steps (eq fastHALS_a) on the compressed data.
//
// One kernel serves both halves of an iteration:
//   W side:  S = Xc (m x k'), C = Hc = Q_R^T Ht, G = Hc^T Hc, F = W,  Qb = Q_L
//   H side:  S = Xh (n x k'), C = Wh = Q_L^T W,  G = Wh^T Wh, F = Ht, Qb = Q_R
// For each row f of F (rows are independent):
//   h = s C                       (the row of X-check B-check or X-hat^T A-hat)
//   for j = 1..r:  f_j <- [f_j + (h_j - f G_j) / G_jj]_+      (skip if G_jj <= 0)
// (with sparsity alpha and smoothness beta: f_j <- [(f_j G_jj + h_j - f G_j - alpha)
//  / (G_jj + beta)]_+ , Sec 4.1).  The swept rows are written back and the
// workgroup accumulates its partial Qb^T F (for the other side's compressed
// factor, Sec 4) on MFMA and the column sums of F^2 (for a_j / ||a_j||).
//
// A workgroup owns 128 rows at a time (one thread per row for the sweep) and
// loops over row tiles so the number of partials stays bounded.
#include "common.h"

namespace {

constexpr int TR = 128;        // rows per tile (threads per workgroup)
constexpr int MAXBLK = 512;    // cap on workgroups (and partials)

template <int RMAX, int KPMAX>
__global__ void __launch_bounds__(TR)
halfstep_kernel(HalfStepArgs a, int do_sweep) {
  constexpr int SROW = KPMAX + 4;
  constexpr int FROW = RMAX + 1;
  constexpr int NTM = KPMAX / 32, NTN = (RMAX + 31) / 32;   // partial tiles (k' x r)
  constexpr int NT = NTM * NTN;
  constexpr int TPW = (NT + 1) / 2;                          // tiles per wave (2 waves)
  __shared__ __attribute__((aligned(16))) float Ss[TR * SROW];   // S tile, then Qb tile
  __shared__ float Fs[TR * FROW];
  __shared__ __attribute__((aligned(16))) float Cs[KPMAX * RMAX];
  __shared__ float Gs[RMAX * RMAX];
  __shared__ float scl[RMAX];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kp = a.kp, r = a.r;
  const bool plain = (a.alpha == 0.f && a.beta == 0.f);

  for (int e = tid; e < KPMAX * RMAX; e += TR) {
    const int c = e / RMAX, j = e % RMAX;
    Cs[e] = (do_sweep && c < kp && j < r) ? a.C[c * r + j] : 0.f;
  }
  for (int e = tid; e < RMAX * RMAX; e += TR) {
    const int l = e / RMAX, j = e % RMAX;
    Gs[e] = (do_sweep && l < r && j < r) ? a.G[l * r + j] : 0.f;
  }
  for (int j = tid; j < RMAX; j += TR) scl[j] = (j < r) ? (a.scale ? a.scale[j] : 1.f) : 0.f;

  f32x16 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[t][q] = 0.f;
  float colsq = 0.f;   // thread j < r: running sum of F[:, j]^2

  const int64_t ntiles = ceil_div(a.N, TR);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * TR;
    const int rows = (int)((a.N - row0) < TR ? (a.N - row0) : TR);
    __syncthreads();   // previous tile's LDS readers are done
    // ---- stage F (scaled) and S
    for (int e = tid; e < TR * r; e += TR) {
      const int i = e / r, j = e % r;
      Fs[i * FROW + j] = (i < rows) ? a.F[(row0 + i) * r + j] * scl[j] : 0.f;
    }
    if (do_sweep) {
      const int nv = kp / 4;   // kp % 4 == 0 (padded sketches)
      for (int e = tid; e < TR * nv; e += TR) {
        const int i = e / nv, c4 = e % nv;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (i < rows) v = *(const f32x4*)(a.S + (row0 + i) * a.lds + 4 * c4);
        *(f32x4*)(Ss + i * SROW + 4 * c4) = v;
      }
    }
    __syncthreads();
    // ---- sweep: one thread per row
    if (do_sweep) {
      float f[RMAX], h[RMAX];
#pragma unroll
      for (int j = 0; j < RMAX; ++j) {
        f[j] = (j < r) ? Fs[tid * FROW + j] : 0.f;
        h[j] = 0.f;
      }
      for (int c = 0; c < kp; c += 4) {
        const f32x4 sv = *(const f32x4*)(Ss + tid * SROW + c);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float s = sv[u];
#pragma unroll
          for (int j = 0; j < RMAX; ++j) h[j] += s * Cs[(c + u) * RMAX + j];
        }
      }
#pragma unroll
      for (int j = 0; j < RMAX; ++j) {
        const float gjj = Gs[j * RMAX + j];
        if (gjj + a.beta > 0.f) {
          float t = h[j];
#pragma unroll
          for (int l = 0; l < RMAX; ++l) t -= f[l] * Gs[l * RMAX + j];
          const float v = plain ? f[j] + t / gjj : (f[j] * gjj + t - a.alpha) / (gjj + a.beta);
          f[j] = v > 0.f ? v : 0.f;
        }
      }
#pragma unroll
      for (int j = 0; j < RMAX; ++j)
        if (j < r) Fs[tid * FROW + j] = (tid < rows) ? f[j] : 0.f;
    }
    __syncthreads();
    // ---- write F back (coalesced) and stage the basis tile
    if (do_sweep) {
      for (int e = tid; e < rows * r; e += TR) {
        const int i = e / r, j = e % r;
        a.F[(row0 + i) * r + j] = Fs[i * FROW + j];
      }
    }
    {
      const int nv = kp / 4;
      for (int e = tid; e < TR * nv; e += TR) {
        const int i = e / nv, c4 = e % nv;
        f32x4 v = {0.f, 0.f, 0.f, 0.f};
        if (i < rows) v = *(const f32x4*)(a.Qb + (row0 + i) * a.ldq + 4 * c4);
        *(f32x4*)(Ss + i * SROW + 4 * c4) = v;
      }
      for (int e = tid; e < TR * (KPMAX - kp); e += TR) {   // zero the padded columns
        const int i = e / (KPMAX - kp), c = kp + e % (KPMAX - kp);
        Ss[i * SROW + c] = 0.f;
      }
    }
    __syncthreads();
    // ---- column sums of squares
    if (tid < r) {
      float s = 0.f;
      for (int i = 0; i < rows; ++i) {
        const float v = Fs[i * FROW + tid];
        s += v * v;
      }
      colsq += s;
    }
    // ---- partial Qb^T F on MFMA: A[c][i] = Qb[i][c], B[i][j] = F[i][j], contraction over rows
    const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = wave + 2 * t;
      if (tt < NT) {
        const int tm = tt / NTN, tn = tt % NTN;
        const int c = tm * 32 + l32, j = tn * 32 + l32;
        for (int kb = 0; kb < TR; kb += 8) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int i = kb + 4 * half + s;
            const float av = Ss[i * SROW + c];
            const float bv = (j < r) ? Fs[i * FROW + j] : 0.f;
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[t], 0, 0, 0);
          }
        }
      }
    }
  }
  // ---- write this workgroup's partial: [kp x r] then [r]
  float* P = a.part + (int64_t)blockIdx.x * (kp * r + r);
  const int half = lane >> 5, l32 = lane & 31;
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tt = wave + 2 * t;
    if (tt < NT) {
      const int tm = tt / NTN, tn = tt % NTN;
      const int j = tn * 32 + l32;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int c = tm * 32 + (q >> 2) * 8 + half * 4 + (q & 3);
        if (c < kp && j < r) P[c * r + j] = acc[t][q];
      }
    }
  }
  if (tid < r) P[kp * r + tid] = colsq;
}

// Sum partials in FP64 (fixed order), derive column norms, normalise, Gram.
// Every workgroup reduces 64 outputs with 4 thread groups; the last workgroup
// to finish (completion counter) does the r x r work and resets the counter.
__global__ void __launch_bounds__(256) finalize_kernel(FinalizeArgs a) {
  __shared__ double red[4][64];
  __shared__ int last;
  const int tid = threadIdx.x;
  const int ne = a.kp * a.r + a.r;
  const int e = blockIdx.x * 64 + (tid & 63), g = tid >> 6;
  double s = 0.0;
  if (e < ne)
    for (int b = g; b < a.nblk; b += 4) s += (double)a.part[(int64_t)b * ne + e];
  red[g][tid & 63] = s;
  __syncthreads();
  if (g == 0 && e < ne) a.accum[e] = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
  __threadfence();
  __syncthreads();
  if (tid == 0) last = (atomicAdd(a.counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int kp = a.kp, r = a.r;
  const volatile double* acc = a.accum;
  __shared__ double sc[256];
  for (int j = tid; j < r; j += 256) {
    double sj = 1.0;
    if (a.use_norms && a.normalize) {
      const double nrm = sqrt(acc[kp * r + j]);
      sj = nrm > 0.0 ? nrm : 1.0;
    }
    sc[j] = sj;
    if (a.use_norms) {
      if (a.scale_self) a.scale_self[j] = (float)(1.0 / sj);
      if (a.scale_other) a.scale_other[j] = (a.normalize == 1) ? (float)sj : 1.f;
    }
  }
  __syncthreads();
  for (int x = tid; x < kp * r; x += 256) a.C[x] = (float)(acc[x] / sc[x % r]);
  for (int x = tid; x < r * r; x += 256) {
    const int l = x / r, j = x % r;
    double t = 0.0;
    for (int c = 0; c < kp; ++c) t += (acc[c * r + l] / sc[l]) * (acc[c * r + j] / sc[j]);
    a.G[x] = (float)t;
  }
  if (tid == 0) *a.counter = 0u;
}

template <int RMAX, int KPMAX>
hipError_t run(const HalfStepArgs& a, int do_sweep, hipStream_t st) {
  hipLaunchKernelGGL((halfstep_kernel<RMAX, KPMAX>), dim3(halfstep_blocks(a.N)), dim3(TR), 0, st, a,
                     do_sweep);
  return hipGetLastError();
}

}  // namespace

int halfstep_blocks(int64_t N) {
  int64_t t = ceil_div(N, TR);
  if (t < 1) t = 1;
  return (int)(t < MAXBLK ? t : MAXBLK);
}

size_t halfstep_part_floats(int64_t N, int kp, int r) {
  return (size_t)halfstep_blocks(N) * (kp * r + r);
}

hipError_t launch_halfstep(const HalfStepArgs& a, int do_sweep, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  if (a.kp % 4 || a.lds % 4 || a.ldq % 4) return hipErrorInvalidValue;
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

hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t st) {
  const int ne = a.kp * a.r + a.r;
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)ceil_div(ne, 64)), dim3(256), 0, st, a);
  return hipGetLastError();
}
