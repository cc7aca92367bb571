// Learned warm start for H (extension; the paper has no learned component).
// Net: z1 = x W1 + b1, a1 = relu(z1); z2 = a1 W2 + b2, a2 = relu(z2);
// z3 = a2 W3 + b3, y = softplus(z3).  Inputs are the rows x-hat of Xh scaled by
// 1/||x-hat|| (H is positively homogeneous in X), outputs are multiplied back.
// Loss L = 1/(2B) sum ||y - t / ||x-hat||||^2, Adam (Kingma & Ba) on all
// parameters, He-normal initial weights, zero biases.
#include "common.h"

namespace {

// C[M x N] = op(A) op(B) (+ bias) with an epilogue, FP32 MFMA (32x32x2).
//   AT: A stored K x M (used transposed); BT: B stored N x K (used transposed).
//   EPI 0: plain; 1: relu; 2: multiply by (aux > 0) (ReLU backward mask).
// 64 x 64 output tile per 256-thread workgroup, waves 2 x 2 of 32 x 32.
template <bool AT, bool BT, int EPI>
__global__ void __launch_bounds__(256)
mlp_gemm_kernel(const float* __restrict__ A, int lda, const float* __restrict__ B, int ldb,
                float* __restrict__ C, int ldc, int M, int N, int K, const float* __restrict__ bias,
                const float* __restrict__ aux, int ldaux) {
  // BK = 64: eight K steps for the 512-deep layers, so fewer global-load
  // latencies are exposed between the (short) MFMA phases
  constexpr int BM = 64, BN = 64, BK = 64;
  constexpr int NV = BM * BK / 4 / 256;   // float4 per thread per operand (4)
  constexpr int NS = BM * BK / 256;       // scalars per thread per operand (16)
  static_assert(BM == BN, "square tiles");
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int i0 = blockIdx.x * BM, j0 = blockIdx.y * BN;
  f32x16 acc;
#pragma unroll
  for (int x = 0; x < 16; ++x) acc[x] = 0.f;
  // Operand tiles: A is BM x BK, B is BK x BN.  With vec (leading dimensions
  // multiples of 4, 16-byte aligned bases, K % 4 == 0) each thread loads two
  // float4 of each along the contiguous dimension; otherwise eight scalars.
  const bool vec = ((lda | ldb) & 3) == 0 && (K & 3) == 0 && (((uintptr_t)A | (uintptr_t)B) & 15) == 0;
  float va[NS], vb[NS];
  auto load = [&](int k0) {
    if (vec) {
#pragma unroll
      for (int p = 0; p < NV; ++p) {
        const int e = tid + 256 * p;
        int i, k;                 // A: float4 along k (!AT) or along i (AT)
        if (!AT) { i = e / (BK / 4); k = 4 * (e % (BK / 4)); } else { k = e / (BM / 4); i = 4 * (e % (BM / 4)); }
        const int gi = i0 + i, gk = k0 + k;
        f32x4 a = {0.f, 0.f, 0.f, 0.f};
        if (!AT) {
          if (gi < M && gk < K) a = *(const f32x4*)(A + (int64_t)gi * lda + gk);
        } else if (gk < K) {
          if (gi + 3 < M) a = *(const f32x4*)(A + (int64_t)gk * lda + gi);
          else
            for (int d = 0; d < 4; ++d) a[d] = gi + d < M ? A[(int64_t)gk * lda + gi + d] : 0.f;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) va[4 * p + d] = a[d];
        int j, kb;                // B: float4 along k (BT) or along j (!BT)
        if (BT) { j = e / (BK / 4); kb = 4 * (e % (BK / 4)); } else { kb = e / (BN / 4); j = 4 * (e % (BN / 4)); }
        const int gj = j0 + j, gkb = k0 + kb;
        f32x4 b = {0.f, 0.f, 0.f, 0.f};
        if (BT) {
          if (gj < N && gkb < K) b = *(const f32x4*)(B + (int64_t)gj * ldb + gkb);
        } else if (gkb < K) {
          if (gj + 3 < N) b = *(const f32x4*)(B + (int64_t)gkb * ldb + gj);
          else
            for (int d = 0; d < 4; ++d) b[d] = gj + d < N ? B[(int64_t)gkb * ldb + gj + d] : 0.f;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) vb[4 * p + d] = b[d];
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const int e = tid + 256 * p;
      int i, k;
      if (!AT) { i = e / BK; k = e % BK; } else { k = e / BM; i = e % BM; }
      const int gi = i0 + i, gk = k0 + k;
      va[p] = (gi < M && gk < K) ? (AT ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]) : 0.f;
      int j, kb;
      if (BT) { j = e / BK; kb = e % BK; } else { kb = e / BN; j = e % BN; }
      const int gj = j0 + j, gkb = k0 + kb;
      vb[p] = (gj < N && gkb < K) ? (BT ? B[(int64_t)gj * ldb + gkb] : B[(int64_t)gkb * ldb + gj]) : 0.f;
    }
  };
  auto store = [&]() {
    if (vec) {
#pragma unroll
      for (int p = 0; p < NV; ++p) {
        const int e = tid + 256 * p;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          if (!AT) As[4 * (e % (BK / 4)) + d][e / (BK / 4)] = va[4 * p + d];
          else As[e / (BM / 4)][4 * (e % (BM / 4)) + d] = va[4 * p + d];
          if (BT) Bs[4 * (e % (BK / 4)) + d][e / (BK / 4)] = vb[4 * p + d];
          else Bs[e / (BN / 4)][4 * (e % (BN / 4)) + d] = vb[4 * p + d];
        }
      }
      return;
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      const int e = tid + 256 * p;
      int i, k;
      if (!AT) { i = e / BK; k = e % BK; } else { k = e / BM; i = e % BM; }
      As[k][i] = va[p];
      int j, kb;
      if (BT) { j = e / BK; kb = e % BK; } else { kb = e / BN; j = e % BN; }
      Bs[kb][j] = vb[p];
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  load(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
#pragma unroll 8
    for (int kk = 0; kk < BK; kk += 2) {
      const float a = As[kk + half][wm * 32 + l32];
      const float b = Bs[kk + half][wn * 32 + l32];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
  }
  // D[i][j]: lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
  const int gj = j0 + wn * 32 + l32;
#pragma unroll
  for (int x = 0; x < 16; ++x) {
    const int gi = i0 + wm * 32 + (x >> 2) * 8 + half * 4 + (x & 3);
    if (gi < M && gj < N) {
      float v = acc[x];
      if (bias) v += bias[gj];
      if (EPI == 1) v = v > 0.f ? v : 0.f;
      if (EPI == 2) v = aux[(int64_t)gi * ldaux + gj] > 0.f ? v : 0.f;
      C[(int64_t)gi * ldc + gj] = v;
    }
  }
}

// Row norms of X (B x k) and the scaled rows: Xs = X / ||x|| (0 for a zero row);
// T (if given) is scaled the same way into Ts.  Source row b is idx[b] when an
// index list is given (a training batch drawn from the pair set), else b.
__global__ void __launch_bounds__(256)
scale_rows_kernel(const float* __restrict__ X, int64_t ldx, const int* __restrict__ idx, int64_t nsrc, int Bn,
                  int k, const float* __restrict__ T, int64_t ldt, int r, float* __restrict__ Xs,
                  float* __restrict__ Ts, float* __restrict__ nrm) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= Bn) return;
  const int64_t src = idx ? (int64_t)idx[row] : (int64_t)row;
  if (src < 0 || src >= nsrc) {   // an index outside the pair set contributes a zero pair
    for (int c = lane; c < k; c += 64) Xs[(int64_t)row * k + c] = 0.f;
    if (T)
      for (int c = lane; c < r; c += 64) Ts[(int64_t)row * r + c] = 0.f;
    if (lane == 0) nrm[row] = 0.f;
    return;
  }
  double s = 0.0;
  for (int c = lane; c < k; c += 64) {
    const double v = X[src * ldx + c];
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  const double nv = sqrt(s);
  const float inv = nv > 0.0 ? (float)(1.0 / nv) : 0.f;
  for (int c = lane; c < k; c += 64) Xs[(int64_t)row * k + c] = X[src * ldx + c] * inv;
  if (T)
    for (int c = lane; c < r; c += 64) Ts[(int64_t)row * r + c] = T[src * ldt + c] * inv;
  if (lane == 0) nrm[row] = (float)nv;
}

NMF_DEV float quad_bcast_f(float v, int src) {
  const int x = __builtin_bit_cast(int, v);
  int y;
  switch (src) {   // folds to one DPP move once src is a constant
    case 0: y = __builtin_amdgcn_mov_dpp(x, 0x00, 0xF, 0xF, false); break;
    case 1: y = __builtin_amdgcn_mov_dpp(x, 0x55, 0xF, 0xF, false); break;
    case 2: y = __builtin_amdgcn_mov_dpp(x, 0xAA, 0xF, 0xF, false); break;
    default: y = __builtin_amdgcn_mov_dpp(x, 0xFF, 0xF, 0xF, false); break;
  }
  return __builtin_bit_cast(float, y);
}

// Column NNLS min_{h >= 0} ||x - Wh h||^2 for every row x of Xr (n x k), by
// repeated H sweeps of eq fastHALS_a with Wh fixed, starting from h = 0 (or
// from the rows already in H when warm):
//   h_j <- [h_j + (p_j - (G h)_j) / G_jj]_+ ,  p = Wh^T x,  G = Wh^T Wh,
// j ascending (Gauss-Seidel); components with G_jj = 0 stay unchanged.
// A quad of lanes per row; lane q owns components q RQ .. q RQ + RQ - 1 of h,
// p and the gradient g = p - G h.  g is formed afresh at the start of every
// sweep (each lane sums over all components, taking the others' h from their
// lanes); within the sweep, component j's change d = h_j' - h_j is passed from
// its lane to the quad and every lane takes g -= G[:, j] d for its components.
// The serial chain per component is then the update, one lane move and one
// FMA (the same arithmetic as the direct form up to rounding).  Wh, G and
// 1/G_jj are staged in LDS, zero padded to RMAX columns.  64 rows per
// 256-thread block.
template <int RMAX>
__global__ void __launch_bounds__(256)
nnls_rows_kernel(const float* __restrict__ Xr, int64_t ldx, int n, int k, const float* __restrict__ Wh, int r,
                 int sweeps, int warm, float* __restrict__ H, int64_t ldh) {
  constexpr int RQ = RMAX / 4;
  extern __shared__ float sm[];
  float* whs = sm;                      // k x RMAX
  float* gs = sm + k * RMAX;            // RMAX x RMAX
  float* rd = gs + RMAX * RMAX;         // RMAX
  for (int e = threadIdx.x; e < k * RMAX; e += 256) {
    const int c = e / RMAX, j = e % RMAX;
    whs[e] = j < r ? Wh[(int64_t)c * r + j] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < RMAX * RMAX; e += 256) {
    const int a = e / RMAX, b = e % RMAX;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += (double)whs[c * RMAX + a] * whs[c * RMAX + b];
    gs[e] = (float)s;
    if (a == b) rd[a] = s > 0.0 ? (float)(1.0 / s) : 0.f;
  }
  __syncthreads();
  const int q = threadIdx.x & 3;
  const int row = blockIdx.x * 64 + (threadIdx.x >> 2);
  const bool valid = row < n;
  const int c0 = q * RQ;
  float f[RQ], p[RQ];
#pragma unroll
  for (int t = 0; t < RQ; ++t) {
    f[t] = (warm && valid && c0 + t < r) ? H[(int64_t)row * ldh + c0 + t] : 0.f;
    p[t] = 0.f;
  }
  for (int c = 0; c < k; ++c) {
    const float x = valid ? Xr[(int64_t)row * ldx + c] : 0.f;
#pragma unroll
    for (int t = 0; t < RQ; t += 4) {
      const f32x4 w = *(const f32x4*)(whs + c * RMAX + c0 + t);
      p[t] = fmaf(x, w[0], p[t]);
      p[t + 1] = fmaf(x, w[1], p[t + 1]);
      p[t + 2] = fmaf(x, w[2], p[t + 2]);
      p[t + 3] = fmaf(x, w[3], p[t + 3]);
    }
  }
  for (int it = 0; it < sweeps; ++it) {
    // g = p - G h, with h of every component taken from its lane
    float g[RQ];
#pragma unroll
    for (int t = 0; t < RQ; ++t) g[t] = p[t];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
      for (int u = 0; u < RQ; ++u) {
        const float hv = quad_bcast_f(f[u], qq);          // h of component qq RQ + u
        const int col = qq * RQ + u;
#pragma unroll
        for (int t = 0; t < RQ; t += 4) {
          const f32x4 gv = *(const f32x4*)(gs + col * RMAX + c0 + t);   // G symmetric: G[c0 + t][col]
          g[t] = fmaf(-gv[0], hv, g[t]);
          g[t + 1] = fmaf(-gv[1], hv, g[t + 1]);
          g[t + 2] = fmaf(-gv[2], hv, g[t + 2]);
          g[t + 3] = fmaf(-gv[3], hv, g[t + 3]);
        }
      }
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
      const float rdj = rd[j];
      if (rdj > 0.f) {                  // uniform over the block
        const int t = j % RQ;
        const float fn = fmaxf(fmaf(g[t], rdj, f[t]), 0.f);
        const float d = quad_bcast_f(fn - f[t], j / RQ);  // the owner's change
        if (q == j / RQ) f[t] = fn;
#pragma unroll
        for (int u = 0; u < RQ; u += 4) {
          const f32x4 gv = *(const f32x4*)(gs + j * RMAX + c0 + u);
          g[u] = fmaf(-gv[0], d, g[u]);
          g[u + 1] = fmaf(-gv[1], d, g[u + 1]);
          g[u + 2] = fmaf(-gv[2], d, g[u + 2]);
          g[u + 3] = fmaf(-gv[3], d, g[u + 3]);
        }
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int t = 0; t < RQ; ++t)
      if (c0 + t < r) H[(int64_t)row * ldh + c0 + t] = f[t];
  }
}

// The same column NNLS for wide factors (64 < r <= 128, k <= 256), where Wh and
// G no longer fit in LDS together.  G = Wh^T Wh is formed by each workgroup on
// FP64 MFMA from Wh in global memory (upper 16 x 16 blocks, mirrored) and staged
// permuted; p = Wh^T x goes through LDS in 64-row chunks of Wh.  Components are
// interleaved over the quad (lane q owns components 4 u + q), and the gradient
// g = p - G h is formed once from the starting rows, then kept exact by
// g -= G[:, j] d after every change d of component j, over all sweeps.
__global__ void __launch_bounds__(256)
nnls_rows_wide_kernel(const float* __restrict__ Xr, int64_t ldx, int n, int k, const float* __restrict__ Wh, int r,
                      int sweeps, int warm, float* __restrict__ H, int64_t ldh) {
  constexpr int RM = 128, RQ = RM / 4, CH = 64;
  __shared__ __attribute__((aligned(16))) float Gq[RM * RM];    // Gq[c][q][u] = G[c][4 u + q]
  __shared__ __attribute__((aligned(16))) float Wq[CH * RM];    // Wq[c][q][u] = Wh[c0 + c][4 u + q]
  __shared__ float rd[RM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, g4 = lane >> 4;
  // G on FP64 MFMA: blocks (ti, tj), ti <= tj, dealt over the four waves
  for (int t = wave; t < 36; t += 4) {
    int ti = 0, rem = t;
    while (rem >= 8 - ti) { rem -= 8 - ti; ++ti; }
    const int tj = ti + rem;
    f64x4 d = {0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < k; c0 += 4) {
      const int c = c0 + g4;
      const int ja = 16 * ti + l16, jb = 16 * tj + l16;
      const double a = (c < k && ja < r) ? (double)Wh[(int64_t)c * r + ja] : 0.0;
      const double b = (c < k && jb < r) ? (double)Wh[(int64_t)c * r + jb] : 0.0;
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {   // D[i][j] in lane j + 16 (i % 4), register i / 4
      const int i = 16 * ti + 4 * x + g4, j = 16 * tj + l16;
      const float v = (float)d[x];
      Gq[i * RM + (j & 3) * RQ + (j >> 2)] = v;
      Gq[j * RM + (i & 3) * RQ + (i >> 2)] = v;
      if (i == j) rd[i] = (i < r && d[x] > 0.0) ? (float)(1.0 / d[x]) : 0.f;
    }
  }
  const int q = tid & 3;
  const int row = blockIdx.x * 64 + (tid >> 2);
  const bool valid = row < n;
  float f[RQ], g[RQ];
#pragma unroll
  for (int u = 0; u < RQ; ++u) {
    const int c = 4 * u + q;
    f[u] = (warm && valid && c < r) ? H[(int64_t)row * ldh + c] : 0.f;
    g[u] = 0.f;
  }
  // p = Wh^T x (into g)
  for (int c0 = 0; c0 < k; c0 += CH) {
    __syncthreads();
    for (int e = tid; e < CH * RM; e += 256) {
      const int c = e / RM, j = e % RM;
      Wq[c * RM + (j & 3) * RQ + (j >> 2)] = (c0 + c < k && j < r) ? Wh[(int64_t)(c0 + c) * r + j] : 0.f;
    }
    __syncthreads();
    const int cn = k - c0 < CH ? k - c0 : CH;
    for (int c = 0; c < cn; ++c) {
      const float x = valid ? Xr[(int64_t)row * ldx + c0 + c] : 0.f;
      const float* w = Wq + c * RM + q * RQ;
#pragma unroll
      for (int u = 0; u < RQ; u += 4) {
        const f32x4 wv = *(const f32x4*)(w + u);
        g[u] = fmaf(x, wv[0], g[u]);
        g[u + 1] = fmaf(x, wv[1], g[u + 1]);
        g[u + 2] = fmaf(x, wv[2], g[u + 2]);
        g[u + 3] = fmaf(x, wv[3], g[u + 3]);
      }
    }
  }
  __syncthreads();
  // g = p - G h with h of every component from its lane (G symmetric: G[4u+q][col] = Gq[col][q][u])
  if (warm) {
#pragma unroll
    for (int qq = 0; qq < 4; ++qq)
#pragma unroll
      for (int v = 0; v < RQ; ++v) {
        const float hv = quad_bcast_f(f[v], qq);
        const float* gr = Gq + (4 * v + qq) * RM + q * RQ;
#pragma unroll
        for (int u = 0; u < RQ; u += 4) {
          const f32x4 gv = *(const f32x4*)(gr + u);
          g[u] = fmaf(-gv[0], hv, g[u]);
          g[u + 1] = fmaf(-gv[1], hv, g[u + 1]);
          g[u + 2] = fmaf(-gv[2], hv, g[u + 2]);
          g[u + 3] = fmaf(-gv[3], hv, g[u + 3]);
        }
      }
  }
  for (int it = 0; it < sweeps; ++it) {
    // fully unrolled (compile-time register indices), no branch: a component with
    // G_jj = 0 (1/G_jj stored as 0) keeps its value, so its d is 0
#pragma clang loop unroll(full)
    for (int j = 0; j < RM; ++j) {
      const float rdj = rd[j];
      const int t = j >> 2;
      const float fn = rdj > 0.f ? fmaxf(fmaf(g[t], rdj, f[t]), 0.f) : f[t];
      const float d = quad_bcast_f(fn - f[t], j & 3);   // the owner's change
      if (q == (j & 3)) f[t] = fn;
      const float* gr = Gq + j * RM + q * RQ;
#pragma unroll
      for (int u = 0; u < RQ; u += 4) {
        const f32x4 gv = *(const f32x4*)(gr + u);
        g[u] = fmaf(-gv[0], d, g[u]);
        g[u + 1] = fmaf(-gv[1], d, g[u + 1]);
        g[u + 2] = fmaf(-gv[2], d, g[u + 2]);
        g[u + 3] = fmaf(-gv[3], d, g[u + 3]);
      }
      __builtin_amdgcn_sched_barrier(0);   // keep each step's loads with it (register pressure)
    }
  }
  if (valid) {
#pragma unroll
    for (int u = 0; u < RQ; ++u) {
      const int c = 4 * u + q;
      if (c < r) H[(int64_t)row * ldh + c] = f[u];
    }
  }
}

NMF_DEV float softplusf(float z) { return fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))); }
NMF_DEV float sigmoidf(float z) {
  if (z >= 0.f) return 1.f / (1.f + expf(-z));
  const float e = expf(z);
  return e / (1.f + e);
}

// dZ3 = (softplus(z3) - t) / B * sigmoid(z3); per-block FP64 partial of the loss.
__global__ void __launch_bounds__(256)
loss_grad_kernel(const float* __restrict__ Z3, const float* __restrict__ Ts, int Bn, int r,
                 float* __restrict__ dZ3, double* __restrict__ lpart) {
  __shared__ double red[256];
  const int64_t total = (int64_t)Bn * r;
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const float z = Z3[e];
    const float d = softplusf(z) - Ts[e];
    s += (double)d * d;
    dZ3[e] = d / (float)Bn * sigmoidf(z);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// loss = sum(lpart) / (2B), accumulated into *acc (FP64); one thread.
__global__ void loss_sum_kernel(const double* __restrict__ lpart, int nb, int Bn, double* __restrict__ out,
                                double* __restrict__ acc) {
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += lpart[i];
  s /= 2.0 * Bn;
  out[0] = s;
  if (acc) acc[0] += s;
}

// gb[j] = sum_i dZ[i][j] (FP64, fixed order over rows in 8 slices).
__global__ void __launch_bounds__(256)
colsum_kernel(const float* __restrict__ dZ, int Bn, int N, float* __restrict__ gb) {
  __shared__ double red[8][33];
  const int jj = threadIdx.x & 31, sl = threadIdx.x >> 5;
  const int j = blockIdx.x * 32 + jj;
  double s = 0.0;
  if (j < N)
    for (int i = sl; i < Bn; i += 8) s += dZ[(int64_t)i * N + j];
  red[sl][jj] = s;
  __syncthreads();
  if (sl == 0 && j < N) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) t += red[q][jj];
    gb[j] = (float)t;
  }
}

__global__ void __launch_bounds__(256)
adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1, float* __restrict__ m2,
            int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float gv = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gv;
    const float b = b2 * m2[e] + (1.f - b2) * gv * gv;
    m1[e] = a;
    m2[e] = b;
    p[e] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
}

// out = softplus(z3) * ||x||
__global__ void __launch_bounds__(256)
infer_out_kernel(const float* __restrict__ Z3, const float* __restrict__ nrm, int Bn, int r,
                 float* __restrict__ out, int64_t ldo) {
  const int64_t total = (int64_t)Bn * r;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / r, j = e - i * r;
    out[i * ldo + j] = softplusf(Z3[e]) * nrm[i];
  }
}

// Warm-start selection: rho(h) = ||x - Wh h||^2 in FP64 for the net's and the
// cold rows; keep the net's row unless it is worse.  One wave per row; lane c
// (and c + 64, ... up to k) forms (Wh h)_c with j ascending, the lanes' squared
// differences are summed over c ascending and then across the wave.  Wh is
// staged in LDS transposed (whs[j][c], row stride kpp = k rounded up to 64, zero
// padded) so the lanes read consecutive words.
__global__ void __launch_bounds__(256)
select_kernel(const float* __restrict__ Xh, int64_t ldx, int n, int k, const float* __restrict__ Wh, int r,
              const float* __restrict__ Hn, const float* __restrict__ Hc, float* __restrict__ Hout,
              int* __restrict__ rejected) {
  extern __shared__ float whs[];                 // r x kpp
  __shared__ float hs[4][2][128];                // the wave's rows of Hn and Hc (r <= 128)
  const int kpp = (k + 63) & ~63, nt = kpp >> 6;
  for (int e = threadIdx.x; e < kpp * r; e += 256) {
    const int j = e / kpp, c = e - j * kpp;
    whs[e] = c < k ? Wh[c * r + j] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int row = blockIdx.x * 4 + wave; row < n; row += gridDim.x * 4) {
    double pn[4] = {0.0, 0.0, 0.0, 0.0}, pc[4] = {0.0, 0.0, 0.0, 0.0};
    const float* hn = Hn + (int64_t)row * r;
    const float* hc = Hc + (int64_t)row * r;
    for (int j = lane; j < 128; j += 64) {
      hs[wave][0][j] = j < r ? hn[j] : 0.f;
      hs[wave][1][j] = j < r ? hc[j] : 0.f;
    }
    for (int j = 0; j < r; ++j) {
      const double a = hs[wave][0][j], b = hs[wave][1][j];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nt) {
          const double w = whs[j * kpp + 64 * t + lane];
          pn[t] += w * a;
          pc[t] += w * b;
        }
    }
    double rn = 0.0, rc = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 64 * t + lane;
      if (c < k) {
        const double x = Xh[(int64_t)row * ldx + c];
        rn += (x - pn[t]) * (x - pn[t]);
        rc += (x - pc[t]) * (x - pc[t]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      rn += __shfl_xor(rn, off);
      rc += __shfl_xor(rc, off);
    }
    const bool rej = rn > rc;
    for (int j = lane; j < r; j += 64) Hout[(int64_t)row * r + j] = rej ? hc[j] : hn[j];
    if (lane == 0) rejected[row] = rej ? 1 : 0;
  }
}

__global__ void count_kernel(const int* __restrict__ flags, int n, long long* __restrict__ out) {
  __shared__ long long red[256];
  long long s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += flags[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

unsigned g1(int64_t total) {
  int64_t g = ceil_div(total, 256);
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_mlp_gemm(int at, int bt, int epi, const float* A, int lda, const float* B, int ldb,
                           float* C, int ldc, int M, int N, int K, const float* bias, const float* aux,
                           int ldaux, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 grid((unsigned)ceil_div(M, 64), (unsigned)ceil_div(N, 64));
#define MLP_GEMM_CASE(AT_, BT_, EPI_)                                                                  \
  if (at == AT_ && bt == BT_ && epi == EPI_) {                                                         \
    hipLaunchKernelGGL((mlp_gemm_kernel<AT_, BT_, EPI_>), grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, \
                       M, N, K, bias, aux, ldaux);                                                     \
    return hipGetLastError();                                                                          \
  }
  MLP_GEMM_CASE(false, false, 0)
  MLP_GEMM_CASE(false, false, 1)
  MLP_GEMM_CASE(false, true, 0)
  MLP_GEMM_CASE(false, true, 2)
  MLP_GEMM_CASE(true, false, 0)
#undef MLP_GEMM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_scale_rows(const float* X, int64_t ldx, const int* idx, int64_t nsrc, int Bn, int k,
                             const float* T, int64_t ldt, int r, float* Xs, float* Ts, float* nrm, hipStream_t st) {
  if (Bn == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)ceil_div(Bn, 4)), dim3(256), 0, st, X, ldx, idx, nsrc, Bn,
                     k, T, ldt, r, Xs, Ts, nrm);
  return hipGetLastError();
}

size_t nnls_rows_lds_bytes(int k, int r) {
  if (r > 64) return 0;   // the wide-factor kernel has static LDS only
  const int rmax = r <= 16 ? 16 : r <= 32 ? 32 : 64;
  return (size_t)(k * rmax + rmax * rmax + rmax) * sizeof(float);
}

hipError_t launch_nnls_rows(const float* Xr, int64_t ldx, int n, int k, const float* Wh, int r, int sweeps,
                            int warm, float* H, int64_t ldh, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t lds = nnls_rows_lds_bytes(k, r);
  const dim3 grid((unsigned)ceil_div(n, 64));
  if (r <= 16)
    hipLaunchKernelGGL(nnls_rows_kernel<16>, grid, dim3(256), lds, st, Xr, ldx, n, k, Wh, r, sweeps, warm, H, ldh);
  else if (r <= 32)
    hipLaunchKernelGGL(nnls_rows_kernel<32>, grid, dim3(256), lds, st, Xr, ldx, n, k, Wh, r, sweeps, warm, H, ldh);
  else if (r <= 64)
    hipLaunchKernelGGL(nnls_rows_kernel<64>, grid, dim3(256), lds, st, Xr, ldx, n, k, Wh, r, sweeps, warm, H, ldh);
  else if (r <= 128 && k <= 256)
    hipLaunchKernelGGL(nnls_rows_wide_kernel, grid, dim3(256), 0, st, Xr, ldx, n, k, Wh, r, sweeps, warm, H, ldh);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int loss_blocks(int Bn, int r) { return (int)g1((int64_t)Bn * r) < 256 ? (int)g1((int64_t)Bn * r) : 256; }

hipError_t launch_loss_grad(const float* Z3, const float* Ts, int Bn, int r, float* dZ3, double* lpart,
                            double* loss_out, double* loss_acc, hipStream_t st) {
  const int nb = loss_blocks(Bn, r);
  hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(256), 0, st, Z3, Ts, Bn, r, dZ3, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(1), 0, st, lpart, nb, Bn, loss_out, loss_acc);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* dZ, int Bn, int N, float* gb, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((unsigned)ceil_div(N, 32)), dim3(256), 0, st, dZ, Bn, N, gb);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m1, float* m2, int64_t n, float lr, int t,
                       hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = (float)(1.0 - pow(0.9, t)), c2 = (float)(1.0 - pow(0.999, t));
  hipLaunchKernelGGL(adam_kernel, dim3(g1(n)), dim3(256), 0, st, p, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_infer_out(const float* Z3, const float* nrm, int Bn, int r, float* out, int64_t ldo,
                            hipStream_t st) {
  hipLaunchKernelGGL(infer_out_kernel, dim3(g1((int64_t)Bn * r)), dim3(256), 0, st, Z3, nrm, Bn, r, out, ldo);
  return hipGetLastError();
}

hipError_t launch_count(const int* flags, int n, long long* count, hipStream_t st) {
  hipLaunchKernelGGL(count_kernel, dim3(1), dim3(256), 0, st, flags, n, count);
  return hipGetLastError();
}

hipError_t launch_select(const float* Xh, int64_t ldx, int n, int k, const float* Wh, int r, const float* Hn,
                         const float* Hc, float* Hout, int* rejected, long long* count, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (k > 256 || r > 128) return hipErrorInvalidValue;
  const int64_t nb = ceil_div(n, 4);
  const size_t lds = (size_t)((k + 63) & ~63) * r * sizeof(float);
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)(nb < 256 ? nb : 256)), dim3(256), lds, st, Xh, ldx, n, k, Wh,
                     r, Hn, Hc, Hout, rejected);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(count_kernel, dim3(1), dim3(256), 0, st, rejected, n, count);
  return hipGetLastError();
}
