// FastHALS-RP half-steps (eq fastHALS_a) for wide factors: r up to 128 and k'
// up to 256, where the compressed factor C (k' x r) and its Gram G (r x r) no
// longer fit beside the row tiles in one workgroup's LDS.  The half-step is
// four launches (plus the fixed-order sum of the partials):
//
//   prep   C = (the other side's Qb'^T F') / its column norms when they come
//          from the W side (the normalisation at the end of Sec 4), G = C^T C
//          on FP64 MFMA, 1/(G_jj + beta), the column scales of F;
//   grad   a = S C - (F diag(scl)) U for every row, U the strictly lower
//          triangle of G (a_l = the row of X-check B-check or X-hat^T A-hat at
//          l minus the terms of the components after l), one FP32 MFMA product
//          with the two operand pairs concatenated along K;
//   sweep  the Gauss-Seidel sweep j = 1..r of each row (the rule
//          f_j <- [f_j + g_j / G_jj]_+, Sec 4.1: [(f_j G_jj + g_j - alpha) /
//          (G_jj + beta)]_+) as a forward substitution over a;
//   qtf    this side's partials Qb^T F (the other side's compressed factor)
//          and the column sums of F^2, per workgroup, on FP32 MFMA.
//
// Semantics (scales, published C / G / 1/||a_j||, alpha, beta, normalisation
// modes) are those of the fused kernel for narrower factors.
#include <algorithm>

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
// a (N x r, ld r) = [S | F diag(scl)] [C ; -U]: K runs over the kp columns of S
// (padded to a multiple of 32 with zeros), then over the BR columns of F, with
// U[i][l] = G_il for i > l, else 0, and alpha subtracted.  A component that
// keeps its value (1/(G_ll + beta) = 0: a zero column of C, or padding) gets
// a_l = f_l scl_l instead (column l of C zeroed, column l of -U the unit vector,
// no alpha), and its row of G stays whole in the product (the sweep never
// corrects for it).
// 256 threads, 2 x 2 waves over a BM x 128 tile; v_mfma_f32_32x32x2_f32 with
// the k order permuted within groups of 8 so that a lane reads its four A and
// its four B values of a group as one 16-byte LDS load each (lanes 0-31 take
// k = 8 g + s, lanes 32-63 k = 8 g + 4 + s in step s): A is staged row-major
// and B transposed (each thread loads a 4 x 4 block of B and transposes it in
// registers), both with row stride 36 floats, which keeps 16-byte accesses
// free of bank conflicts.  The fragments of group g + 1 are read from LDS while
// the MFMAs of group g run, and the next K step is loaded into registers while
// the LDS tile is consumed.
template <int BM, bool FVEC>   // FVEC: rows of F are 16-byte aligned (r % 4 == 0)
__global__ void __launch_bounds__(256)
hs_grad_kernel(const float* __restrict__ S, int64_t lds, const float* __restrict__ F, const float* __restrict__ scl,
               const float* __restrict__ Cp, const float* __restrict__ Gp, const float* __restrict__ rdiag,
               float alpha, float* __restrict__ gout, int64_t N, int kp, int r) {
  constexpr int BK = 32, BN = BR, WM = 2, WN = 2;
  constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  constexpr int AROW = BK + 4, BROW = BK + 4;
  constexpr int AP = BM * BK / 4 / 256;    // A float4 per thread
  static_assert(BK * BN / 16 == 256, "one 4 x 4 block of B per thread");
  __shared__ __attribute__((aligned(16))) float As[BM * AROW];
  __shared__ __attribute__((aligned(16))) float Bt[BN * BROW];   // Bt[j][k] = B[k][j]
  __shared__ float sc[BR], rdl[BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  if (tid < BR) {
    sc[tid] = scl[tid];
    rdl[tid] = rdiag[tid];
  }
  // any component below r that keeps its value (rare): the general operand masks
  const bool anykept = __syncthreads_or(tid < r && rdiag[tid] == 0.f);
  const int ks = (kp + BK - 1) / BK;       // K steps over S, then BR / BK over F
  f32x16 acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.f;
  f32x4 ra[AP];                            // A: row (t / 8) + 32 p, columns 4 (t % 8) .. +3 of the step
  f32x4 rb[4];                             // B: rows 4 kq .. +3, columns 4 c4 .. +3 of the step
  const int kq = tid >> 5, c4 = tid & 31, ca = 4 * (tid & 7);
  const f32x4 z4 = {0.f, 0.f, 0.f, 0.f};
  auto kept = [&](int l) { return l < r && rdl[l] == 0.f; };
  // Loads are unconditional, from clamped addresses, and out-of-range elements
  // are zeroed when the tile is stored: guarded loads become exec-masked blocks
  // whose waits serialise them.  Rows of C up to 255 and of G up to 127 lie
  // inside their buffers.
  auto loadS = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int64_t gi = i0 + (tid >> 3) + 32 * p;
      const bool ok = gi < N && k0 + ca < kp;
      ra[p] = *(const f32x4*)(S + (ok ? gi * lds + k0 + ca : 0));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = *(const f32x4*)(Cp + (int64_t)(k0 + 4 * kq + e) * BR + 4 * c4);
  };
  auto loadF = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int64_t gi = i0 + (tid >> 3) + 32 * p;
      if (FVEC) {
        const bool ok = gi < N && k0 + ca < r;
        ra[p] = *(const f32x4*)(F + (ok ? gi * r + k0 + ca : 0));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[p][e] = F[(gi < N && k0 + ca + e < r) ? gi * r + k0 + ca + e : 0];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = *(const f32x4*)(Gp + (int64_t)(k0 + 4 * kq + e) * BR + 4 * c4);
  };
  auto storeA = [&](int k0, int lim, bool fs) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int row = (tid >> 3) + 32 * p;
      const bool rok = i0 + row < N;
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = fs ? ra[p][e] * sc[k0 + ca + e] : ra[p][e];   // the pending column scales of F
        v[e] = (rok && k0 + ca + e < lim) ? x : 0.f;
      }
      *(f32x4*)(As + row * AROW + ca) = v;
    }
  };
  // column 4 c4 + d of the rows 4 kq .. 4 kq + 3 goes to Bt[4 c4 + d][4 kq ..]
  auto storeS = [&](int k0) {
    storeA(k0, kp, false);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int l = 4 * c4 + d;
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = k0 + 4 * kq + e < kp ? rb[e][d] : 0.f;   // rows of C past kp are stale
      if (anykept && kept(l)) v = z4;
      *(f32x4*)(Bt + l * BROW + 4 * kq) = v;
    }
  };
  auto storeF = [&](int k0) {
    storeA(k0, r, true);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int l = 4 * c4 + d;
      f32x4 v;
      if (!anykept) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = k0 + 4 * kq + e > l ? -rb[e][d] : 0.f;
      } else {
        const bool kl = kept(l);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = k0 + 4 * kq + e;
          v[e] = kl ? (i == l ? 1.f : 0.f) : ((kept(i) || i > l) ? -rb[e][d] : 0.f);
        }
      }
      *(f32x4*)(Bt + l * BROW + 4 * kq) = v;
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  auto mma = [&]() {
#pragma unroll
    for (int gq = 0; gq < BK / 8; ++gq) {
      const int kb = 8 * gq + 4 * half;
      f32x4 af[TM], bf[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) af[x] = *(const f32x4*)(As + (wm * (BM / WM) + 32 * x + l32) * AROW + kb);
#pragma unroll
      for (int y = 0; y < TN; ++y) bf[y] = *(const f32x4*)(Bt + (wn * (BN / WN) + 32 * y + l32) * BROW + kb);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int x = 0; x < TM; ++x)
#pragma unroll
          for (int y = 0; y < TN; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[x][s], bf[y][s], acc[x][y], 0, 0, 0);
    }
  };
  // the next step's loads are issued before this step's MFMAs (the scheduler
  // would otherwise sink them behind the MFMAs and expose their latency)
  __syncthreads();
  loadS(0);
  for (int t = 0; t < ks; ++t) {
    storeS(t * BK);
    __syncthreads();
    if (t + 1 < ks) loadS((t + 1) * BK);
    else loadF(0);
    __builtin_amdgcn_sched_barrier(0);
    mma();
    __syncthreads();
  }
  for (int t = 0; t < BR / BK; ++t) {
    storeF(t * BK);
    __syncthreads();
    if (t + 1 < BR / BK) loadF((t + 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
    mma();
    __syncthreads();
  }
  // D[i][j] of a 32 x 32 tile: lane j + 32 ((i / 4) % 2), register (i / 8) 4 + i % 4
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      const int j = wn * (BN / WN) + 32 * y + l32;
      const float aj = kept(j) ? 0.f : alpha;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int il = (e >> 2) * 8 + half * 4 + (e & 3);
        const int64_t gi = i0 + wm * (BM / WM) + 32 * x + il;
        if (gi < N && j < r) gout[gi * r + j] = acc[x][y][e] - aj;
      }
    }
}

// hi and lo BF16 halves of (a, b), packed (a in the low half), nearest even:
// v = hi + lo + d with |d| <= 2^-16 |v|, v - hi exact in FP32.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
NMF_DEV void split_pair(float a, float b, uint32_t& h, uint32_t& l) {
  const f32x2_t v = {a, b};
  h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
  const f32x2_t w = {a - __builtin_bit_cast(float, h << 16), b - __builtin_bit_cast(float, h & 0xFFFF0000u)};
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector(w, bf16x2_t));
}
// Three BF16 parts: v = hi + mid + lo exactly (v - hi and then v - hi - mid are
// exact in FP32 and the last remainder has at most 8 significant bits), unless
// the parts fall below the BF16 normal range.
NMF_DEV void split3_pair(float a, float b, uint32_t& h, uint32_t& m, uint32_t& l) {
  split_pair(a, b, h, m);
  const float ra = a - __builtin_bit_cast(float, h << 16), rb = b - __builtin_bit_cast(float, h & 0xFFFF0000u);
  const f32x2_t w = {ra - __builtin_bit_cast(float, m << 16), rb - __builtin_bit_cast(float, m & 0xFFFF0000u)};
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector(w, bf16x2_t));
}

// The gradient product of hs_grad_kernel on BF16 MFMA with three-part operands:
// every operand value is carried as hi + mid + lo (split3_pair, exact), and a
// term as the six products of parts whose orders sum to at most two (lo lo,
// lo mid and mid lo, below 2^-24 |s||c|, are dropped), on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation: FP32 accuracy.  Two parts
// do not suffice here: a = S C - F U nearly cancels as the sweep converges, and
// 16-bit operands move the factors measurably (the Q^T F product, a sum of
// like-signed terms, keeps two parts).  Loads, masks, scales and the epilogue
// are those of the FP32 kernel.  The split happens when a step is stored to
// LDS: A rows and the transposed B rows are K-contiguous halves with row stride
// 40 (16-byte fragment reads of 16 consecutive rows fall in distinct banks); a
// lane's fragment is the 8 values k = 8 (lane / 32) .. +7 of a 16-deep substep.
template <int BM, bool FVEC>
__global__ void __launch_bounds__(256)
hs_grad_split_kernel(const float* __restrict__ S, int64_t lds, const float* __restrict__ F,
                     const float* __restrict__ scl, const float* __restrict__ Cp, const float* __restrict__ Gp,
                     const float* __restrict__ rdiag, float alpha, float* __restrict__ gout, int64_t N, int kp,
                     int r) {
  constexpr int BK = 32, BN = BR, WM = 2, WN = 2, ST = BK + 8;
  constexpr int TM = BM / WM / 32, TN = BN / WN / 32;
  constexpr int AP = BM * BK / 4 / 256;    // A float4 per thread
  static_assert(BK * BN / 16 == 256, "one 4 x 4 block of B per thread");
  __shared__ __attribute__((aligned(16))) uint16_t AsH[BM * ST], AsM[BM * ST], AsL[BM * ST];
  __shared__ __attribute__((aligned(16))) uint16_t BsH[BN * ST], BsM[BN * ST], BsL[BN * ST];   // Bs[j][k] = B[k][j]
  __shared__ float sc[BR], rdl[BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  const int64_t i0 = (int64_t)blockIdx.x * BM;
  if (tid < BR) {
    sc[tid] = scl[tid];
    rdl[tid] = rdiag[tid];
  }
  const bool anykept = __syncthreads_or(tid < r && rdiag[tid] == 0.f);
  const int ks = (kp + BK - 1) / BK;
  f32x16 acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.f;
  f32x4 ra[AP];
  f32x4 rb[4];
  const int kq = tid >> 5, c4 = tid & 31, ca = 4 * (tid & 7);
  auto kept = [&](int l) { return l < r && rdl[l] == 0.f; };
  auto loadS = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int64_t gi = i0 + (tid >> 3) + 32 * p;
      const bool ok = gi < N && k0 + ca < kp;
      ra[p] = *(const f32x4*)(S + (ok ? gi * lds + k0 + ca : 0));
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = *(const f32x4*)(Cp + (int64_t)(k0 + 4 * kq + e) * BR + 4 * c4);
  };
  auto loadF = [&](int k0) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int64_t gi = i0 + (tid >> 3) + 32 * p;
      if (FVEC) {
        const bool ok = gi < N && k0 + ca < r;
        ra[p] = *(const f32x4*)(F + (ok ? gi * r + k0 + ca : 0));
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[p][e] = F[(gi < N && k0 + ca + e < r) ? gi * r + k0 + ca + e : 0];
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = *(const f32x4*)(Gp + (int64_t)(k0 + 4 * kq + e) * BR + 4 * c4);
  };
  auto put = [&](uint16_t* H, uint16_t* Mi, uint16_t* L, int off, const f32x4& v) {
    uint32_t h0, m0, l0, h1, m1, l1;
    split3_pair(v[0], v[1], h0, m0, l0);
    split3_pair(v[2], v[3], h1, m1, l1);
    *(uint2*)(H + off) = make_uint2(h0, h1);
    *(uint2*)(Mi + off) = make_uint2(m0, m1);
    *(uint2*)(L + off) = make_uint2(l0, l1);
  };
  auto storeA = [&](int k0, int lim, bool fs) {
#pragma unroll
    for (int p = 0; p < AP; ++p) {
      const int row = (tid >> 3) + 32 * p;
      const bool rok = i0 + row < N;
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float x = fs ? ra[p][e] * sc[k0 + ca + e] : ra[p][e];
        v[e] = (rok && k0 + ca + e < lim) ? x : 0.f;
      }
      put(AsH, AsM, AsL, row * ST + ca, v);
    }
  };
  auto storeS = [&](int k0) {
    storeA(k0, kp, false);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int l = 4 * c4 + d;
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = k0 + 4 * kq + e < kp ? rb[e][d] : 0.f;
      if (anykept && kept(l)) v = (f32x4){0.f, 0.f, 0.f, 0.f};
      put(BsH, BsM, BsL, l * ST + 4 * kq, v);
    }
  };
  auto storeF = [&](int k0) {
    storeA(k0, r, true);
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int l = 4 * c4 + d;
      f32x4 v;
      if (!anykept) {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = k0 + 4 * kq + e > l ? -rb[e][d] : 0.f;
      } else {
        const bool kl = kept(l);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = k0 + 4 * kq + e;
          v[e] = kl ? (i == l ? 1.f : 0.f) : ((kept(i) || i > l) ? -rb[e][d] : 0.f);
        }
      }
      put(BsH, BsM, BsL, l * ST + 4 * kq, v);
    }
  };
  const int half = lane >> 5, l32 = lane & 31;
  auto mma = [&]() {
#pragma unroll
    for (int q = 0; q < BK / 16; ++q) {
      const int kb = 16 * q + 8 * half;
      bf16x8 ah[TM], am[TM], al[TM], bh[TN], bm[TN], bl[TN];
#pragma unroll
      for (int x = 0; x < TM; ++x) {
        const int row = wm * (BM / WM) + 32 * x + l32;
        ah[x] = *(const bf16x8*)(AsH + row * ST + kb);
        am[x] = *(const bf16x8*)(AsM + row * ST + kb);
        al[x] = *(const bf16x8*)(AsL + row * ST + kb);
      }
#pragma unroll
      for (int y = 0; y < TN; ++y) {
        const int col = wn * (BN / WN) + 32 * y + l32;
        bh[y] = *(const bf16x8*)(BsH + col * ST + kb);
        bm[y] = *(const bf16x8*)(BsM + col * ST + kb);
        bl[y] = *(const bf16x8*)(BsL + col * ST + kb);
      }
      // small terms first; the accumulators alternate between dependent MFMAs
#define HS_MM(A, B)                                                                                       \
  _Pragma("unroll") for (int x = 0; x < TM; ++x) _Pragma("unroll") for (int y = 0; y < TN; ++y) acc[x][y] = \
      __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[x], B[y], acc[x][y], 0, 0, 0)
      HS_MM(al, bh);
      HS_MM(am, bm);
      HS_MM(ah, bl);
      HS_MM(am, bh);
      HS_MM(ah, bm);
      HS_MM(ah, bh);
#undef HS_MM
    }
  };
  __syncthreads();
  loadS(0);
  for (int t = 0; t < ks; ++t) {
    storeS(t * BK);
    __syncthreads();
    if (t + 1 < ks) loadS((t + 1) * BK);
    else loadF(0);
    __builtin_amdgcn_sched_barrier(0);
    mma();
    __syncthreads();
  }
  for (int t = 0; t < BR / BK; ++t) {
    storeF(t * BK);
    __syncthreads();
    if (t + 1 < BR / BK) loadF((t + 1) * BK);
    __builtin_amdgcn_sched_barrier(0);
    mma();
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) {
      const int j = wn * (BN / WN) + 32 * y + l32;
      const float aj = kept(j) ? 0.f : alpha;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int il = (e >> 2) * 8 + half * 4 + (e & 3);
        const int64_t gi = i0 + wm * (BM / WM) + 32 * x + il;
        if (gi < N && j < r) gout[gi * r + j] = acc[x][y][e] - aj;
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
// The sweep j = 1..r of one row as a forward substitution with a ReLU: with the
// gradient kernel's a_l = (S C)_l - sum_{i > l} f_i G_il - alpha, the rule
// f_l <- [(f_l G_ll + g_l - alpha) / (G_ll + beta)]_+ (Sec 4.1; the plain rule
// at alpha = beta = 0) reads n_l = [(a_l - sum_{i < l} n_i G_il) rho_l]_+ with
// rho_l = 1 / (G_ll + beta), over the new values n_i of the components before l,
// so the old f never enters the sweep and each component needs one register.
// The LDS copy of G holds only its strictly lower triangle (Gs[j][c] = G_cj for
// c > j, else 0), so from step j on the register of component j keeps its
// final a_j (every later update subtracts an exact zero) and n_j = [a_j rho_j]_+
// is formed again when the row is stored.  A component that keeps its value
// arrives as a_l = f_l scl_l and passes with rho = 1; its row and column of Gs
// are zero.
//
// One quad of lanes per row: lane q owns components 16 u + 4 q + c (u = 0..7,
// c = 0..3), so a row is read and written as 16-byte pieces, a lane's slice of a
// row of Gs is one 16-byte LDS load per 16 components, and after component j
// the components still to come are spread evenly over the quad (all four lanes
// skip the blocks u < floor(j / 16)).  At step j the owner lane ((j / 4) % 4)
// forms n_j and the quad receives it by DPP.  A quad sweeps R rows at once
// (rows t, t + 64, ... of a 64 R-row tile): they share every read of Gs, and
// the reads of step j + 1 are in flight during step j.  A workgroup sweeps the
// tiles blockIdx.x, blockIdx.x + gridDim.x, ...
template <int R>
__global__ void __launch_bounds__(256)
hs_sweep_kernel(const float* __restrict__ ain, const float* __restrict__ Gp, const float* __restrict__ rdiag,
                float* __restrict__ F, int64_t N, int r) {
  constexpr int RQ = BR / 4;   // slots per lane
  // rho first: its reads then take immediate LDS offsets
  __shared__ __attribute__((aligned(16))) float sm[BR + BR * BR];
  float* rho = sm;
  float* Gs = sm + BR;
  if (threadIdx.x < BR) {
    const float d = rdiag[threadIdx.x];
    rho[threadIdx.x] = d == 0.f ? 1.f : d;
  }
  for (int e = threadIdx.x; e < BR * BR; e += 256) {
    const int j = e / BR, c = e % BR;
    Gs[e] = (c > j && rdiag[j] != 0.f && rdiag[c] != 0.f) ? Gp[e] : 0.f;   // G is symmetric
  }
  __syncthreads();
  const int q = threadIdx.x & 3, ql = threadIdx.x >> 2;
  const bool vec = (r & 3) == 0;
  const int64_t ntiles = ceil_div(N, 64 * R);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // slot 4 u + c of a row holds component 16 u + 4 q + c
    float a[R][RQ];
    // unconditional loads (guarded ones would serialise on their waits): a row
    // past N reads row N - 1 and is never stored (rows are independent); a
    // component past r reads as zero
    if (vec) {
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const int64_t row = std::min<int64_t>(tile * 64 * R + 64 * p + ql, N - 1);
#pragma unroll
        for (int u = 0; u < RQ / 4; ++u) {
          const int c0 = 16 * u + 4 * q;
          const bool ok = c0 < r;
          const f32x4 v = *(const f32x4*)(ain + row * r + (ok ? c0 : 0));
#pragma unroll
          for (int c = 0; c < 4; ++c) a[p][4 * u + c] = ok ? v[c] : 0.f;
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const int64_t row = std::min<int64_t>(tile * 64 * R + 64 * p + ql, N - 1);
#pragma unroll
        for (int u = 0; u < RQ / 4; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int cc = 16 * u + 4 * q + c;
            const bool ok = cc < r;
            const float v = ain[row * r + (ok ? cc : 0)];
            a[p][4 * u + c] = ok ? v : 0.f;
          }
      }
    }
    f32x4 gb[2][RQ / 4];
    float rb[2];
    auto gload = [&](int j, int b) {
      rb[b] = rho[j];
#pragma unroll
      for (int u = j >> 4; u < RQ / 4; ++u) gb[b][u] = *(const f32x4*)(Gs + j * BR + 16 * u + 4 * q);
    };
    gload(0, 0);
    // fully unrolled: every register index below is a compile-time constant
#pragma clang loop unroll(full)
    for (int j = 0; j < BR; ++j) {
      const int b = j & 1, qj = (j >> 2) & 3, sj = 4 * (j >> 4) + (j & 3);
      if (j + 1 < BR) gload(j + 1, b ^ 1);
      float nb[R];
#pragma unroll
      for (int p = 0; p < R; ++p) {
        const float v = a[p][sj] * rb[b];
        nb[p] = quad_bcast_b(v > 0.f ? v : 0.f, qj);
      }
#pragma unroll
      for (int u = j >> 4; u < RQ / 4; ++u)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int p = 0; p < R; ++p) a[p][4 * u + c] -= nb[p] * gb[b][u][c];
      if ((j & 15) == 15) {   // block j / 16 is final: pin it here rather than let its last updates sink to the store
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int p = 0; p < R; ++p) asm volatile("" : "+v"(a[p][4 * (j >> 4) + c]));
      }
      __builtin_amdgcn_sched_barrier(0);   // keep each step's work together (register pressure)
    }
#pragma unroll
    for (int u = 0; u < RQ / 4; ++u) {
      const f32x4 rv = *(const f32x4*)(rho + 16 * u + 4 * q);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int p = 0; p < R; ++p) {
          const float v = a[p][4 * u + c] * rv[c];
          a[p][4 * u + c] = v > 0.f ? v : 0.f;
        }
    }
#pragma unroll
    for (int p = 0; p < R; ++p) {
      const int64_t row = tile * 64 * R + 64 * p + ql;
      if (row >= N) continue;
      float* fr = F + row * r;
#pragma unroll
      for (int u = 0; u < RQ / 4; ++u) {
        const int c0 = 16 * u + 4 * q;
        if (vec) {
          if (c0 < r) *(f32x4*)(fr + c0) = (f32x4){a[p][4 * u], a[p][4 * u + 1], a[p][4 * u + 2], a[p][4 * u + 3]};
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            if (c0 + c < r) fr[c0 + c] = a[p][4 * u + c];
        }
      }
    }
  }
}

// ------------------------------------------------------------------- qtf
// Workgroup partial Qb^T (F diag(sc)) (kp x r) and column sums of its squares,
// over the TRW-row tiles blockIdx.x, blockIdx.x + gridDim.x, ...  The tiles of
// Qb and F are staged in LDS; v_mfma_f32_32x32x2_f32 with A[c][i] = Qb[i][c] and
// B[i][j] = F[i][j], contraction over the tile's rows.  Wave w owns the 32-row
// blocks c of its quarter and all four 32-column blocks j.
template <int KPMAX, int TRW, bool FVEC>   // FVEC: rows of F are 16-byte aligned (r % 4 == 0)
__global__ void __launch_bounds__(256)
hs_qtf_kernel(const float* __restrict__ Qb, int64_t ldq, const float* __restrict__ F, const float* __restrict__ scale,
              int64_t N, int kp, int r, float* __restrict__ part) {
  constexpr int QROW = KPMAX + 4, FROW = BR + 4;
  constexpr int NTM = KPMAX / 32 / 4;       // 32-row blocks of the output per wave
  constexpr int QV = TRW * KPMAX / 4 / 256; // float4 of Qb per thread
  constexpr int FV = TRW * BR / 4 / 256;    // float4 of F per thread
  __shared__ __attribute__((aligned(16))) float Qs[TRW * QROW];
  __shared__ __attribute__((aligned(16))) float Fs[TRW * FROW];
  __shared__ __attribute__((aligned(16))) float sc[BR];
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
  f32x4 fv[FV];
  auto load = [&](int64_t tile) {
    const int64_t row0 = tile * TRW;
    if (tile >= ntiles) return;
    // unconditional loads from clamped addresses (guarded loads would serialise
    // on their waits); the tile is masked when it is stored
#pragma unroll
    for (int p = 0; p < QV; ++p) {
      const int e = tid + 256 * p, i = e / (KPMAX / 4), c4 = e % (KPMAX / 4);
      const bool ok = row0 + i < N && 4 * c4 < kp;
      qv[p] = *(const f32x4*)(Qb + (ok ? (row0 + i) * ldq + 4 * c4 : 0));
    }
#pragma unroll
    for (int p = 0; p < FV; ++p) {
      const int e = tid + 256 * p, i = e / (BR / 4), j = 4 * (e % (BR / 4));
      const bool ok = row0 + i < N;
      if (FVEC) {
        fv[p] = *(const f32x4*)(F + ((ok && j < r) ? (row0 + i) * r + j : 0));
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) fv[p][c] = F[(ok && j + c < r) ? (row0 + i) * r + j + c : 0];
      }
    }
  };
  __syncthreads();
  load(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * TRW;
#pragma unroll
    for (int p = 0; p < QV; ++p) {
      const int e = tid + 256 * p, i = e / (KPMAX / 4), c4 = e % (KPMAX / 4);
      *(f32x4*)(Qs + i * QROW + 4 * c4) = (row0 + i < N && 4 * c4 < kp) ? qv[p] : z4;
    }
#pragma unroll
    for (int p = 0; p < FV; ++p) {   // padding is zero
      const int e = tid + 256 * p, i = e / (BR / 4), j = 4 * (e % (BR / 4));
      const f32x4 sv = *(const f32x4*)(sc + j);
      f32x4 v;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float x = fv[p][c] * sv[c];
        v[c] = (row0 + i < N && j + c < r) ? x : 0.f;
      }
      *(f32x4*)(Fs + i * FROW + j) = v;
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
    // the operands of step k + 2 are read from LDS while the MFMAs of step k run
    float av[2][NTM], bv[2][4];
    auto frag = [&](int k, int b) {
      const int i = k + half;
#pragma unroll
      for (int x = 0; x < NTM; ++x) av[b][x] = Qs[i * QROW + 32 * (wave * NTM + x) + l32];
#pragma unroll
      for (int y = 0; y < 4; ++y) bv[b][y] = Fs[i * FROW + 32 * y + l32];
    };
    frag(0, 0);
#pragma clang loop unroll(full)
    for (int k = 0; k < TRW; k += 2) {
      const int b = (k >> 1) & 1;
      if (k + 2 < TRW) frag(k + 2, b ^ 1);
#pragma unroll
      for (int x = 0; x < NTM; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b][x], bv[b][y], acc[x][y], 0, 0, 0);
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

// hs_qtf_kernel on split-BF16 MFMA (hi hi + hi lo + lo hi, FP32 accumulation).
// The contraction runs over the tile's rows, so both operands are staged
// K-contiguous: QsT[c][i] = Qb[row0 + i][c] and FsT[j][i] = F[row0 + i][j] sc[j]
// as hi and lo halves (row stride TRW + 8: 16-byte fragment reads of 16
// consecutive rows fall in distinct banks).  Each thread loads 4 x 4 blocks
// (four rows, four columns; a wave reads whole row segments) and transposes
// them in registers when it stores the halves.  The column sums of the squares
// of F diag(sc) are formed in FP32 from the same registers; each thread keeps
// the sums of its four columns over its rows, added over the threads of a
// column in a fixed order at the end.
template <int KPMAX, int TRW, bool FVEC>
__global__ void __launch_bounds__(256)
hs_qtf_split_kernel(const float* __restrict__ Qb, int64_t ldq, const float* __restrict__ F,
                    const float* __restrict__ scale, int64_t N, int kp, int r, float* __restrict__ part) {
  constexpr int ST = TRW + 8;
  constexpr int NTM = KPMAX / 32 / 4;       // 32-row blocks of the output per wave
  constexpr int QCB = KPMAX / 4, FCB = BR / 4;
  constexpr int QB = TRW / 4 * QCB / 256;   // 4 x 4 blocks of Qb per thread
  constexpr int FB = TRW / 4 * FCB / 256;   // 4 x 4 blocks of F per thread
  static_assert(QB >= 1 && FB >= 1, "tile shape");
  __shared__ __attribute__((aligned(16))) uint16_t QH[KPMAX * ST], QL[KPMAX * ST];
  __shared__ __attribute__((aligned(16))) uint16_t FH[BR * ST], FL[BR * ST];
  __shared__ __attribute__((aligned(16))) float sc[BR];
  __shared__ float csum[256 / FCB][BR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < BR) sc[tid] = (scale && tid < r) ? scale[tid] : 1.f;
  f32x16 acc[NTM][4];
#pragma unroll
  for (int x = 0; x < NTM; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[x][y][e] = 0.f;
  float colsq[FB][4];
#pragma unroll
  for (int p = 0; p < FB; ++p)
#pragma unroll
    for (int d = 0; d < 4; ++d) colsq[p][d] = 0.f;
  const int64_t ntiles = ceil_div(N, TRW);
  const int half = lane >> 5, l32 = lane & 31;
  f32x4 qv[QB][4], fv[FB][4];
  // block b = tid + 256 p: rows 4 (b / ncb) .. +3, columns 4 (b % ncb) .. +3
  auto load = [&](int64_t tile) {
    if (tile >= ntiles) return;
    const int64_t row0 = tile * TRW;
#pragma unroll
    for (int p = 0; p < QB; ++p) {
      const int b = tid + 256 * p, i = 4 * (b / QCB), c = 4 * (b % QCB);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool ok = row0 + i + e < N && c < kp;
        qv[p][e] = *(const f32x4*)(Qb + (ok ? (row0 + i + e) * ldq + c : 0));
      }
    }
#pragma unroll
    for (int p = 0; p < FB; ++p) {
      const int b = tid + 256 * p, i = 4 * (b / FCB), j = 4 * (b % FCB);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool ok = row0 + i + e < N;
        if (FVEC) {
          fv[p][e] = *(const f32x4*)(F + ((ok && j < r) ? (row0 + i + e) * r + j : 0));
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) fv[p][e][c] = F[(ok && j + c < r) ? (row0 + i + e) * r + j + c : 0];
        }
      }
    }
  };
  __syncthreads();
  load(blockIdx.x);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * TRW;
#pragma unroll
    for (int p = 0; p < QB; ++p) {
      const int b = tid + 256 * p, i = 4 * (b / QCB), c = 4 * (b % QCB);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (row0 + i + e < N && c + d < kp) ? qv[p][e][d] : 0.f;
        uint32_t h0, l0, h1, l1;
        split_pair(v[0], v[1], h0, l0);
        split_pair(v[2], v[3], h1, l1);
        *(uint2*)(QH + (c + d) * ST + i) = make_uint2(h0, h1);
        *(uint2*)(QL + (c + d) * ST + i) = make_uint2(l0, l1);
      }
    }
#pragma unroll
    for (int p = 0; p < FB; ++p) {
      const int b = tid + 256 * p, i = 4 * (b / FCB), j = 4 * (b % FCB);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x = fv[p][e][d] * sc[j + d];
          v[e] = (row0 + i + e < N && j + d < r) ? x : 0.f;
          colsq[p][d] += v[e] * v[e];
        }
        uint32_t h0, l0, h1, l1;
        split_pair(v[0], v[1], h0, l0);
        split_pair(v[2], v[3], h1, l1);
        *(uint2*)(FH + (j + d) * ST + i) = make_uint2(h0, h1);
        *(uint2*)(FL + (j + d) * ST + i) = make_uint2(l0, l1);
      }
    }
    __syncthreads();
    load(tile + gridDim.x);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < TRW / 16; ++q) {
      const int kb = 16 * q + 8 * half;
      bf16x8 ah[NTM], al[NTM], bh[4], bl[4];
#pragma unroll
      for (int x = 0; x < NTM; ++x) {
        const int c = 32 * (wave * NTM + x) + l32;
        ah[x] = *(const bf16x8*)(QH + c * ST + kb);
        al[x] = *(const bf16x8*)(QL + c * ST + kb);
      }
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int j = 32 * y + l32;
        bh[y] = *(const bf16x8*)(FH + j * ST + kb);
        bl[y] = *(const bf16x8*)(FL + j * ST + kb);
      }
#pragma unroll
      for (int x = 0; x < NTM; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[x], bh[y], acc[x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < NTM; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bl[y], acc[x][y], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < NTM; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[x], bh[y], acc[x][y], 0, 0, 0);
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
  // column j = 4 (tid % FCB) + d: threads tid % FCB == j / 4, rows blocks tid / FCB (+ 256 / FCB p)
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    float t = 0.f;
#pragma unroll
    for (int p = 0; p < FB; ++p) t += colsq[p][d];
    csum[tid / FCB][4 * (tid % FCB) + d] = t;
  }
  __syncthreads();
  if (tid < r) {
    float t = 0.f;
    for (int g = 0; g < 256 / FCB; ++g) t += csum[g][tid];
    P[kp * r + tid] = t;
  }
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
    const bool fv = (a.r & 3) == 0;
    const dim3 g128((unsigned)ceil_div(a.N, 128)), g64((unsigned)ceil_div(a.N, 64));
#define HS_GRAD(K, BM, FV, G)                                                                                      \
  hipLaunchKernelGGL((K<BM, FV>), G, dim3(256), 0, st, a.S, a.lds, a.F, scl, Cp, Gp, rdiag, a.alpha, a.gbuf, a.N, \
                     a.kp, a.r)
    const bool tall = a.N >= 128 * 512;
    if (a.split) {
      if (tall) {
        if (fv) HS_GRAD(hs_grad_split_kernel, 128, true, g128);
        else HS_GRAD(hs_grad_split_kernel, 128, false, g128);
      } else {
        if (fv) HS_GRAD(hs_grad_split_kernel, 64, true, g64);
        else HS_GRAD(hs_grad_split_kernel, 64, false, g64);
      }
    } else {
      if (tall) {
        if (fv) HS_GRAD(hs_grad_kernel, 128, true, g128);
        else HS_GRAD(hs_grad_kernel, 128, false, g128);
      } else {
        if (fv) HS_GRAD(hs_grad_kernel, 64, true, g64);
        else HS_GRAD(hs_grad_kernel, 64, false, g64);
      }
    }
#undef HS_GRAD
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // 64 R-row tiles; at most two workgroups per CU are resident (LDS), so at
    // most 512 loop over the tiles.  R = 4 rows per quad for tall sides, fewer
    // where that would leave CUs idle.
    const int R = a.N >= 131072 ? 4 : (a.N >= 32768 ? 2 : 1);
    const unsigned sblk = (unsigned)std::min<int64_t>(ceil_div(a.N, 64 * R), 512);
    if (R == 4)
      hipLaunchKernelGGL(hs_sweep_kernel<4>, dim3(sblk), dim3(256), 0, st, a.gbuf, Gp, rdiag, a.F, a.N, a.r);
    else if (R == 2)
      hipLaunchKernelGGL(hs_sweep_kernel<2>, dim3(sblk), dim3(256), 0, st, a.gbuf, Gp, rdiag, a.F, a.N, a.r);
    else
      hipLaunchKernelGGL(hs_sweep_kernel<1>, dim3(sblk), dim3(256), 0, st, a.gbuf, Gp, rdiag, a.F, a.N, a.r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // after a sweep F is final; without one its pending column scales apply on load
  const float* qscale = do_sweep ? nullptr : a.scale;
  const bool fv = (a.r & 3) == 0;
  const dim3 qg((unsigned)nblk);
#define HS_QTF(K, KP, TR, FV) \
  hipLaunchKernelGGL((K<KP, TR, FV>), qg, dim3(256), 0, st, a.Qb, a.ldq, a.F, qscale, a.N, a.kp, a.r, a.part)
  if (a.split) {
    if (a.kp <= 128) {
      if (fv) HS_QTF(hs_qtf_split_kernel, 128, 64, true);
      else HS_QTF(hs_qtf_split_kernel, 128, 64, false);
    } else {
      if (fv) HS_QTF(hs_qtf_split_kernel, 256, 32, true);
      else HS_QTF(hs_qtf_split_kernel, 256, 32, false);
    }
  } else {
    if (a.kp <= 128) {
      if (fv) HS_QTF(hs_qtf_kernel, 128, 64, true);
      else HS_QTF(hs_qtf_kernel, 128, 64, false);
    } else {
      if (fv) HS_QTF(hs_qtf_kernel, 256, 32, true);
      else HS_QTF(hs_qtf_kernel, 256, 32, false);
    }
  }
#undef HS_QTF
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_partials_f32(a.part, nblk, (int64_t)a.kp * a.r + a.r, a.acc_out, st);
}
