// Host runtime and C ABI of the compressed-NMF library (declared in nmfrp.h).
// A context owns no device memory: every buffer is carved from the caller's
// workspace.  All kernels run on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nmfrp.h"
#include "common.h"

namespace {

thread_local std::string g_err;

struct Plan {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  }
};

// Workspace layout; offsets relative to the workspace base.
struct Layout {
  int64_t KP;  // k' padded to a multiple of 4 (padding columns stay zero)
  size_t omL, omR, QL, TM, Xc, QR, TN, Xh, W, Ht;
  size_t gemm_part, gram_part, G, R, qr_status;     // chain 0 (left range finder)
  size_t gemm_part2, gram_part2, G2, R2;             // chain 1 (right range finder); status at qr_status + 8
  size_t hs_part, acc_w, acc_h, counters, Hc, GH, Wh, GW, scale_w;
  size_t hs_aux;                      // wide-factor half-steps: C, G, 1/G_jj, scales
  size_t res_part, res_out, flags, proxy_part, proxy_out, xsq_part;
  size_t rsplit;                      // split-BF16 residual: BF16 splits of W diag(sw) and Ht
  size_t alignM, whref;               // warm start: Q_train^T Q_L (k' x k'), Q_L^T W_ref (k' x r)
  int64_t ldq, ldqt;                 // low-precision copies of X: m x ldq and n x ldqt
  size_t Xq, XqT, Ex, Bt, Eb, Bt2, Eb2;
  size_t St, St2;                     // split-BF16 thin operands (hi, then lo) of the sketch products
  size_t total;
  size_t gemm_part_bytes, gram_splits_max;
};

bool valid_params(const nmf_params* p, std::string* why) {
  if (!p) { *why = "null params"; return false; }
  if (p->m <= 0 || p->n <= 0 || p->r <= 0) { *why = "m, n, r must be positive"; return false; }
  if (!(p->r < p->k_sketch)) { *why = "need r < k' (Sec 3.1)"; return false; }
  if (p->k_sketch > p->m || p->k_sketch > p->n) { *why = "need k' <= min(m, n)"; return false; }
  if (p->k_sketch > 256) { *why = "k' > 256 is not supported by this build"; return false; }
  if (p->r > 128) { *why = "r > 128 is not supported by this build"; return false; }
  if (p->q < 0) { *why = "q must be >= 0"; return false; }
  if (p->prec < NMF_FP32 || p->prec > NMF_FP8_E4M3) { *why = "prec must be FP32, BF16 or FP8_E4M3"; return false; }
  if (p->refine_fp32 < 0 || p->refine_fp32 > 2) { *why = "refine_fp32 must be 0, 1 or 2"; return false; }
  if (p->normalize < 0 || p->normalize > 2) { *why = "normalize must be 0, 1 or 2"; return false; }
  if (p->n % 4) { *why = "n must be a multiple of 4"; return false; }
  if (p->alpha < 0 || p->beta < 0) { *why = "alpha, beta must be >= 0"; return false; }
  if (p->lowp_sketches < 0 || p->lowp_sketches > 2 || (p->lowp_sketches == 1 && p->prec == NMF_FP32)) {
    *why = "lowp_sketches must be 0, 1 (with a low-precision prec) or 2";
    return false;
  }
  if (p->update_prec < 0 || p->update_prec > 1) { *why = "update_prec must be 0 or 1"; return false; }
  if (p->update_prec == 1 && !halfstep_big(p->k_sketch, p->r)) {
    *why = "update_prec 1 (split-BF16 update products) needs the wide-factor half-steps (r > 64 or k' > 128)";
    return false;
  }
  return true;
}

Layout make_layout(const nmf_params* p) {
  Layout L;
  Plan pl;
  const int64_t m = p->m, n = p->n, k = p->k_sketch, r = p->r;
  L.KP = round_up(k, 4);
  const size_t f = sizeof(float), d = sizeof(double);
  L.omL = pl.take(n * L.KP * f);
  L.omR = pl.take(m * L.KP * f);
  L.QL = pl.take(m * L.KP * f);
  L.TM = pl.take(m * L.KP * f);
  L.Xc = pl.take(m * L.KP * f);
  L.QR = pl.take(n * L.KP * f);
  L.TN = pl.take(n * L.KP * f);
  L.Xh = pl.take(n * L.KP * f);
  L.W = pl.take(m * r * f);
  L.Ht = pl.take(n * r * f);
  const int s1 = gemm_f32_pick_splits(m, k, n, 0), s2 = gemm_f32_pick_splits(n, k, m, 1);
  size_t gp = gemm_f32_part_floats(m, k, s1);
  size_t gp2 = gemm_f32_part_floats(n, k, s2);
  L.ldq = round_up(n, 128);
  L.ldqt = round_up(m, 128);
  if (p->prec != NMF_FP32) {
    const int bm = 128;
    const int l1 = gemm_lp_pick_splits(m, k, L.ldq, bm), l2 = gemm_lp_pick_splits(n, k, L.ldqt, bm);
    const size_t q1 = l1 > 1 ? (size_t)l1 * m * k : 0, q2 = l2 > 1 ? (size_t)l2 * n * k : 0;
    if (q1 > gp) gp = q1;
    if (q2 > gp2) gp2 = q2;
  }
  const bool split_any = p->lowp_sketches == 2 || (p->prec != NMF_FP32 && p->refine_fp32 == 2);
  if (split_any) {
    const int l1 = gemm_split_pick_splits(m, k, n), l2 = gemm_split_pick_splits(n, k, m);
    const size_t q1 = l1 > 1 ? (size_t)l1 * m * k : 0, q2 = l2 > 1 ? (size_t)l2 * n * k : 0;
    if (q1 > gp) gp = q1;
    if (q2 > gp2) gp2 = q2;
  }
  L.gemm_part_bytes = (gp > gp2 ? gp : gp2) * f;
  L.gemm_part = pl.take(L.gemm_part_bytes);
  L.gemm_part2 = pl.take(L.gemm_part_bytes);
  const int gs1 = gram_pick_splits(m, k), gs2 = gram_pick_splits(n, k);
  L.gram_splits_max = gs1 > gs2 ? gs1 : gs2;
  L.gram_part = pl.take(L.gram_splits_max * k * k * d);
  L.gram_part2 = pl.take(L.gram_splits_max * k * k * d);
  L.G = pl.take(k * k * d);
  L.R = pl.take(k * k * d);
  L.qr_status = pl.take(16 * sizeof(int));
  L.G2 = pl.take(k * k * d);
  L.R2 = pl.take(k * k * d);
  size_t h1 = halfstep_part_floats(m, (int)L.KP, (int)r), h2 = halfstep_part_floats(n, (int)L.KP, (int)r);
  L.hs_part = pl.take((h1 > h2 ? h1 : h2) * f);
  L.acc_w = pl.take((L.KP * r + r) * d);
  L.acc_h = pl.take((L.KP * r + r) * d);
  L.counters = pl.take(8 * sizeof(unsigned));
  L.Hc = pl.take(L.KP * r * f);
  L.GH = pl.take(r * r * f);
  L.Wh = pl.take(L.KP * r * f);
  L.GW = pl.take(r * r * f);
  L.scale_w = pl.take(r * f);
  L.hs_aux = pl.take(halfstep_big_aux_floats() * f);
  L.res_part = pl.take(2 * (size_t)residual_blocks(m, n) * d);
  L.res_out = pl.take(2 * d);
  L.rsplit = pl.take(residual_split_halves(m, n, r) * sizeof(uint16_t));
  L.flags = pl.take(8 * sizeof(int));
  L.alignM = pl.take(L.KP * L.KP * f);
  L.whref = pl.take(L.KP * r * f);
  L.proxy_part = pl.take(2 * 256 * d);
  L.proxy_out = pl.take(3 * d);            // proxy sums, then ||X||^2 from compression
  {
    const int64_t qp = quant_sq_parts(m, n, round_up(n, 128), round_up(m, 128));
    const int64_t gp3 = gemm_f32_sq_parts(m, k, n, 64);
    const int64_t gp4 = gemm_split_sq_parts(m, k, gemm_split_pick_splits(m, k, n));
    L.xsq_part = pl.take((size_t)std::max(qp, std::max(gp3, gp4)) * d);
  }
  L.Xq = L.XqT = L.Ex = L.Bt = L.Eb = L.Bt2 = L.Eb2 = 0;
  if (p->prec != NMF_FP32) {
    const size_t es = p->prec == NMF_BF16 ? 2 : 1;
    L.Xq = pl.take((size_t)m * L.ldq * es);
    // BF16: X^T products read Xq through the transposing kernel (k' <= 128); FP8,
    // and BF16 with wider sketches, keep a copy of X^T too
    L.XqT = (p->prec == NMF_BF16 && k <= 128) ? 0 : pl.take((size_t)n * L.ldqt * es);
    L.Ex = pl.take((size_t)ceil_div(m, 128) * ceil_div(n, 128) * sizeof(int));
    L.Bt = pl.take((size_t)k * (L.ldq > L.ldqt ? L.ldq : L.ldqt) * es);
    L.Eb = pl.take((size_t)ceil_div(L.ldq > L.ldqt ? L.ldq : L.ldqt, 128) * sizeof(int));
    L.Bt2 = pl.take((size_t)k * (L.ldq > L.ldqt ? L.ldq : L.ldqt) * es);
    L.Eb2 = pl.take((size_t)ceil_div(L.ldq > L.ldqt ? L.ldq : L.ldqt, 128) * sizeof(int));
  }
  L.St = L.St2 = 0;
  if (split_any) {   // hi and lo halves, k x max(ldq, ldqt) BF16 each, per chain
    L.St = pl.take((size_t)2 * k * std::max(L.ldq, L.ldqt) * 2);
    L.St2 = pl.take((size_t)2 * k * std::max(L.ldq, L.ldqt) * 2);
  }
  L.total = pl.off;
  return L;
}

}  // namespace

void nmf_set_thread_error(const char* msg) { g_err = msg; }

struct nmf_ctx {
  nmf_params p;
  Layout L;
  char* ws;
  hipStream_t st;
  bool compressed = false, initialized = false, stepped = false;
  bool xsq_valid = false;  // ||X||^2 of the compressed X is in proxy_out[2]
  std::string err;
  hipEvent_t ev[6];
  bool have_ev = false;
  hipStream_t st2 = nullptr;          // second stream of nmf_compress (right range finder)
  hipEvent_t fork = nullptr, join = nullptr;
  // third stream: the warm start's alignment products, which need only Q_L, run
  // on it from ql_ready (recorded by nmf_compress once Q_L is final) under the
  // sketch products; aligned marks their end
  hipStream_t st3 = nullptr;
  hipEvent_t ql_ready = nullptr, aligned = nullptr;
  bool ql_event = false;              // ql_ready belongs to the current Q_L
  float ms_compress = 0, ms_step = 0, ms_residual = 0;
  bool t_compress = false, t_step = false, t_residual = false;
  double* hout = nullptr;             // pinned host results (gather_host), device view hout_dev
  double* hout_dev = nullptr;
  template <class T> T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Pinned, device-mapped, coherent host buffers for the results the host reads
// after a synchronisation (a kernel writes them there, so no copy command runs).
// They are taken from a process-wide pool and returned to it, never freed: a
// context's buffer is reused by the next context.
constexpr size_t HOUT_DOUBLES = 16;
std::mutex g_hout_mu;
std::vector<double*> g_hout_free;

double* take_host_out() {
  std::lock_guard<std::mutex> lk(g_hout_mu);
  if (!g_hout_free.empty()) {
    double* p = g_hout_free.back();
    g_hout_free.pop_back();
    return p;
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, HOUT_DOUBLES * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return nullptr;
  return (double*)p;
}

void give_host_out(double* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_hout_mu);
  g_hout_free.push_back(p);
}

}  // namespace

namespace {

nmf_status fail(nmf_ctx* c, nmf_status s, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return s;
}

#define HIPCHK(c, expr)                                                          \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail((c), NMF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Orthonormalise Y (rows x k, ld) in place.  final: CholeskyQR2 with the
// shifted third pass on breakdown (the bases the sketches are built on).  Not
// final (an intermediate basis of the subspace iteration, which only has to
// span the same space and be well conditioned): one CholeskyQR pass, shifted
// on breakdown; its orthogonality error is about kappa(Y)^2 u_fp64.
//
// bt (intermediate bases only): the basis is written only as the transposed
// BF16 operand of the next product (k x ldbt), not back into Y.
hipError_t orth(float* Y, int64_t ld, int64_t rows, int k, double* gram_part, double* G,
                double* R, int* status, hipStream_t st, bool final = true, uint16_t* bt = nullptr,
                int64_t ldbt = 0) {
  hipError_t e;
  const int splits = gram_pick_splits(rows, k);
  const int passes = final ? 3 : 1;       // the first pass resets the shift flags
  for (int attempt = 0; attempt < passes; ++attempt) {
    if ((e = launch_gram_f64(Y, ld, rows, k, gram_part, splits, G, attempt == 2 ? status : nullptr, st)))
      return e;
    if ((e = launch_cholesky(G, k, rows, R, status, attempt, st))) return e;
    if ((e = launch_apply_rinv(Y, ld, rows, k, R, status, attempt, st, final ? nullptr : bt, ldbt))) return e;
  }
  return hipSuccess;
}

// Scratch and stream of one range-finder chain (the two chains of nmf_compress
// run concurrently, each with its own buffers).
struct Chain {
  hipStream_t st;
  float* gemm_part;
  double *gp, *G, *R;
  int* qs;
  void* Bt;
  int* Eb;
};

Chain chain(nmf_ctx* c, int which) {
  Layout& L = c->L;
  Chain ch;
  ch.st = which ? c->st2 : c->st;
  ch.gemm_part = c->at<float>(which ? L.gemm_part2 : L.gemm_part);
  ch.gp = c->at<double>(which ? L.gram_part2 : L.gram_part);
  ch.G = c->at<double>(which ? L.G2 : L.G);
  ch.R = c->at<double>(which ? L.R2 : L.R);
  ch.qs = c->at<int>(L.qr_status) + (which ? 8 : 0);
  ch.Bt = (L.Bt == 0) ? nullptr : (void*)c->at<char>(which ? L.Bt2 : L.Bt);
  ch.Eb = (L.Eb == 0) ? nullptr : c->at<int>(which ? L.Eb2 : L.Eb);
  return ch;
}

hipError_t gemm(nmf_ctx* c, const Chain& ch, const float* A, int64_t lda, int at, const float* B, float* C,
                int64_t M, int64_t K) {
  const int64_t N = c->p.k_sketch;
  const int s = gemm_f32_pick_splits(M, N, K, at);
  return launch_gemm_f32(A, lda, at, B, c->L.KP, C, c->L.KP, M, N, K, s, ch.gemm_part, ch.st);
}

// Low-precision range-finder product: side 0 -> X B (B is n x k'), side 1 ->
// X^T B (B is m x k'); the thin operand is rounded (and transposed) first.
hipError_t gemm_lowp(nmf_ctx* c, const Chain& ch, int side, const float* B, float* C, bool prepared = false) {
  Layout& L = c->L;
  const int64_t m = c->p.m, n = c->p.n, k = c->p.k_sketch;
  const int64_t M = side ? n : m, K = side ? m : n, Kpad = side ? L.ldqt : L.ldq;
  const int s = gemm_lp_pick_splits(M, k, Kpad, 128);
  float* part = ch.gemm_part;
  hipError_t e;
  if (c->p.prec == NMF_BF16) {
    uint16_t* Bt = (uint16_t*)ch.Bt;
    // prepared: the orthonormalisation that produced B already wrote its BF16 copy
    if (!prepared && (e = launch_prep_b_bf16(B, L.KP, K, k, Bt, Kpad, ch.st))) return e;
    // X B: Xq rows are K-contiguous; X^T B: the same Xq, transposed while staged,
    // or (k' > 128) the copy of X^T
    if (side && L.XqT)
      return launch_gemm_bf16_nt(c->at<uint16_t>(L.XqT), L.ldqt, Bt, Kpad, C, L.KP, M, k, Kpad, s, part, ch.st);
    return launch_gemm_bf16_nt(c->at<uint16_t>(L.Xq), L.ldq, Bt, Kpad, C, L.KP, M, k, Kpad, s, part, ch.st, true,
                               side, K);
  }
  uint8_t* Bt = (uint8_t*)ch.Bt;
  int* Eb = ch.Eb;
  if ((e = launch_prep_b_fp8(B, L.KP, K, k, Eb, Bt, Kpad, ch.st))) return e;
  const uint8_t* A = side ? c->at<uint8_t>(L.XqT) : c->at<uint8_t>(L.Xq);
  const int64_t tn = ceil_div(n, 128);
  // X tile (a, b) exponent at Ex[a * tn + b]; A = X: (ti, tk) = (a, b); A = X^T: (ti, tk) = (b, a)
  return launch_gemm_fp8_nt(A, Kpad, c->at<int>(L.Ex), side ? 1 : tn, side ? tn : 1, Bt, Kpad, Eb, C,
                            L.KP, M, k, Kpad, s, part, ch.st);
}

// W half-step: sweep W against (Xc, Hc, G_H) derived from the summed H-side
// partials; leaves Q_L^T W and the column sums of W^2 in acc_w.
hipError_t halfstep_w(nmf_ctx* c) {
  Layout& L = c->L;
  HalfStepArgs a;
  a.S = c->at<float>(L.Xc); a.lds = L.KP;
  a.acc_in = c->at<double>(L.acc_h); a.norm_in = 0; a.normalize = c->p.normalize;
  a.F = c->at<float>(L.W); a.scale = c->at<float>(L.scale_w); a.scale_pub = nullptr;
  a.C_pub = c->at<float>(L.Hc); a.G_pub = c->at<float>(L.GH);
  a.Qb = c->at<float>(L.QL); a.ldq = L.KP;
  a.N = c->p.m; a.kp = (int)L.KP; a.r = c->p.r;
  a.part = c->at<float>(L.hs_part); a.acc_out = c->at<double>(L.acc_w);
  a.alpha = 0.f; a.beta = 0.f;
  a.gbuf = c->at<float>(L.TM); a.aux = c->at<float>(L.hs_aux); a.split = c->p.update_prec;   // the m-side temporary is free while stepping
  return launch_halfstep(a, 1, c->st);
}

// H half-step: normalise W's columns (compensated in Ht), sweep Ht against
// (Xh, Wh, G_W); leaves Q_R^T Ht in acc_h.  do_sweep = 0 only forms acc_h.
hipError_t halfstep_h(nmf_ctx* c, int do_sweep) {
  Layout& L = c->L;
  HalfStepArgs a;
  a.S = c->at<float>(L.Xh); a.lds = L.KP;
  a.acc_in = c->at<double>(L.acc_w); a.norm_in = do_sweep; a.normalize = c->p.normalize;
  a.F = c->at<float>(L.Ht); a.scale = nullptr;
  a.scale_pub = do_sweep ? c->at<float>(L.scale_w) : nullptr;
  a.C_pub = do_sweep ? c->at<float>(L.Wh) : nullptr; a.G_pub = do_sweep ? c->at<float>(L.GW) : nullptr;
  a.Qb = c->at<float>(L.QR); a.ldq = L.KP;
  a.N = c->p.n; a.kp = (int)L.KP; a.r = c->p.r;
  a.part = c->at<float>(L.hs_part); a.acc_out = c->at<double>(L.acc_h);
  a.alpha = c->p.alpha; a.beta = c->p.beta;
  a.gbuf = c->at<float>(L.TN); a.aux = c->at<float>(L.hs_aux); a.split = c->p.update_prec;   // the n-side temporary is free while stepping
  return launch_halfstep(a, do_sweep, c->st);
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

extern "C" {

size_t nmf_workspace_bytes(const nmf_params* p) {
  std::string why;
  if (!valid_params(p, &why)) { g_err = why; return 0; }
  return make_layout(p).total;
}

nmf_status nmf_create(const nmf_params* p, void* workspace, size_t ws_bytes, void* hip_stream,
                      nmf_ctx** out) {
  std::string why;
  if (!out) return fail(nullptr, NMF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!valid_params(p, &why)) return fail(nullptr, NMF_EINVAL, why);
  Layout L = make_layout(p);
  if (!workspace || ((uintptr_t)workspace & 255)) return fail(nullptr, NMF_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(nullptr, NMF_ENOMEM, "workspace too small");
  nmf_ctx* c = new nmf_ctx();
  c->p = *p;
  c->L = L;
  c->ws = (char*)workspace;
  c->st = (hipStream_t)hip_stream;
  hipError_t e = launch_fill_f32((float*)workspace, (int64_t)(L.total / 4), 0.f, c->st);
  if (e != hipSuccess) { delete c; return fail(nullptr, NMF_EHIP, hipGetErrorString(e)); }
  for (int i = 0; i < 6; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) { delete c; return fail(nullptr, NMF_EHIP, "event create"); }
  c->have_ev = true;
  // second stream of the range finder (default priority) and its fork/join events
  if (hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->st3, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ql_ready, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->aligned, hipEventDisableTiming) != hipSuccess) {
    nmf_destroy(c);
    return fail(nullptr, NMF_EHIP, "stream/event create");
  }
  c->hout = take_host_out();
  if (!c->hout || hipHostGetDevicePointer((void**)&c->hout_dev, c->hout, 0) != hipSuccess) {
    nmf_destroy(c);
    return fail(nullptr, NMF_EHIP, "pinned host buffer");
  }
  *out = c;
  return NMF_OK;
}

void nmf_destroy(nmf_ctx* c) {
  if (!c) return;
  if (c->hout) {   // no gather into the buffer may still be in flight when it is reused
    (void)hipStreamSynchronize(c->st);
    give_host_out(c->hout);
  }
  if (c->have_ev)
    for (int i = 0; i < 6; ++i) (void)hipEventDestroy(c->ev[i]);
  if (c->st2) {
    (void)hipStreamSynchronize(c->st2);
    (void)hipStreamDestroy(c->st2);
  }
  if (c->st3) {
    (void)hipStreamSynchronize(c->st3);
    (void)hipStreamDestroy(c->st3);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->join) (void)hipEventDestroy(c->join);
  if (c->ql_ready) (void)hipEventDestroy(c->ql_ready);
  if (c->aligned) (void)hipEventDestroy(c->aligned);
  delete c;
}

const char* nmf_last_error(const nmf_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

nmf_status nmf_validate(nmf_ctx* c, const float* X, int64_t ldx) {
  if (!c || !X || ldx < c->p.n) return fail(c, NMF_EINVAL, "bad arguments");
  int* flags = c->at<int>(c->L.flags);
  HIPCHK(c, launch_fill_i32(flags, 2, 0, c->st));
  HIPCHK(c, launch_check_nonneg(X, ldx, c->p.m, c->p.n, flags, c->st));
  int h[2];
  HIPCHK(c, hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (h[1]) return fail(c, NMF_ENONFINITE, "X has non-finite entries");
  if (h[0]) return fail(c, NMF_EINVAL, "X has negative entries (NMF needs X >= 0)");
  return NMF_OK;
}

nmf_status nmf_compress(nmf_ctx* c, const float* X, int64_t ldx, const float* omega_L,
                        const float* omega_R) {
  if (!c || !X) return fail(c, NMF_EINVAL, "null argument");
  if (ldx < c->p.n || ldx % 4 || !aligned16(X)) return fail(c, NMF_EINVAL, "X needs ldx >= n, ldx % 4 == 0, 16-byte alignment");
  Layout& L = c->L;
  const int64_t m = c->p.m, n = c->p.n;
  const int k = c->p.k_sketch, q = c->p.q;
  hipStream_t st = c->st;
  float *omL = c->at<float>(L.omL), *omR = c->at<float>(L.omR);
  float *QL = c->at<float>(L.QL), *TM = c->at<float>(L.TM), *Xc = c->at<float>(L.Xc);
  float *QR = c->at<float>(L.QR), *TN = c->at<float>(L.TN), *Xh = c->at<float>(L.Xh);
  HIPCHK(c, hipEventRecord(c->ev[0], st));
  HIPCHK(c, launch_fill_i32(c->at<int>(L.qr_status), 16, 0, st));
  // test matrices (Sec 3)
  if (omega_L) HIPCHK(c, launch_copy2d(omL, L.KP, omega_L, k, n, k, st));
  else HIPCHK(c, launch_philox_normal(omL, n, k, L.KP, 3u, c->p.seed, st));
  if (omega_R) HIPCHK(c, launch_copy2d(omR, L.KP, omega_R, k, m, k, st));
  else HIPCHK(c, launch_philox_normal(omR, m, k, L.KP, 4u, c->p.seed, st));
  // range-finder products: FP32 on X, or on its low-precision copy (extension)
  const bool lp = c->p.prec != NMF_FP32;
  const bool lps = lp && c->p.lowp_sketches == 1;
  const bool split = c->p.lowp_sketches == 2;
  // ||X||^2 in FP64 from the quantiser's pass over X when there is one and the
  // sketch products are low precision or split; else from the X Q_R pass
  const bool xsq_quant = lp && (lps || split);
  if (lp) {
    double* sqp = xsq_quant ? c->at<double>(L.xsq_part) : nullptr;
    double* sqo = xsq_quant ? c->at<double>(L.proxy_out) + 2 : nullptr;
    if (c->p.prec == NMF_BF16 && L.XqT)
      HIPCHK(c, launch_quant_bf16(X, ldx, m, n, c->at<uint16_t>(L.Xq), L.ldq, c->at<uint16_t>(L.XqT), L.ldqt, st,
                                  sqp, sqo));
    else if (c->p.prec == NMF_BF16)
      HIPCHK(c, launch_quant_bf16_rows(X, ldx, m, n, c->at<uint16_t>(L.Xq), L.ldq, st, sqp, sqo));
    else
      HIPCHK(c, launch_quant_fp8(X, ldx, m, n, c->at<int>(L.Ex), c->at<uint8_t>(L.Xq), L.ldq,
                                 c->at<uint8_t>(L.XqT), L.ldqt, st, sqp, sqo));
  }
  const Chain cl = chain(c, 0), cr = chain(c, 1);
  // BF16 range finder: an intermediate basis whose next consumer is a BF16
  // product is written only as that product's transposed BF16 operand
  const bool fuse = c->p.prec == NMF_BF16 && k <= 64;
  auto XB = [&](const Chain& ch, const float* B, float* C, bool prep) -> hipError_t {   // X B  (m x k')
    return lp ? gemm_lowp(c, ch, 0, B, C, prep) : gemm(c, ch, X, ldx, 0, B, C, m, n);
  };
  auto XtB = [&](const Chain& ch, const float* B, float* C, bool prep) -> hipError_t {  // X^T B (n x k')
    return lp ? gemm_lowp(c, ch, 1, B, C, prep) : gemm(c, ch, X, ldx, 1, B, C, n, m);
  };
  // next_lp: the basis feeds a low-precision product next
  auto ORTH = [&](const Chain& ch, float* Y, int64_t rows, bool final, bool next_lp) -> hipError_t {
    if (!final && fuse && next_lp)
      return orth(Y, L.KP, rows, k, ch.gp, ch.G, ch.R, ch.qs, ch.st, false, (uint16_t*)ch.Bt,
                  rows == m ? L.ldqt : L.ldq);
    return orth(Y, L.KP, rows, k, ch.gp, ch.G, ch.R, ch.qs, ch.st, final);
  };
  const bool refine = lp && c->p.refine_fp32;
  // Each range finder is a list of stages (a product, then the orthonormalisation
  // of its result); only the last orthonormalisation of each side is a full
  // CholeskyQR2.  Left: Q_L = orth(X Omega_L); q x { Z = orth(X^T Q_L); Q_L = orth(X Z) }.
  // Right: the same on X^T with Omega_R.
  // A stage is a product and (except for the projections) the orthonormalisation
  // of its result, enqueued separately (see below).
  using Fn = std::function<hipError_t()>;
  struct Stage {
    Fn prod, orth;
  };
  std::vector<Stage> left, right;
  const bool last0 = q == 0 && !refine;
  // (the left chain's first stage is enqueued by hand below, around the fork)
  const bool q0 = q > 0;      // the first basis feeds the power iterations
  const bool pf = fuse;       // products after a fused orthonormalisation find B prepared
  right.push_back({[&] { return XtB(cr, omR, QR, false); }, [&, last0, q0] { return ORTH(cr, QR, n, last0, q0); }});
  for (int it = 0; it < q; ++it) {
    const bool last = it == q - 1 && !refine;
    const bool more = it < q - 1;   // another power iteration follows
    left.push_back({[&, pf] { return XtB(cl, QL, TN, pf); }, [&] { return ORTH(cl, TN, n, false, true); }});
    left.push_back({[&, pf] { return XB(cl, TN, QL, pf); }, [&, last, more] { return ORTH(cl, QL, m, last, more); }});
    right.push_back({[&, pf] { return XB(cr, QR, TM, pf); }, [&] { return ORTH(cr, TM, m, false, true); }});
    right.push_back({[&, pf] { return XtB(cr, TM, QR, pf); }, [&, last, more] { return ORTH(cr, QR, n, last, more); }});
  }
  // split-BF16 product op(X) B on X itself (refine_fp32 = 2, lowp_sketches = 2),
  // the thin operand split into the chain's hi / lo buffers first
  auto SPLIT = [&](const Chain& ch, int which, int at, const float* B, float* C, int64_t M, int64_t K,
                   double* sq) -> hipError_t {
    const int64_t ldbt = at ? L.ldqt : L.ldq;
    uint16_t* H = c->at<uint16_t>(which ? L.St2 : L.St);
    uint16_t* Lo = H + (size_t)k * ldbt;
    hipError_t e = launch_prep_bt(B, L.KP, K, k, H, Lo, ldbt, ch.st);
    return e ? e : launch_gemm_split(X, ldx, at, H, Lo, ldbt, C, L.KP, M, k, K, gemm_split_pick_splits(M, k, K),
                                     ch.gemm_part, ch.st, sq);
  };
  if (refine && c->p.refine_fp32 == 2) {   // the refinement on split-BF16 products (about 16 significant bits)
    left.push_back({[&] { return SPLIT(cl, 0, 1, QL, TN, n, m, nullptr); }, [&] { return ORTH(cl, TN, n, false, false); }});
    left.push_back({[&] { return SPLIT(cl, 0, 0, TN, QL, m, n, nullptr); }, [&] { return ORTH(cl, QL, m, true, false); }});
    right.push_back({[&] { return SPLIT(cr, 1, 0, QR, TM, m, n, nullptr); }, [&] { return ORTH(cr, TM, m, false, false); }});
    right.push_back({[&] { return SPLIT(cr, 1, 1, TM, QR, n, m, nullptr); }, [&] { return ORTH(cr, QR, n, true, false); }});
  } else if (refine) {   // optional FP32 refinement: one power iteration per side on the exact X
    left.push_back({[&] { return gemm(c, cl, X, ldx, 1, QL, TN, n, m); }, [&] { return ORTH(cl, TN, n, false, false); }});
    left.push_back({[&] { return gemm(c, cl, X, ldx, 0, TN, QL, m, n); }, [&] { return ORTH(cl, QL, m, true, false); }});
    right.push_back({[&] { return gemm(c, cr, X, ldx, 0, QR, TM, m, n); }, [&] { return ORTH(cr, TM, m, false, false); }});
    right.push_back({[&] { return gemm(c, cr, X, ldx, 1, TM, QR, n, m); }, [&] { return ORTH(cr, QR, n, true, false); }});
  }
  // projected data (Sec 4): Xh = X^T Q_L (X-hat^T), Xc = X Q_R (X-check); FP32 on X,
  // or on the low-precision copy like the range finder (lowp_sketches).  Q_L is
  // final when the left projection starts: ql_ready marks that point.
  c->ql_event = false;
  auto mark_ql = [&]() -> hipError_t {
    const hipError_t e = hipEventRecord(c->ql_ready, cl.st);
    if (!e) c->ql_event = true;
    return e;
  };
  if (lps) {
    left.push_back({[&] { hipError_t e = mark_ql(); return e ? e : XtB(cl, QL, Xh, false); }, nullptr});
    right.push_back({[&] { return XB(cr, QR, Xc, false); }, nullptr});
  } else if (split) {   // split-BF16 products on X
    left.push_back({[&] {
      uint16_t* H = c->at<uint16_t>(L.St);
      uint16_t* Lo = H + (size_t)k * L.ldqt;
      hipError_t e = mark_ql();
      if (!e) e = launch_prep_bt(QL, L.KP, m, k, H, Lo, L.ldqt, cl.st);
      return e ? e : launch_gemm_split(X, ldx, 1, H, Lo, L.ldqt, Xh, L.KP, n, k, m,
                                       gemm_split_pick_splits(n, k, m), cl.gemm_part, cl.st);
    }, nullptr});
    right.push_back({[&] {
      uint16_t* H = c->at<uint16_t>(L.St2);
      uint16_t* Lo = H + (size_t)k * L.ldq;
      const int s = gemm_split_pick_splits(m, k, n);
      double* sqp = xsq_quant ? nullptr : c->at<double>(L.xsq_part);
      hipError_t e = launch_prep_bt(QR, L.KP, n, k, H, Lo, L.ldq, cr.st);
      if (!e) e = launch_gemm_split(X, ldx, 0, H, Lo, L.ldq, Xc, L.KP, m, k, n, s, cr.gemm_part, cr.st, sqp);
      if (e || xsq_quant) return e;
      return launch_sum_partials_f64(sqp, gemm_split_sq_parts(m, k, s), 1, c->at<double>(L.proxy_out) + 2, nullptr,
                                     cr.st);
    }, nullptr});
  } else {
    left.push_back({[&] { hipError_t e = mark_ql(); return e ? e : gemm(c, cl, X, ldx, 1, QL, Xh, n, m); }, nullptr});
    right.push_back({[&] {   // Xc = X Q_R, with ||X||^2 in FP64 from the same pass (for the proxy residual)
      const int s = gemm_f32_pick_splits(m, k, n, 0);
      double* sqp = c->at<double>(L.xsq_part);
      hipError_t e = launch_gemm_f32(X, ldx, 0, QR, L.KP, Xc, L.KP, m, k, n, s, cr.gemm_part, cr.st, sqp);
      return e ? e : launch_sum_partials_f64(sqp, gemm_f32_sq_parts(m, k, n, s), 1, c->at<double>(L.proxy_out) + 2,
                                            nullptr, cr.st);
    }, nullptr});
  }
  // The two range finders are independent: the right one runs on a second
  // stream forked after the left one's first product and joined below, so that
  // each chain's latency-bound orthonormalisations run under the other's
  // products.  The host enqueues the stages alternately so that neither stream
  // waits for the host to finish the other's list.
  HIPCHK(c, XB(cl, omL, QL, false));
  HIPCHK(c, hipEventRecord(c->fork, st));
  HIPCHK(c, hipStreamWaitEvent(c->st2, c->fork, 0));
  HIPCHK(c, ORTH(cl, QL, m, last0, q0));
  // The host enqueues both chains' products of a stage before their
  // orthonormalisations: an orthonormalisation is up to twelve short launches,
  // and the other stream must not wait for the host to get through them before
  // its next (long) product is enqueued.
  for (size_t i = 0; i < right.size(); ++i) {
    const bool l = i < left.size();
    HIPCHK(c, right[i].prod());
    if (l) HIPCHK(c, left[i].prod());
    if (right[i].orth) HIPCHK(c, right[i].orth());
    if (l && left[i].orth) HIPCHK(c, left[i].orth());
  }
  HIPCHK(c, hipEventRecord(c->join, c->st2));
  HIPCHK(c, hipStreamWaitEvent(st, c->join, 0));
  HIPCHK(c, hipEventRecord(c->ev[1], st));
  c->t_compress = true;
  c->compressed = true;
  // factors set before this compression: their Q_R^T Ht follows the new basis
  if (c->initialized) HIPCHK(c, halfstep_h(c, 0));
  c->stepped = false;
  c->xsq_valid = true;
  return NMF_OK;
}

nmf_status nmf_init(nmf_ctx* c, const float* W0, const float* Ht0, float init_scale) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  Layout& L = c->L;
  const int64_t m = c->p.m, n = c->p.n;
  const int r = c->p.r;
  float *W = c->at<float>(L.W), *Ht = c->at<float>(L.Ht);
  if (W0) HIPCHK(c, launch_copy2d(W, r, W0, r, m, r, c->st));
  else HIPCHK(c, launch_philox_uniform(W, m, r, r, 5u, c->p.seed, init_scale, c->st));
  if (Ht0 && Ht0 != Ht) HIPCHK(c, launch_copy2d(Ht, r, Ht0, r, n, r, c->st));
  else if (!Ht0) HIPCHK(c, launch_philox_uniform(Ht, n, r, r, 6u, c->p.seed, init_scale, c->st));
  HIPCHK(c, launch_fill_f32(c->at<float>(L.scale_w), r, 1.f, c->st));
  // acc_h = Q_R^T Ht (Hc for the first W half-step); formed by nmf_compress when
  // the factors come first
  if (c->compressed) HIPCHK(c, halfstep_h(c, 0));
  c->initialized = true;
  c->stepped = false;
  return NMF_OK;
}

namespace {

nmf_status init_learned_impl(nmf_ctx* c, nmf_mlp* net, const float* align_M, const float* Wh_ref,
                             const float* W0, int64_t ldw0, const float* Ht_cold, float init_scale,
                             int32_t refine_sweeps, int64_t* n_rejected) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  if (!Wh_ref) return fail(c, NMF_EINVAL, "null Wh_ref");
  if (refine_sweeps < 0) return fail(c, NMF_EINVAL, "refine_sweeps must be >= 0");
  if (!c->compressed) return fail(c, NMF_ESTATE, "init needs the sketches: call nmf_compress or nmf_set_state first");
  const int k = c->p.k_sketch, r = c->p.r;
  if (net) {
    int nk, nh, nr;
    mlp_dims(net, &nk, &nh, &nr);
    if (nk != k || nr != r) return fail(c, NMF_EINVAL, "network must map k' inputs to r outputs");
  }
  Layout& L = c->L;
  const int64_t n = c->p.n;
  long long* cnt = reinterpret_cast<long long*>(c->at<double>(L.res_out));
  float* Ht = c->at<float>(L.Ht);
  if (!net) {   // the control without a network: the cold rows go to the sweeps as they are
    if (Ht_cold) HIPCHK(c, launch_copy2d(Ht, r, Ht_cold, r, n, r, c->st));
    else HIPCHK(c, launch_philox_uniform(Ht, n, r, r, 6u, c->p.seed, init_scale, c->st));
    int* ones = reinterpret_cast<int*>(c->at<float>(L.TN));
    HIPCHK(c, launch_fill_i32(ones, n, 1, c->st));
    HIPCHK(c, launch_count(ones, (int)n, cnt, c->st));
  }
  // 1. network input: x-tilde = M x-hat (rows: Xh M^T), else x-hat itself
  const float* in = c->at<float>(L.Xh);
  int64_t ld_in = L.KP;
  if (net && align_M) {
    float* Xa = c->at<float>(L.omL);  // n x k' (the test matrix is not needed after compression)
    HIPCHK(c, launch_mlp_gemm(0, 1, 0, in, (int)L.KP, align_M, k, Xa, k, (int)n, k, k, nullptr, nullptr, 0, c->st));
    in = Xa;
    ld_in = k;
  }
  if (net) {
    // 2. the network's rows and the cold rows
    float* Hn = c->at<float>(L.TN);
    HIPCHK(c, mlp_infer_rows(net, in, ld_in, n, Hn, r, c->st));
    if (Ht_cold) HIPCHK(c, launch_copy2d(Ht, r, Ht_cold, r, n, r, c->st));
    else HIPCHK(c, launch_philox_uniform(Ht, n, r, r, 6u, c->p.seed, init_scale, c->st));
    // 3. per-row choice by the compressed residual against Wh_ref, in place into Ht
    int* rej = reinterpret_cast<int*>(Hn + n * r);   // TN is n x KP floats, r < KP
    HIPCHK(c, launch_select(c->at<float>(L.Xh), L.KP, (int)n, k, Wh_ref, r, Hn, Ht, Ht, rej, cnt, c->st));
  }
  // 4. optional column-NNLS sweeps against Wh_ref from the selected rows (each
  //    sweep lowers every row's compressed residual)
  if (refine_sweeps > 0)
    HIPCHK(c, launch_nnls_rows(c->at<float>(L.Xh), L.KP, (int)n, k, Wh_ref, r, refine_sweeps, 1, Ht, r, c->st));
  // 5. W as in nmf_init; the first update is the W half-step
  const float* W0c = W0;
  if (W0 && ldw0 != r) {   // nmf_init copies W0 with leading dimension r
    HIPCHK(c, launch_copy2d(c->at<float>(L.W), r, W0, ldw0, c->p.m, r, c->st));
    W0c = c->at<float>(L.W);
  }
  nmf_status s = nmf_init(c, W0c, Ht, init_scale);
  if (s != NMF_OK) return s;
  if (n_rejected) {
    long long h = 0;
    HIPCHK(c, hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    *n_rejected = h;
  }
  return NMF_OK;
}

}  // namespace

nmf_status nmf_init_learned(nmf_ctx* c, nmf_mlp* net, const float* align_M, const float* Wh_ref,
                            const float* W0, const float* Ht_cold, float init_scale, int32_t refine_sweeps,
                            int64_t* n_rejected) {
  return init_learned_impl(c, net, align_M, Wh_ref, W0, c ? c->p.r : 0, Ht_cold, init_scale, refine_sweeps,
                           n_rejected);
}

nmf_status nmf_init_learned_ref(nmf_ctx* c, nmf_mlp* net, const float* Q_train, int64_t ldq, const float* W_ref,
                                int64_t ldw, const float* Ht_cold, float init_scale, int32_t refine_sweeps,
                                int64_t* n_rejected) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  if (!Q_train || !W_ref) return fail(c, NMF_EINVAL, "null Q_train or W_ref");
  const int k = c->p.k_sketch, r = c->p.r;
  if (ldq < k || ldw < r) return fail(c, NMF_EINVAL, "leading dimension too small");
  if (!c->compressed) return fail(c, NMF_ESTATE, "init needs the sketches: call nmf_compress or nmf_set_state first");
  Layout& L = c->L;
  const int64_t m = c->p.m;
  const int splits = gram_pick_splits(m, k);
  float* M = c->at<float>(L.alignM);
  float* Wh = c->at<float>(L.whref);
  double* part = c->at<double>(L.gram_part);
  double* C64 = c->at<double>(L.G);
  // M = Q_train^T Q_L (k' x k'), Wh_ref = Q_L^T W_ref (k' x r), FP64 sums over the m rows.
  // They need only Q_L: on the third stream from the point nmf_compress marked
  // (Q_L final), so that they run under the sketch products, one after the other
  // in the left range finder's Gram scratch (its last use precedes that point;
  // the right range finder's may still be running).  Only the first warm start
  // after a compression starts there; after nmf_set_state or a previous warm start
  // (whose network may still read M), from the present point of the context's stream.
  if (!c->ql_event) HIPCHK(c, hipEventRecord(c->ql_ready, c->st));
  c->ql_event = false;
  HIPCHK(c, hipStreamWaitEvent(c->st3, c->ql_ready, 0));
  HIPCHK(c, launch_atb_f32out(Q_train, ldq, k, c->at<float>(L.QL), L.KP, k, m, part, splits, C64, M, c->st3));
  HIPCHK(c, launch_atb_f32out(c->at<float>(L.QL), L.KP, k, W_ref, ldw, r, m, part, splits, C64, Wh, c->st3));
  HIPCHK(c, hipEventRecord(c->aligned, c->st3));
  HIPCHK(c, hipStreamWaitEvent(c->st, c->aligned, 0));
  return init_learned_impl(c, net, M, Wh, W_ref, ldw, Ht_cold, init_scale, refine_sweeps, n_rejected);
}

nmf_status nmf_step(nmf_ctx* c, int32_t iters) {
  if (!c || iters < 0) return fail(c, NMF_EINVAL, "bad arguments");
  if (!c->initialized) return fail(c, NMF_ESTATE, "step needs nmf_init");
  if (!c->compressed) return fail(c, NMF_ESTATE, "step needs the sketches: call nmf_compress or nmf_set_state first");
  HIPCHK(c, hipEventRecord(c->ev[2], c->st));
  for (int t = 0; t < iters; ++t) {
    HIPCHK(c, halfstep_w(c));
    HIPCHK(c, halfstep_h(c, 1));
  }
  HIPCHK(c, hipEventRecord(c->ev[3], c->st));
  c->t_step = true;
  if (iters > 0) c->stepped = true;
  return NMF_OK;
}

nmf_status nmf_fasthals_step(nmf_ctx* c, const float* X, int64_t ldx, int32_t iters) {
  if (!c || !X || iters < 0) return fail(c, NMF_EINVAL, "bad arguments");
  if (ldx < c->p.n || ldx % 4 || !aligned16(X)) return fail(c, NMF_EINVAL, "X needs ldx >= n, ldx % 4 == 0, 16-byte alignment");
  if (!c->initialized) return fail(c, NMF_ESTATE, "fasthals step needs factors (nmf_init)");
  if (iters == 0) return NMF_OK;
  Layout& L = c->L;
  const int64_t m = c->p.m, n = c->p.n;
  const int r = c->p.r;
  const int64_t rp = round_up(r, 4);   // rows of the working copies: 16-byte aligned operands
  hipStream_t st = c->st;
  float *W = c->at<float>(L.W), *Ht = c->at<float>(L.Ht), *sw = c->at<float>(L.scale_w);
  // working copies in the test-matrix buffers (free after compression; k' > r, so
  // K = k' rounded up to 4 >= rp), products in the temporaries
  float *Wp = c->at<float>(L.omR), *Hp = c->at<float>(L.omL);
  float *PW = c->at<float>(L.TM), *PH = c->at<float>(L.TN);   // X Ht (m x r), X^T W (n x r)
  double* G = c->at<double>(L.G);                             // r x r Gram (r < k')
  double* cs = c->at<double>(L.acc_w);                        // r column sums of W^2
  float* sqp = c->at<float>(L.hs_part);
  float* gp = c->at<float>(L.gemm_part);
  const size_t hs_floats = std::max(halfstep_part_floats(m, (int)L.KP, r), halfstep_part_floats(n, (int)L.KP, r));
  if ((size_t)hals_rows_blocks(m) * r > hs_floats) return fail(c, NMF_ENOMEM, "column-sum partials exceed the scratch");
  // W with the compressed steps' pending column normalisation applied
  HIPCHK(c, launch_fill_f32(Wp, m * rp, 0.f, st));
  HIPCHK(c, launch_fill_f32(Hp, n * rp, 0.f, st));
  HIPCHK(c, launch_scale_cols(Wp, rp, W, r, m, r, sw, st));
  HIPCHK(c, launch_copy2d(Hp, rp, Ht, r, n, r, st));
  // split-K partials within the context's product scratch
  auto splits_for = [&](int64_t M, int64_t K, int at) {
    int s = gemm_f32_pick_splits(M, r, K, at);
    while (s > 1 && gemm_f32_part_floats(M, r, s) * sizeof(float) > L.gemm_part_bytes) s /= 2;
    return s;
  };
  const int s_w = splits_for(m, n, 0), s_h = splits_for(n, m, 1);
  const bool nrm = c->p.normalize != 0;
  for (int it = 0; it < iters; ++it) {
    // W sweep against X Ht and Ht^T Ht, then a_j / ||a_j||
    HIPCHK(c, launch_gemm_f32(X, ldx, 0, Hp, rp, PW, rp, m, r, n, s_w, gp, st));
    HIPCHK(c, launch_gram_f64(Hp, rp, n, r, c->at<double>(L.gram_part), gram_pick_splits(n, r), G, nullptr, st));
    HIPCHK(c, launch_hals_rows(PW, rp, G, m, r, Wp, rp, nrm ? sqp : nullptr, st));
    if (nrm) {
      HIPCHK(c, launch_sum_partials_f32(sqp, hals_rows_blocks(m), r, cs, st));
      HIPCHK(c, launch_col_normalise(Wp, m, Hp, n, r, rp, cs, c->p.normalize, st));
    }
    // H sweep against X^T W and W^T W
    HIPCHK(c, launch_gemm_f32(X, ldx, 1, Wp, rp, PH, rp, n, r, m, s_h, gp, st));
    HIPCHK(c, launch_gram_f64(Wp, rp, m, r, c->at<double>(L.gram_part), gram_pick_splits(m, r), G, nullptr, st));
    HIPCHK(c, launch_hals_rows(PH, rp, G, n, r, Hp, rp, nullptr, st));
  }
  HIPCHK(c, launch_copy2d(W, r, Wp, rp, m, r, st));
  HIPCHK(c, launch_copy2d(Ht, r, Hp, rp, n, r, st));
  HIPCHK(c, launch_fill_f32(sw, r, 1.f, st));
  // the compressed update's state (Q_R^T Ht) follows the new factors
  if (c->compressed) HIPCHK(c, halfstep_h(c, 0));
  c->stepped = false;
  return NMF_OK;
}

nmf_status nmf_residual(nmf_ctx* c, const float* X, int64_t ldx, double* rel_err) {
  if (!c || !X || !rel_err || ldx < c->p.n) return fail(c, NMF_EINVAL, "bad arguments");
  if (!c->initialized) return fail(c, NMF_ESTATE, "residual needs factors (nmf_init)");
  Layout& L = c->L;
  HIPCHK(c, hipEventRecord(c->ev[4], c->st));
  HIPCHK(c, launch_residual(X, ldx, c->p.m, c->p.n, c->at<float>(L.W), c->at<float>(L.scale_w),
                            c->at<float>(L.Ht), c->p.r, c->at<double>(L.res_part),
                            c->at<double>(L.res_out), c->at<unsigned>(L.counters) + 4, c->st));
  HIPCHK(c, hipEventRecord(c->ev[5], c->st));
  HIPCHK(c, launch_gather_host(nullptr, c->at<double>(L.res_out), c->at<int>(L.qr_status), c->hout_dev, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double* hr = c->hout;
  const double h[2] = {hr[3], hr[4]};
  c->t_residual = true;
  if (hr[5] != 0.0 || hr[6] != 0.0) return fail(c, NMF_EBREAKDOWN, "Cholesky breakdown in the range finder");
  *rel_err = (h[1] > 0) ? std::sqrt(h[0] / h[1]) : 0.0;
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(c, NMF_ENONFINITE, "non-finite residual");
  return NMF_OK;
}

namespace {

// Bound on |e32 - e| for the residual from FP32 products (W, Ht >= 0), e32 its
// value and xsq = ||X||^2.  With u = 2^-23 and g = (r + 1) u / (1 - (r + 1) u):
// each P_ij is a sum of r nonnegative products of FP32 values (one of them scaled
// by sw), so |P32_ij - P_ij| <= g P_ij; the subtraction adds u' |E32_ij|,
// u' = u / (1 - u); ||P|| <= ||X|| (1 + e).  Hence
// |e32 - e| <= (g (1 + e32) + u' e32) / (1 - g), plus r 2^-126 sqrt(m n) / ||X||
// for products flushed to zero below the FP32 normal range, and 1e-12 e32 for
// the FP64 sums.
// |e_s - e| for the split-BF16 residual, W, Ht >= 0: per product the FP32
// scaling of W (2^-24) and the split representation (v = hi + lo + d with
// |d| <= 2^-16 |v|: the three kept terms miss at most 3.03 2^-16 |v_a v_b|), per
// element 3 KR FP32 additions over terms whose magnitudes sum to at most
// 1.02 sum |w h| (u = 2^-23 covers truncation as well as nearest rounding); the
// elementwise bound g sum_k |w_ik h_jk| has norm g ||W Ht^T|| <= g (1 + e) ||X||,
// and the subtraction X - P adds u' e.
double split_residual_bound(int KR, int64_t m, int64_t n, double es, double xsq) {
  const double u = std::ldexp(1.0, -23), up = u / (1.0 - u);
  const double g0 = std::ldexp(1.0, -24) + 3.03 * std::ldexp(1.0, -16) + 1.02 * 3 * KR * u;
  const double g = g0 / (1.0 - g0);
  double b = (g * (1.0 + es) + up * es) / (1.0 - g) + 1e-12 * es;
  if (xsq > 0) b += 3 * KR * std::ldexp(1.0, -126) * std::sqrt((double)m * (double)n) / std::sqrt(xsq);
  return b;
}

}  // namespace

namespace {

// The split-BF16 residual over all of X and its bound (split_residual_bound).
nmf_status split_check(nmf_ctx* c, const float* X, int64_t ldx, double* es, double* beta) {
  Layout& L = c->L;
  HIPCHK(c, hipEventRecord(c->ev[4], c->st));
  HIPCHK(c, launch_residual_split(X, ldx, c->p.m, c->p.n, c->at<float>(L.W), c->at<float>(L.scale_w),
                                  c->at<float>(L.Ht), c->p.r, c->at<uint16_t>(L.rsplit), c->at<double>(L.res_part),
                                  c->at<double>(L.res_out), c->at<unsigned>(L.counters) + 4, c->st));
  HIPCHK(c, hipEventRecord(c->ev[5], c->st));
  HIPCHK(c, launch_gather_host(nullptr, c->at<double>(L.res_out), c->at<int>(L.qr_status), c->hout_dev, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double* hr = c->hout;
  c->t_residual = true;
  if (hr[5] != 0.0 || hr[6] != 0.0) return fail(c, NMF_EBREAKDOWN, "Cholesky breakdown in the range finder");
  if (!std::isfinite(hr[3]) || !std::isfinite(hr[4])) return fail(c, NMF_ENONFINITE, "non-finite residual");
  *es = (hr[4] > 0) ? std::sqrt(hr[3] / hr[4]) : 0.0;
  *beta = split_residual_bound(residual_split_kr(c->p.r), c->p.m, c->p.n, *es, hr[4]);
  return NMF_OK;
}

}  // namespace

nmf_status nmf_residual_check(nmf_ctx* c, const float* X, int64_t ldx, double eps, double* rel_err, double* bound,
                              int32_t* exact) {
  if (!c || !X || !rel_err || ldx < c->p.n) return fail(c, NMF_EINVAL, "bad arguments");
  if (!c->initialized) return fail(c, NMF_ESTATE, "residual needs factors (nmf_init)");
  double e32 = 0.0, b = 0.0;
  nmf_status s;
  if ((s = split_check(c, X, ldx, &e32, &b)) != NMF_OK) return s;
  if (std::fabs(e32 - eps) <= b) {   // either side of eps within the bound: the exact value decides
    if (exact) *exact = 1;
    if (bound) *bound = 0.0;
    return nmf_residual(c, X, ldx, rel_err);
  }
  if (exact) *exact = 0;
  if (bound) *bound = b;
  *rel_err = e32;
  return NMF_OK;
}

nmf_status nmf_proxy_residual(nmf_ctx* c, double* rel_err) {
  if (!c || !rel_err) return fail(c, NMF_EINVAL, "bad arguments");
  if (!c->stepped) return fail(c, NMF_ESTATE, "the proxy needs at least one nmf_step after init");
  if (!c->xsq_valid) return fail(c, NMF_ESTATE, "the proxy needs ||X||^2 from nmf_compress (not nmf_set_state)");
  Layout& L = c->L;
  const int nb = proxy_blocks(c->p.n);
  HIPCHK(c, launch_proxy(c->at<float>(L.Xh), L.KP, c->at<float>(L.Ht), c->p.r, c->at<float>(L.Wh), c->p.k_sketch,
                         c->p.n, c->at<double>(L.proxy_part), c->st));
  HIPCHK(c, launch_sum_partials_f64(c->at<double>(L.proxy_part), nb, 2, c->at<double>(L.proxy_out), nullptr, c->st));
  HIPCHK(c, launch_gather_host(c->at<double>(L.proxy_out), nullptr, nullptr, c->hout_dev, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double h[3] = {c->hout[0], c->hout[1], c->hout[2]};
  if (!(h[2] > 0)) return fail(c, NMF_ENONFINITE, "||X||^2 is zero or not finite");
  const double e2 = (h[2] - h[1] + h[0]) / h[2];
  if (!std::isfinite(e2)) return fail(c, NMF_ENONFINITE, "non-finite proxy");
  *rel_err = std::sqrt(e2 > 0 ? e2 : 0.0);
  return NMF_OK;
}

nmf_status nmf_sketch_spectrum(nmf_ctx* c, double* sigma) {
  if (!c || !sigma) return fail(c, NMF_EINVAL, "bad arguments");
  if (!c->compressed) return fail(c, NMF_ESTATE, "the spectrum needs the compressed data (nmf_compress or nmf_set_state)");
  Layout& L = c->L;
  const int k = c->p.k_sketch;
  const int64_t n = c->p.n;
  // X-hat X-hat^T = Xh^T Xh (k' x k', FP64) in the second chain's scratch, then its eigenvalues
  double* G = c->at<double>(L.G2);
  double* w = c->at<double>(L.R2);
  int* info = (int*)(c->hout_dev + 8);
  HIPCHK(c, launch_gram_f64(c->at<float>(L.Xh), L.KP, n, k, c->at<double>(L.gram_part2), gram_pick_splits(n, k), G,
                            nullptr, c->st));
  HIPCHK(c, launch_sym_eig(G, k, k, 1, w, info, c->st));
  HIPCHK(c, hipMemcpyAsync(sigma, w, (size_t)k * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const int* hi = (const int*)(c->hout + 8);
  if (hi[1]) return fail(c, NMF_ENONFINITE, "non-finite compressed data");
  return NMF_OK;
}

namespace {

// Residual estimated on a sample of the rows: the split-BF16 sums over every
// s-th 256-row strip (s = strips / 64, about 64 strips; all of them for
// m <= 16384), e_hat^2 = sum (X - P)^2 / sum X^2 over the sample.  A scheduling
// signal only: no stop is decided on it.
nmf_status sampled_residual(nmf_ctx* c, const float* X, int64_t ldx, double* eh) {
  Layout& L = c->L;
  const int64_t strips = ceil_div(c->p.m, (int64_t)256);
  const int64_t sstep = strips > 64 ? strips / 64 : 1;
  HIPCHK(c, launch_residual_split(X, ldx, c->p.m, c->p.n, c->at<float>(L.W), c->at<float>(L.scale_w),
                                  c->at<float>(L.Ht), c->p.r, c->at<uint16_t>(L.rsplit), c->at<double>(L.res_part),
                                  c->at<double>(L.res_out), c->at<unsigned>(L.counters) + 4, c->st, nullptr, 0.0,
                                  sstep));
  HIPCHK(c, launch_gather_host(nullptr, c->at<double>(L.res_out), c->at<int>(L.qr_status), c->hout_dev, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double* hr = c->hout;
  if (hr[5] != 0.0 || hr[6] != 0.0) return fail(c, NMF_EBREAKDOWN, "Cholesky breakdown in the range finder");
  if (!std::isfinite(hr[3]) || !std::isfinite(hr[4])) return fail(c, NMF_ENONFINITE, "non-finite residual");
  *eh = (hr[4] > 0) ? std::sqrt(hr[3] / hr[4]) : 0.0;
  return NMF_OK;
}

// Adaptive schedule.  After every chunk (5 first, then 1.2x the iterations a
// straight-line extrapolation of the last two readings needs to reach the
// target, 5..50; with one reading 20, 10 or 5 by its distance from it) the
// residual is estimated on a sample of the rows (sampled_residual).  The target
// is eps - beta, beta the bound of the split-BF16 residual (split_check) at the
// estimate: below it the split residual decides e <= eps by itself.  The split
// residual over all of X runs once the estimate reaches the target, once it is
// within 1 % of eps with the target out of reach (more than 20 further
// iterations at the current rate, or no progress), and after the last chunk.
// A split value within its bound of eps leaves the side of eps open: if the
// target is a few iterations away (at most 10 at the current rate) the
// iterations continue and the split residual runs again; otherwise, and for a
// second open value in a row or after the last chunk, the exact FP64 residual
// settles it.  Every stop decision is therefore that of the exact e; an
// estimate that errs high only delays a stop.
nmf_status fit_sampled_schedule(nmf_ctx* c, const float* X, int64_t ldx, int32_t max_iters, double eps,
                                int* iters_done, double* rel_err) {
  nmf_status s;
  int done = 0, chunk = 5;
  bool open = false;
  double e = NAN;
  bool fresh = false;     // e belongs to the current factors
  int t_prev = -1;
  double v_prev = 0.0;
  const double kr3 = 3.0 * residual_split_kr(c->p.r);
  // the bound at e, with ||X|| large enough that the underflow term is negligible
  auto beta_at = [&](double v) {
    const double u = std::ldexp(1.0, -23), up = u / (1.0 - u);
    const double g0 = std::ldexp(1.0, -24) + 3.03 * std::ldexp(1.0, -16) + 1.02 * kr3 * u, g = g0 / (1.0 - g0);
    return (g * (1.0 + v) + up * v) / (1.0 - g) + 1e-12 * v;
  };
  // iterations to reach `target` from v at the rate of the last two readings (inf: no progress)
  auto need_for = [&](double v, int t, double target) {
    const double slope = t_prev >= 0 && t > t_prev ? (v_prev - v) / (t - t_prev) : 0.0;
    if (v <= target) return 0.0;
    return slope > 0 ? (v - target) / slope : HUGE_VAL;
  };
  auto next_chunk = [&](double v, int t, double target, int lo) {
    const double need = need_for(v, t, target);
    int ch;
    if (std::isfinite(need) && t_prev >= 0) {
      const double n12 = std::ceil(1.2 * need);
      ch = n12 < lo ? lo : n12 > 50 ? 50 : (int)n12;
    } else {
      const double gap = (v - target) / (target > 0 ? target : 1.0);
      ch = gap > 0.1 ? 20 : gap > 0.01 ? 10 : 5;
      if (ch < lo) ch = lo;
    }
    t_prev = t;
    v_prev = v;
    return ch;
  };
  while (done < max_iters) {
    if (chunk > max_iters - done) chunk = max_iters - done;
    if ((s = nmf_step(c, chunk)) != NMF_OK) return s;
    done += chunk;
    fresh = false;
    double v;
    if ((s = sampled_residual(c, X, ldx, &v)) != NMF_OK) return s;
    const bool last = done >= max_iters;
    int lo = 5;
    const double target = eps - beta_at(v);
    const bool stalled = v <= eps * 1.01 && (t_prev < 0 || need_for(v, done, target) > 20.0);
    if (v <= target || stalled || open || last) {
      double es, b;
      if ((s = split_check(c, X, ldx, &es, &b)) != NMF_OK) return s;
      if (std::fabs(es - eps) > b) {           // decided by the split value
        e = es;
        fresh = true;
        open = false;
        if (e <= eps) break;
      } else if (open || last || need_for(es, done, eps - b) > 10.0) {   // settled by the exact residual
        if ((s = nmf_residual(c, X, ldx, &e)) != NMF_OK) return s;
        fresh = true;
        open = false;
        if (e <= eps) break;
        es = e;
      } else {
        open = true;
        lo = 2;
      }
      v = es;
    }
    chunk = next_chunk(v, done, eps - beta_at(v), lo);
  }
  if (!fresh && (s = nmf_residual(c, X, ldx, &e)) != NMF_OK) return s;
  *iters_done = done;
  *rel_err = e;
  return NMF_OK;
}

}  // namespace

nmf_status nmf_fit(nmf_ctx* c, const float* X, int64_t ldx, int32_t max_iters, double eps,
                   int32_t check_every, int32_t* iters_done, double* rel_err) {
  if (!c || !X || check_every < 0 || max_iters < 0) return fail(c, NMF_EINVAL, "bad arguments");
  if (check_every == 0 && max_iters > 0 && c->xsq_valid && c->initialized) {
    int it = 0;
    double ee = 0.0;
    const nmf_status st = fit_sampled_schedule(c, X, ldx, max_iters, eps, &it, &ee);
    if (iters_done) *iters_done = it;
    if (rel_err) *rel_err = ee;
    return st;
  }
  int done = 0;
  double e = 0.0;
  nmf_status s;
  // Adaptive schedule: after two checks, step 1.5x the iterations a linear
  // extrapolation of the last two errors needs to reach eps (5..50); before
  // that, by the relative gap to eps.
  int t_prev = -1;
  double e_prev = 0.0;
  auto next_chunk = [&](int t, double err) {
    int ch;
    const double slope = t_prev >= 0 && t > t_prev ? (e_prev - err) / (t - t_prev) : 0.0;
    if (t_prev >= 0 && slope > 0) {
      const double need = std::ceil(1.5 * (err - eps) / slope);
      ch = need < 5 ? 5 : need > 50 ? 50 : (int)need;
    } else if (t_prev >= 0) {
      ch = 50;
    } else {
      const double gap = (err - eps) / (eps > 0 ? eps : 1.0);
      ch = gap > 0.1 ? 50 : gap > 0.01 ? 20 : gap > 0.003 ? 10 : 5;
    }
    t_prev = t;
    e_prev = err;
    return ch;
  };
  int chunk = check_every;
  if (max_iters == 0 || check_every == 0) {   // the adaptive schedule starts from e at the current factors
    if ((s = nmf_residual(c, X, ldx, &e)) != NMF_OK) return s;
    if (check_every == 0) {
      if (e <= eps) max_iters = 0;
      chunk = next_chunk(0, e);
    }
  }
  while (done < max_iters) {
    if (chunk > max_iters - done) chunk = max_iters - done;
    if ((s = nmf_step(c, chunk)) != NMF_OK) return s;
    done += chunk;
    if ((s = nmf_residual(c, X, ldx, &e)) != NMF_OK) return s;
    if (e <= eps) break;
    if (check_every == 0) chunk = next_chunk(done, e);
  }
  if (iters_done) *iters_done = done;
  if (rel_err) *rel_err = e;
  return NMF_OK;
}

nmf_status nmf_get_factors(nmf_ctx* c, float* W, float* Ht) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  if (!c->initialized) return fail(c, NMF_ESTATE, "no factors yet");
  Layout& L = c->L;
  const int r = c->p.r;
  if (W) HIPCHK(c, launch_scale_cols(W, r, c->at<float>(L.W), r, c->p.m, r, c->at<float>(L.scale_w), c->st));
  if (Ht) HIPCHK(c, launch_copy2d(Ht, r, c->at<float>(L.Ht), r, c->p.n, r, c->st));
  return NMF_OK;
}

nmf_status nmf_get_state(nmf_ctx* c, float* QL, float* QR, float* Xh, float* Xc) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  if (!c->compressed) return fail(c, NMF_ESTATE, "no sketches yet");
  Layout& L = c->L;
  const int k = c->p.k_sketch;
  if (QL) HIPCHK(c, launch_copy2d(QL, k, c->at<float>(L.QL), L.KP, c->p.m, k, c->st));
  if (QR) HIPCHK(c, launch_copy2d(QR, k, c->at<float>(L.QR), L.KP, c->p.n, k, c->st));
  if (Xh) HIPCHK(c, launch_copy2d(Xh, k, c->at<float>(L.Xh), L.KP, c->p.n, k, c->st));
  if (Xc) HIPCHK(c, launch_copy2d(Xc, k, c->at<float>(L.Xc), L.KP, c->p.m, k, c->st));
  return NMF_OK;
}

nmf_status nmf_set_state(nmf_ctx* c, const float* QL, const float* QR, const float* Xh,
                         const float* Xc) {
  if (!c || !QL || !QR || !Xh || !Xc) return fail(c, NMF_EINVAL, "null argument");
  Layout& L = c->L;
  const int k = c->p.k_sketch;
  HIPCHK(c, launch_copy2d(c->at<float>(L.QL), L.KP, QL, k, c->p.m, k, c->st));
  HIPCHK(c, launch_copy2d(c->at<float>(L.QR), L.KP, QR, k, c->p.n, k, c->st));
  HIPCHK(c, launch_copy2d(c->at<float>(L.Xh), L.KP, Xh, k, c->p.n, k, c->st));
  HIPCHK(c, launch_copy2d(c->at<float>(L.Xc), L.KP, Xc, k, c->p.m, k, c->st));
  HIPCHK(c, launch_fill_i32(c->at<int>(L.qr_status), 16, 0, c->st));
  c->ql_event = false;
  c->compressed = true;
  c->stepped = false;
  c->xsq_valid = false;
  c->initialized = false;
  return NMF_OK;
}

nmf_status nmf_sync(nmf_ctx* c, int32_t* shifted) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  int qs[16];
  HIPCHK(c, hipMemcpyAsync(qs, c->at<int>(c->L.qr_status), sizeof(qs), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (shifted) *shifted = qs[2] + qs[10];
  if (qs[1] || qs[9]) return fail(c, NMF_EBREAKDOWN, "Cholesky breakdown in the range finder");
  return NMF_OK;
}

nmf_status nmf_stage_times(nmf_ctx* c, double* compress_ms, double* step_ms, double* residual_ms) {
  if (!c) return fail(c, NMF_EINVAL, "null context");
  HIPCHK(c, hipStreamSynchronize(c->st));
  float t;
  if (compress_ms) { *compress_ms = -1; if (c->t_compress && hipEventElapsedTime(&t, c->ev[0], c->ev[1]) == hipSuccess) *compress_ms = t; }
  if (step_ms) { *step_ms = -1; if (c->t_step && hipEventElapsedTime(&t, c->ev[2], c->ev[3]) == hipSuccess) *step_ms = t; }
  if (residual_ms) { *residual_ms = -1; if (c->t_residual && hipEventElapsedTime(&t, c->ev[4], c->ev[5]) == hipSuccess) *residual_ms = t; }
  return NMF_OK;
}

nmf_status nmf_gaussian(float* out, int64_t rows, int64_t cols, int64_t ld, uint32_t sid,
                        uint64_t seed, void* hs) {
  if (!out || rows < 0 || cols < 0 || ld < cols) return fail(nullptr, NMF_EINVAL, "bad arguments");
  hipError_t e = launch_philox_normal(out, rows, cols, ld, sid, seed, (hipStream_t)hs);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

nmf_status nmf_uniform(float* out, int64_t rows, int64_t cols, int64_t ld, uint32_t sid,
                       uint64_t seed, float scale, void* hs) {
  if (!out || rows < 0 || cols < 0 || ld < cols) return fail(nullptr, NMF_EINVAL, "bad arguments");
  hipError_t e = launch_philox_uniform(out, rows, cols, ld, sid, seed, scale, (hipStream_t)hs);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

size_t nmf_gemm_workspace_bytes(int64_t M, int64_t N, int64_t K, int32_t a_trans) {
  const int s = gemm_f32_pick_splits(M, N, K, a_trans);
  return gemm_f32_part_floats(M, N, s) * sizeof(float) + 256;
}

nmf_status nmf_gemm(const float* A, int64_t lda, int32_t a_trans, const float* B, int64_t ldb,
                    float* C, int64_t ldc, int64_t M, int64_t N, int64_t K, void* ws, size_t ws_bytes,
                    void* hs) {
  if (M < 0 || N < 0 || K < 0 || N > 256 || ldc < N) return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0 || N == 0) return NMF_OK;
  if (!A || !B || !C) return fail(nullptr, NMF_EINVAL, "null pointer");
  if (lda % 4 || ldb % 4 || !aligned16(A) || !aligned16(B)) return fail(nullptr, NMF_EINVAL, "lda, ldb % 4 and 16-byte alignment required");
  if ((!a_trans && K % 4) || (a_trans && M % 4)) return fail(nullptr, NMF_EINVAL, "K % 4 (a_trans=0) or M % 4 (a_trans=1) required");
  if ((!a_trans && lda < K) || (a_trans && lda < M) || ldb < N) return fail(nullptr, NMF_EINVAL, "leading dimension too small");
  const int s = gemm_f32_pick_splits(M, N, K, a_trans);
  const size_t need = gemm_f32_part_floats(M, N, s) * sizeof(float);
  if (need && (!ws || ws_bytes < need)) return fail(nullptr, NMF_ENOMEM, "workspace too small");
  hipError_t e = launch_gemm_f32(A, lda, a_trans, B, ldb, C, ldc, M, N, K, s, (float*)ws, (hipStream_t)hs);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

nmf_status nmf_quantize_x(const float* X, int64_t ldx, int64_t m, int64_t n, int32_t prec, void* Xq,
                          int64_t ldq, void* XqT, int64_t ldqt, int32_t* tile_exp, void* hs) {
  if (!X || !Xq || !XqT || m <= 0 || n <= 0 || ldx < n) return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (ldq < n || ldqt < m || ldq % 128 || ldqt % 128) return fail(nullptr, NMF_EINVAL, "ldq, ldqt: >= n, m and multiples of 128");
  hipError_t e;
  if (prec == NMF_BF16) {
    e = launch_quant_bf16(X, ldx, m, n, (uint16_t*)Xq, ldq, (uint16_t*)XqT, ldqt, (hipStream_t)hs);
  } else if (prec == NMF_FP8_E4M3) {
    if (!tile_exp) return fail(nullptr, NMF_EINVAL, "tile_exp required for FP8");
    e = launch_quant_fp8(X, ldx, m, n, tile_exp, (uint8_t*)Xq, ldq, (uint8_t*)XqT, ldqt, (hipStream_t)hs);
  } else {
    return fail(nullptr, NMF_EINVAL, "prec must be BF16 or FP8_E4M3");
  }
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

size_t nmf_gemm_lowp_workspace_bytes(int64_t M, int64_t N, int64_t Kpad) {
  const int s = gemm_lp_pick_splits(M, N, Kpad, 128);
  return (size_t)N * Kpad * 2 + (size_t)ceil_div(Kpad, 128) * 4 + (s > 1 ? (size_t)s * M * N * 4 : 0) + 1024;
}

nmf_status nmf_gemm_lowp(int32_t prec, const void* A, int64_t lda, const int32_t* EA, int64_t ea_i,
                         int64_t ea_k, const float* B, int64_t ldb, int64_t K, int64_t N, float* C,
                         int64_t ldc, int64_t M, int64_t Kpad, void* ws, size_t ws_bytes, void* hs) {
  if (M < 0 || N <= 0 || N > 256 || K <= 0 || Kpad < K || Kpad % 128 || ldb < N || ldc < N || lda < Kpad)
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0) return NMF_OK;
  if (!A || !B || !C || !ws || ws_bytes < nmf_gemm_lowp_workspace_bytes(M, N, Kpad) || ((uintptr_t)ws & 255))
    return fail(nullptr, NMF_EINVAL, "null pointer or workspace too small / misaligned");
  hipStream_t st = (hipStream_t)hs;
  char* p = (char*)ws;
  void* Bt = p;
  p += round_up((int64_t)N * Kpad * 2, 256);
  int* Eb = (int*)p;
  p += round_up(ceil_div(Kpad, 128) * 4, 256);
  float* part = (float*)p;
  const int s = gemm_lp_pick_splits(M, N, Kpad, 128);
  hipError_t e;
  if (prec == NMF_BF16) {
    e = launch_prep_b_bf16(B, ldb, K, N, (uint16_t*)Bt, Kpad, st);
    if (!e) e = launch_gemm_bf16_nt((const uint16_t*)A, lda, (const uint16_t*)Bt, Kpad, C, ldc, M, N, Kpad, s, part, st);
  } else if (prec == NMF_FP8_E4M3) {
    if (!EA) return fail(nullptr, NMF_EINVAL, "EA required for FP8");
    e = launch_prep_b_fp8(B, ldb, K, N, Eb, (uint8_t*)Bt, Kpad, st);
    if (!e) e = launch_gemm_fp8_nt((const uint8_t*)A, lda, EA, ea_i, ea_k, (const uint8_t*)Bt, Kpad, Eb, C, ldc, M, N, Kpad, s, part, st);
  } else {
    return fail(nullptr, NMF_EINVAL, "prec must be BF16 or FP8_E4M3");
  }
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

size_t nmf_gemm_split_workspace_bytes(int64_t M, int64_t N, int64_t K) {
  if (M < 0 || N <= 0 || K <= 0) return 0;
  const int64_t Kpad = round_up(K, 64);
  const int s = gemm_split_pick_splits(M, N, K);
  return (size_t)round_up(2 * N * Kpad * 2, 256) + (s > 1 ? (size_t)s * M * N * 4 : 0) + 1024;
}

nmf_status nmf_gemm_split(const float* X, int64_t ldx, int32_t at, const float* B, int64_t ldb, int64_t K,
                          int64_t N, float* C, int64_t ldc, int64_t M, void* ws, size_t ws_bytes, void* hs) {
  if (M < 0 || N <= 0 || N > 256 || K <= 0 || (at != 0 && at != 1) || ldb < N || ldc < N ||
      ldx < (at ? M : K) || ldx % 4)
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0) return NMF_OK;
  if (!X || !B || !C || !ws || ((uintptr_t)X & 15) || ((uintptr_t)ws & 255) ||
      ws_bytes < nmf_gemm_split_workspace_bytes(M, N, K))
    return fail(nullptr, NMF_EINVAL, "null pointer, X not 16-byte aligned, or workspace too small / misaligned");
  hipStream_t st = (hipStream_t)hs;
  const int64_t Kpad = round_up(K, 64);
  uint16_t* H = (uint16_t*)ws;
  uint16_t* Lo = H + N * Kpad;
  float* part = (float*)((char*)ws + round_up(2 * N * Kpad * 2, 256));
  hipError_t e = launch_prep_bt(B, ldb, K, N, H, Lo, Kpad, st);
  if (!e) e = launch_gemm_split(X, ldx, at, H, Lo, Kpad, C, ldc, M, N, K, gemm_split_pick_splits(M, N, K), part, st);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

nmf_status nmf_split_prepare_thin(const float* B, int64_t ldb, int64_t K, int64_t N, uint16_t* BtH, uint16_t* BtL,
                                  int64_t ldbt, void* hs) {
  if (K <= 0 || N <= 0 || N > 256 || ldb < N || ldbt % 64 || ldbt < round_up(K, 64) || !B || !BtH || !BtL)
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  const hipError_t e = launch_prep_bt(B, ldb, K, N, BtH, BtL, ldbt, (hipStream_t)hs);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

int32_t nmf_gemm_split_splits(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  return gemm_split_pick_splits(M, N, K);
}

nmf_status nmf_gemm_split_prepared(const float* X, int64_t ldx, int32_t at, const uint16_t* BtH, const uint16_t* BtL,
                                   int64_t ldbt, int64_t K, int64_t N, float* C, int64_t ldc, int64_t M,
                                   int32_t splits, void* hs) {
  if (M < 0 || N <= 0 || N > 256 || K <= 0 || (at != 0 && at != 1) || ldc < N || ldx < (at ? M : K) || ldx % 4 ||
      ldbt % 64 || ldbt < round_up(K, 64) || splits < 1 || splits > 64)
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0) return NMF_OK;
  if (!X || !BtH || !BtL || !C || ((uintptr_t)X & 15)) return fail(nullptr, NMF_EINVAL, "null pointer or X not 16-byte aligned");
  const hipError_t e = launch_gemm_split_kernel(X, ldx, at, BtH, BtL, ldbt, C, ldc, M, N, K, splits, C, (hipStream_t)hs);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

nmf_status nmf_lowp_prepare_thin(int32_t prec, const float* B, int64_t ldb, int64_t K, int64_t N, void* Bt,
                                 int64_t Kpad, int32_t* EB, void* hs) {
  if (N <= 0 || N > 256 || K <= 0 || Kpad < K || Kpad % 128 || ldb < N) return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (!B || !Bt || (prec == NMF_FP8_E4M3 && !EB)) return fail(nullptr, NMF_EINVAL, "null pointer");
  hipError_t e;
  if (prec == NMF_BF16) e = launch_prep_b_bf16(B, ldb, K, N, (uint16_t*)Bt, Kpad, (hipStream_t)hs);
  else if (prec == NMF_FP8_E4M3) e = launch_prep_b_fp8(B, ldb, K, N, EB, (uint8_t*)Bt, Kpad, (hipStream_t)hs);
  else return fail(nullptr, NMF_EINVAL, "prec must be BF16 or FP8_E4M3");
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

int32_t nmf_gemm_lowp_splits(int64_t M, int64_t N, int64_t Kpad) {
  if (M <= 0 || N <= 0 || Kpad <= 0) return 1;
  return gemm_lp_pick_splits(M, N, Kpad, 128);
}

nmf_status nmf_gemm_bf16_at_prepared(const void* A, int64_t lda, int64_t K, const void* Bt, int64_t N, float* C,
                                     int64_t ldc, int64_t M, int64_t Kpad, int32_t splits, void* hs) {
  if (M < 0 || N <= 0 || N > 128 || K < 0 || Kpad < K || Kpad % 128 || lda < M || lda % 8 || splits < 1 ||
      splits > 64 || (splits == 1 && ldc < N))
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0) return NMF_OK;
  if (!A || !Bt || !C || ((uintptr_t)A & 15)) return fail(nullptr, NMF_EINVAL, "null pointer or A not 16-byte aligned");
  const hipError_t e = launch_gemm_bf16_nt((const uint16_t*)A, lda, (const uint16_t*)Bt, Kpad, C, ldc, M, N, Kpad,
                                           splits, C, (hipStream_t)hs, false, 1, K);
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

nmf_status nmf_gemm_lowp_prepared(int32_t prec, const void* A, int64_t lda, const int32_t* EA, int64_t ea_i,
                                  int64_t ea_k, const void* Bt, const int32_t* EB, int64_t N, float* C,
                                  int64_t ldc, int64_t M, int64_t Kpad, int32_t splits, void* hs) {
  if (M < 0 || N <= 0 || N > 256 || Kpad <= 0 || Kpad % 128 || lda < Kpad || splits < 1 || splits > 64 ||
      (splits == 1 && ldc < N))
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (M == 0) return NMF_OK;
  if (!A || !Bt || !C || (prec == NMF_FP8_E4M3 && (!EA || !EB))) return fail(nullptr, NMF_EINVAL, "null pointer");
  hipStream_t st = (hipStream_t)hs;
  hipError_t e;
  // splits > 1: the kernel writes partial z at C + z M N (leading dimension N)
  if (prec == NMF_BF16)
    e = launch_gemm_bf16_nt((const uint16_t*)A, lda, (const uint16_t*)Bt, Kpad, C, ldc, M, N, Kpad, splits, C, st,
                            false);
  else if (prec == NMF_FP8_E4M3)
    e = launch_gemm_fp8_nt((const uint8_t*)A, lda, EA, ea_i, ea_k, (const uint8_t*)Bt, Kpad, EB, C, ldc, M, N, Kpad,
                           splits, C, st, false);
  else
    return fail(nullptr, NMF_EINVAL, "prec must be BF16 or FP8_E4M3");
  return e ? fail(nullptr, NMF_EHIP, hipGetErrorString(e)) : NMF_OK;
}

size_t nmf_orth_workspace_bytes(int64_t rows, int32_t k) {
  const int s = gram_pick_splits(rows, k);
  return ((size_t)s * k * k + 2 * (size_t)k * k) * sizeof(double) + 8 * sizeof(int) + 512;
}

nmf_status nmf_orth(float* Y, int64_t ldy, int64_t rows, int32_t k, void* ws, size_t ws_bytes,
                    void* hs, int32_t* shifted) {
  if (!Y || rows < k || k <= 0 || k > 256 || ldy < k || ldy % 4) return fail(nullptr, NMF_EINVAL, "bad arguments");
  if (!ws || ws_bytes < nmf_orth_workspace_bytes(rows, k) || ((uintptr_t)ws & 255)) return fail(nullptr, NMF_ENOMEM, "workspace too small or misaligned");
  const int s = gram_pick_splits(rows, k);
  char* p = (char*)ws;
  double* gp = (double*)p;
  p += (size_t)s * k * k * sizeof(double);
  double* G = (double*)p;
  p += (size_t)k * k * sizeof(double);
  double* R = (double*)p;
  p += (size_t)k * k * sizeof(double);
  int* status = (int*)p;
  hipStream_t st = (hipStream_t)hs;
  hipError_t e = launch_fill_i32(status, 8, 0, st);
  if (!e) e = orth(Y, ldy, rows, k, gp, G, R, status, st);
  int h[2] = {0, 0};
  if (!e) e = hipMemcpyAsync(h, status, sizeof(h), hipMemcpyDeviceToHost, st);
  if (!e) e = hipStreamSynchronize(st);
  if (e) return fail(nullptr, NMF_EHIP, hipGetErrorString(e));
  if (shifted) *shifted = h[0];
  if (h[1]) return fail(nullptr, NMF_EBREAKDOWN, "Cholesky breakdown even with the shift");
  return NMF_OK;
}

nmf_status nmf_sym_eigvals(const double* A, int64_t lda, int32_t k, double* w, void* hs, int32_t* sweeps) {
  if (!A || !w || k <= 0 || k > 128 || lda < k) return fail(nullptr, NMF_EINVAL, "bad arguments");
  double* ho = take_host_out();
  double* hd = nullptr;
  if (!ho || hipHostGetDevicePointer((void**)&hd, ho, 0) != hipSuccess) {
    give_host_out(ho);
    return fail(nullptr, NMF_ENOMEM, "no pinned result buffer");
  }
  hipStream_t st = (hipStream_t)hs;
  hipError_t e = launch_sym_eig(A, lda, k, 0, w, (int*)hd, st);
  if (!e) e = hipStreamSynchronize(st);
  const int h[2] = {((const int*)ho)[0], ((const int*)ho)[1]};
  give_host_out(ho);
  if (e) return fail(nullptr, NMF_EHIP, hipGetErrorString(e));
  if (sweeps) *sweeps = h[0];
  if (h[1]) return fail(nullptr, NMF_ENONFINITE, "non-finite matrix entry");
  return NMF_OK;
}

size_t nmf_gini_workspace_bytes(int64_t rows, int64_t cols) {
  if (rows < 1 || cols < 1 || rows * cols >= (int64_t)1 << 32) return 0;
  return gini_workspace_bytes(rows, cols);
}

nmf_status nmf_gini(const float* B, int64_t ldb, int64_t rows, int64_t cols, void* ws, size_t ws_bytes, void* hs,
                    double* gini) {
  if (!B || !ws || !gini || rows < 1 || cols < 1 || ldb < cols || rows * cols >= (int64_t)1 << 32 ||
      ((uintptr_t)ws & 255) || ws_bytes < gini_workspace_bytes(rows, cols))
    return fail(nullptr, NMF_EINVAL, "bad arguments");
  double* ho = take_host_out();
  double* hd = nullptr;
  if (!ho || hipHostGetDevicePointer((void**)&hd, ho, 0) != hipSuccess) {
    give_host_out(ho);
    return fail(nullptr, NMF_ENOMEM, "no pinned result buffer");
  }
  hipStream_t st = (hipStream_t)hs;
  hipError_t e = launch_gini(B, ldb, rows, cols, ws, hd, st);
  if (!e) e = hipStreamSynchronize(st);
  const double s1 = ho[0], s2 = ho[1];
  give_host_out(ho);
  if (e) return fail(nullptr, NMF_EHIP, hipGetErrorString(e));
  if (!std::isfinite(s1) || !std::isfinite(s2) || s2 == 0.0)
    return fail(nullptr, NMF_ENONFINITE, "Gini undefined (non-finite entries or a zero sum)");
  *gini = s1 / ((double)(rows * cols) * s2);
  return NMF_OK;
}

}  // extern "C"
