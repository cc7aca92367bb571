"""FP64 oracle of plain and compressed NMF (test infrastructure only).

Notation.  The data matrix X is m x n with rows as datapoints (the paper's d x n,
Sec 2).  W (m x r) is the paper's A, Ht (n x r) is the paper's B, so X ~ W Ht^T
(eq 2.1).  The sketch width is k' = r + r_ov (Sec 3).

  Q_L  (m x k')  the paper's L, orthonormal basis of P(X)      (Sec 3.1, eq 3.5)
  Q_R  (n x k')  the paper's R^T, orthonormal basis of P(X^T)   (Sec 3.1)
  Xh   (n x k')  X^T Q_L, the transpose of X-hat = L^T X        (Sec 4, eq 4_6)
  Xc   (m x k')  X Q_R,   X-check = X R^T                        (Sec 4, eq 4_6)
  Wh   (k' x r)  Q_L^T W, A-hat = L^T A                          (Sec 4)
  Hc   (k' x r)  Q_R^T Ht, B-check = R B                         (Sec 4)

Readings of the paper used here (all listed with reasons in the design notes):
  * eq 3.5 is evaluated as subspace iteration: re-orthonormalise after every
    product with X or X^T (same span in exact arithmetic);
  * one iteration = the whole W (A) sweep, then the whole H (B) sweep, each in
    ascending component order (Gauss-Seidel), with the whole-sweep matrices of
    the sparsity/smoothness subsection (H, G, W, P there);
  * normalisation a_j <- a_j/||a_j|| after the W sweep; mode 1 (default)
    compensates b_j <- b_j * ||a_j|| so that W Ht^T is unchanged, mode 2 is the
    uncompensated literal rule, mode 0 skips it;
  * [.]_+ is max(x, 0); a component whose denominator is not positive is left
    unchanged.
"""
import numpy as np


# ----------------------------------------------------------------------------
# Range finder (Sec 3, eqs 3.4 and 3.5; Sec 3.1)
# ----------------------------------------------------------------------------

def householder_q(Y):
    """Orthonormal basis of range(Y) by LAPACK Householder QR (reduced)."""
    return np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")[0]


class CholeskyBreakdown(Exception):
    pass


def cholesky_qr(Y, shift=0.0):
    """One CholeskyQR pass: G = Y^T Y (+ shift I), G = R^T R, Q = Y R^{-1}."""
    Y = np.asarray(Y, dtype=np.float64)
    G = Y.T @ Y + shift * np.eye(Y.shape[1])
    try:
        L = np.linalg.cholesky(G)
    except np.linalg.LinAlgError as exc:
        raise CholeskyBreakdown(str(exc))
    R = L.T
    return Y @ np.linalg.inv(R), R


def cholesky_qr2(Y, force_shift=False):
    """CholeskyQR2 (two passes); on breakdown, shifted CholeskyQR3.

    The shifted variant (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa,
    SIAM J. Sci. Comput. 2020) adds s = 11 (m k + k(k+1)) u ||Y||^2 to the Gram
    diagonal in the first pass, with ||Y||_F^2 as the bound for ||Y||_2^2, then
    runs CholeskyQR2 on the result.  `force_shift` takes that path directly.
    """
    Y = np.asarray(Y, dtype=np.float64)
    try:
        if force_shift:
            raise CholeskyBreakdown("shift requested")
        Q1, _ = cholesky_qr(Y)
        Q2, _ = cholesky_qr(Q1)
        return Q2, False
    except CholeskyBreakdown:
        m, k = Y.shape
        u = np.finfo(np.float64).eps / 2
        s = 11.0 * (m * k + k * (k + 1)) * u * float(np.sum(Y * Y))
        Q1, _ = cholesky_qr(Y, shift=s)
        Q2, _ = cholesky_qr(Q1)
        Q3, _ = cholesky_qr(Q2)
        return Q3, True


class RowPanels:
    """An FP32 data matrix too large to hold in FP64, used through its products:
    X B is formed panel by panel as float64(X_p) B, and X^T B as the sum over
    the panels, in ascending order, of float64(X_p)^T B_p.  The values are those
    of the whole FP64 products up to the order of the FP64 sums."""

    def __init__(self, X, panel=8192, transform=None):
        self.data = X
        self.shape = X.shape
        self.panel = panel
        self.transform = transform   # applied to each FP32 panel before its product

    def _panel(self, i):
        P = np.asarray(self.data[i:i + self.panel])
        if self.transform is not None:
            P = self.transform(P)
        return np.asarray(P, dtype=np.float64)

    def matmul(self, B):
        B = np.asarray(B, dtype=np.float64)
        out = np.empty((self.shape[0], B.shape[1]))
        for i in range(0, self.shape[0], self.panel):
            out[i:i + self.panel] = self._panel(i) @ B
        return out

    def tmatmul(self, B):
        B = np.asarray(B, dtype=np.float64)
        out = np.zeros((self.shape[1], B.shape[1]))
        for i in range(0, self.shape[0], self.panel):
            out += self._panel(i).T @ B[i:i + self.panel]
        return out

    def _split(self, i):
        """hi, lo of the split-BF16 representation of panel i (FP64 values)."""
        from . import quant
        P = np.asarray(self.data[i:i + self.panel], dtype=np.float32)
        hi = quant.bf16_round_bits(P)
        lo = quant.bf16_round_bits(P - hi)      # P - hi is exact in FP32
        return hi.astype(np.float64), lo.astype(np.float64)

    def split_matmul(self, B):
        """split_product(X, B) panel by panel."""
        Bh, Bl = split_bf16(B)
        out = np.empty((self.shape[0], B.shape[1]))
        for i in range(0, self.shape[0], self.panel):
            hi, lo = self._split(i)
            out[i:i + self.panel] = hi @ Bh + hi @ Bl + lo @ Bh
        return out

    def split_tmatmul(self, B):
        """split_product(X^T, B), the panels' contributions added in ascending order."""
        out = np.zeros((self.shape[1], B.shape[1]))
        for i in range(0, self.shape[0], self.panel):
            hi, lo = self._split(i)
            Bh, Bl = split_bf16(B[i:i + self.panel])
            out += hi.T @ Bh + hi.T @ Bl + lo.T @ Bh
        return out

    def quantised(self, fmt):
        """The data as stored for the low-precision products: quantize_data of
        each panel (the panels are whole 128-row tile rows, so the values are
        those of the whole matrix), formed inside each product rather than held."""
        assert self.panel % 128 == 0
        assert self.transform is None
        return RowPanels(self.data, self.panel, transform=lambda P: quantize_data(P, fmt))


def _subspace_iteration(fwd, adj, Omega, q, orth):
    """Q = orth(fwd(Omega)), then q times Z = orth(adj(Q)), Q = orth(fwd(Z))."""
    Q = orth(fwd(np.asarray(Omega, dtype=np.float64)))
    for _ in range(q):
        Z = orth(adj(Q))
        Q = orth(fwd(Z))
    return Q


def range_finder(X, Omega, q, orth=householder_q):
    """Basis Q of P(X) = (X X^T)^q X Omega (eq 3.5), as subspace iteration.

    X: a x b, Omega: b x k'.  Returns a x k' with orthonormal columns.
    """
    X = np.asarray(X, dtype=np.float64)
    return _subspace_iteration(lambda B: X @ B, lambda B: X.T @ B, Omega, q, orth)


def compress(X, Omega_L, Omega_R, q, orth=householder_q):
    """Two-sided compression of Sec 3.1 and the projected data of Sec 4.

    Q_L from P(X) with Omega_L (n x k'), Q_R from P(X^T) with Omega_R (m x k');
    Xh = X^T Q_L (n x k'), Xc = X Q_R (m x k').  X may be a RowPanels.
    """
    if isinstance(X, RowPanels):
        QL = _subspace_iteration(X.matmul, X.tmatmul, Omega_L, q, orth)
        QR = _subspace_iteration(X.tmatmul, X.matmul, Omega_R, q, orth)
        return QL, QR, X.tmatmul(QL), X.matmul(QR)
    X = np.asarray(X, dtype=np.float64)
    QL = range_finder(X, Omega_L, q, orth)
    QR = range_finder(X.T, Omega_R, q, orth)
    return QL, QR, X.T @ QL, X @ QR


def quantize_thin(B, fmt):
    """Thin operand of a low-precision product as the GPU rounds it: BF16 of the
    FP32 values, or e4m3 with one power-of-two scale per 128-row block."""
    from . import quant
    B32 = np.asarray(B, dtype=np.float32)
    if fmt == "bf16":
        return quant.bf16_round(B32)
    out = np.empty(B32.shape)
    for k0 in range(0, B32.shape[0], 128):
        blk = B32[k0:k0 + 128].astype(np.float64)
        amax = float(np.max(np.abs(blk))) if blk.size else 0.0
        e = 0
        if amax > 0:
            e = int(np.ceil(np.log2(amax / 448.0)))
            while amax > 448.0 * 2.0 ** e:
                e += 1
            while amax <= 448.0 * 2.0 ** (e - 1):
                e -= 1
        out[k0:k0 + 128] = quant.e4m3_round(blk * 2.0 ** -e) * 2.0 ** e
    return out


def quantize_data(X, fmt):
    """Data matrix as stored for the low-precision products (BF16, or e4m3 with
    128 x 128 power-of-two block scales), as FP64 values."""
    from . import quant
    if fmt == "bf16":
        return quant.bf16_round(np.asarray(X, dtype=np.float32))
    return quant.e4m3_block_quantise(np.asarray(X, dtype=np.float32).astype(np.float64))[0]


def split_bf16(A):
    """Two-term BF16 representation of FP32 values (extension): hi = bf16(a),
    lo = bf16(a - hi), both round to nearest even; a - hi is exact in FP32.
    |a - hi - lo| <= 2^-16 |a| for normal values.  Returns (hi, lo) as FP64."""
    from . import quant
    A32 = np.asarray(A, dtype=np.float32)
    hi = quant.bf16_round(A32)
    r = A32.astype(np.float64) - hi            # exact, and representable in FP32
    lo = quant.bf16_round(r.astype(np.float32))
    return hi, lo


def split_product(A, B):
    """Product on split-BF16 operands with the lo*lo term dropped:
    Ah Bh + Ah Bl + Al Bh, summed here in FP64 (the GPU accumulates in FP32).
    Differs from A B by at most about 3 * 2^-16 (|A| |B|) elementwise."""
    Ah, Al = split_bf16(A)
    Bh, Bl = split_bf16(B)
    return Ah @ Bh + Ah @ Bl + Al @ Bh


def compress_lowp(X, Omega_L, Omega_R, q, fmt, refine=False, orth=householder_q, lowp_sketches=False):
    """Model of the low-precision compression: every range-finder product uses
    the quantised X and a quantised thin operand; optionally one power iteration
    per side on X itself, its products exact (refine True or 1, the FP32 pass)
    or split-BF16 (refine 2); the projected data use the exact X (lowp_sketches
    0), the quantised X and quantised bases like the other products (1), or
    split-BF16 products on X (2)."""
    if isinstance(X, RowPanels):   # the same steps with the products over row panels
        Xqp = X.quantised(fmt)
        xq, xqt = (lambda B: Xqp.matmul(B)), (lambda B: Xqp.tmatmul(B))
        x, xt = X.matmul, X.tmatmul
        sx, sxt = X.split_matmul, X.split_tmatmul
    else:
        X = np.asarray(X, dtype=np.float64)
        Xq = quantize_data(X, fmt)
        xq, xqt = (lambda B: Xq @ B), (lambda B: Xq.T @ B)
        x, xt = (lambda B: X @ B), (lambda B: X.T @ B)
        sx, sxt = (lambda B: split_product(X, B)), (lambda B: split_product(X.T, B))

    def prod(side, B):   # side 0: Xq B, side 1: Xq^T B, on the rounded thin operand
        return (xqt if side else xq)(quantize_thin(B, fmt))

    QL = orth(prod(0, Omega_L))
    for _ in range(q):
        Z = orth(prod(1, QL))
        QL = orth(prod(0, Z))
    QR = orth(prod(1, Omega_R))
    for _ in range(q):
        Z = orth(prod(0, QR))
        QR = orth(prod(1, Z))
    if refine == 2:
        QL = orth(sx(orth(sxt(QL))))
        QR = orth(sxt(orth(sx(QR))))
    elif refine:
        QL = orth(x(orth(xt(QL))))
        QR = orth(xt(orth(x(QR))))
    if lowp_sketches == 2:
        return QL, QR, sxt(QL), sx(QR)
    if lowp_sketches:
        return QL, QR, prod(1, QL), prod(0, QR)
    return QL, QR, xt(QL), x(QR)


# ----------------------------------------------------------------------------
# Update rules
# ----------------------------------------------------------------------------

def _normalise(W, Ht, normalize):
    """a_j <- a_j / ||a_j||_2 after the A sweep (end of Sec 4)."""
    if normalize == 0:
        return W, Ht
    s = np.sqrt(np.sum(W * W, axis=0))
    for j in range(W.shape[1]):
        if s[j] > 0:
            W[:, j] = W[:, j] / s[j]
            if normalize == 1:
                Ht[:, j] = Ht[:, j] * s[j]
    return W, Ht


def w_sweep(W, XcHc, GH):
    """A sweep of eq fastHALS_a: a_j <- [a_j + (H_j - A G_j) / G_jj]_+ , j ascending."""
    W = W.copy()
    for j in range(W.shape[1]):
        if GH[j, j] > 0:
            W[:, j] = np.maximum(W[:, j] + (XcHc[:, j] - W @ GH[:, j]) / GH[j, j], 0.0)
    return W


def h_sweep(Ht, XhWh, GW):
    """B sweep of eq fastHALS_a: b_j <- [b_j + (P_j - B W_j) / W_jj]_+ , j ascending."""
    Ht = Ht.copy()
    for j in range(Ht.shape[1]):
        if GW[j, j] > 0:
            Ht[:, j] = np.maximum(Ht[:, j] + (XhWh[:, j] - Ht @ GW[:, j]) / GW[j, j], 0.0)
    return Ht


def h_sweep_constrained(Ht, XhWh, GW, alpha, beta):
    """B sweep with sparsity alpha and smoothness beta (Sec 4.1, FastHALS-RP form):

    b_j <- [(b_j W_jj + P_j - B W_j - alpha 1) / (W_jj + beta)]_+
    (the stray transpose on a-hat_j in the printed middle expression is read as
    the matrix-vector product B A-hat^T a-hat_j; 1 has length n).
    """
    Ht = Ht.copy()
    for j in range(Ht.shape[1]):
        den = GW[j, j] + beta
        if den > 0:
            num = Ht[:, j] * GW[j, j] + XhWh[:, j] - Ht @ GW[:, j] - alpha
            Ht[:, j] = np.maximum(num / den, 0.0)
    return Ht


def fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize=1, alpha=0.0, beta=0.0):
    """One FastHALS-RP iteration (eq fastHALS_a; matrices as in Sec 4.1).

    Hc = Q_R^T Ht (B-check), G_H = Hc^T Hc, Xc Hc (X-check B-check); W sweep;
    normalise; Wh = Q_L^T W (A-hat), G_W = Wh^T Wh, Xh Wh (X-hat^T A-hat); H sweep.
    """
    W = np.array(W, dtype=np.float64)
    Ht = np.array(Ht, dtype=np.float64)
    Hc = QR.T @ Ht
    GH = Hc.T @ Hc
    W = w_sweep(W, Xc @ Hc, GH)
    W, Ht = _normalise(W, Ht, normalize)
    Wh = QL.T @ W
    GW = Wh.T @ Wh
    if alpha == 0.0 and beta == 0.0:
        Ht = h_sweep(Ht, Xh @ Wh, GW)
    else:
        Ht = h_sweep_constrained(Ht, Xh @ Wh, GW, alpha, beta)
    return W, Ht


def fasthals_iteration(X, W, Ht, normalize=1):
    """Plain (uncompressed) FastHALS iteration (Sec 2.2): the same sweeps with
    X B and B^T B for the A side and X^T A and A^T A for the B side."""
    X = np.asarray(X, dtype=np.float64)
    W = np.array(W, dtype=np.float64)
    Ht = np.array(Ht, dtype=np.float64)
    W = w_sweep(W, X @ Ht, Ht.T @ Ht)
    W, Ht = _normalise(W, Ht, normalize)
    Ht = h_sweep(Ht, X.T @ W, W.T @ W)
    return W, Ht


def hals_rp_naive_iteration(W, Ht, Xh, Xc, QL, QR, normalize=1):
    """HALS-RP written with the explicit component residuals of eq 4_6 and the
    closed-form minimisers of eq hals_update (brute force, tiny inputs only):

      X-check_j = X-check - A B-check^T + a_j b-check_j^T,
      a_j <- [X-check_j b-check_j / (b-check_j^T b-check_j)]_+ ;
      X-hat_j  = X-hat - A-hat B^T + a-hat_j b_j^T,
      b_j <- [X-hat_j^T a-hat_j / (a-hat_j^T a-hat_j)]_+ .
    """
    W = np.array(W, dtype=np.float64)
    Ht = np.array(Ht, dtype=np.float64)
    r = W.shape[1]
    Hc = QR.T @ Ht
    for j in range(r):
        d = Hc[:, j] @ Hc[:, j]
        if d > 0:
            Xc_j = Xc - W @ Hc.T + np.outer(W[:, j], Hc[:, j])
            W[:, j] = np.maximum(Xc_j @ Hc[:, j] / d, 0.0)
    W, Ht = _normalise(W, Ht, normalize)
    Xhat = Xh.T                      # k' x n
    Wh = QL.T @ W
    for j in range(r):
        d = Wh[:, j] @ Wh[:, j]
        if d > 0:
            Xhat_j = Xhat - Wh @ Ht.T + np.outer(Wh[:, j], Ht[:, j])
            Ht[:, j] = np.maximum(Xhat_j.T @ Wh[:, j] / d, 0.0)
    return W, Ht


def column_nnls(Xh_rows, Wh, sweeps, Ht0=None):
    """min_{h >= 0} ||x-hat - Wh h||^2 for every row x-hat of Xh_rows (n x k'),
    by repeated B sweeps with Wh fixed (the B half of eq fastHALS_a)."""
    Xh_rows = np.asarray(Xh_rows, dtype=np.float64)
    Wh = np.asarray(Wh, dtype=np.float64)
    r = Wh.shape[1]
    Ht = np.zeros((Xh_rows.shape[0], r)) if Ht0 is None else np.array(Ht0, dtype=np.float64)
    GW = Wh.T @ Wh
    P = Xh_rows @ Wh
    for _ in range(sweeps):
        Ht = h_sweep(Ht, P, GW)
    return Ht


# ----------------------------------------------------------------------------
# Objective, residuals, metrics
# ----------------------------------------------------------------------------

def frob_sq_diff(X, W, Ht, block=4096):
    """sum (X - W Ht^T)^2 and sum X^2, directly, in FP64, row blocks."""
    X = X.data if isinstance(X, RowPanels) else np.asarray(X)
    W = np.asarray(W, dtype=np.float64)
    Ht = np.asarray(Ht, dtype=np.float64)
    res = 0.0
    nx = 0.0
    for i in range(0, X.shape[0], block):
        Xb = np.asarray(X[i:i + block], dtype=np.float64)
        D = Xb - W[i:i + block] @ Ht.T
        res += float(np.sum(D * D))
        nx += float(np.sum(Xb * Xb))
    return res, nx


def rel_error(X, W, Ht):
    """e = ||X - W Ht^T||_F / ||X||_F (eq 2.2 as a relative error)."""
    res, nx = frob_sq_diff(X, W, Ht)
    return np.sqrt(res) / np.sqrt(nx)


def objective(X, W, Ht):
    """J = 1/2 ||X - W Ht^T||_F^2 (eq 2.2)."""
    return 0.5 * frob_sq_diff(X, W, Ht)[0]


def proxy_rel_error(normX2, Xh, Wh, Ht):
    """Sketch-only estimate of e: ||X||^2 - ||X-hat||^2 + ||X-hat - A-hat B^T||^2,
    exact when the columns of W lie in range(Q_L)."""
    nxh = float(np.sum(Xh * Xh))
    comp = float(np.sum((Xh - Ht @ Wh.T) ** 2))
    return np.sqrt(max(normX2 - nxh + comp, 0.0) / normX2)


def gini(B):
    """Gini sparsity coefficient of Sec 5.1 over all n*k entries sorted ascending:
    G = sum_i (2i - N - 1) b_i / (N sum_i b_i), i = 1..N."""
    b = np.sort(np.asarray(B, dtype=np.float64).reshape(-1))
    N = b.size
    i = np.arange(1, N + 1, dtype=np.float64)
    return float(np.sum((2 * i - N - 1) * b) / (N * np.sum(b)))


# ----------------------------------------------------------------------------
# Whole runs
# ----------------------------------------------------------------------------

def fasthals_rp(X, Omega_L, Omega_R, q, W0, H0t, iters, normalize=1, orth=householder_q,
                record=False, fmt=None, refine=False, alpha=0.0, beta=0.0, lowp_sketches=False):
    """Compress (exactly, or with the low-precision model when fmt is 'bf16' or
    'fp8'), then `iters` FastHALS-RP iterations.  Returns a dict."""
    if fmt is None:
        QL, QR, Xh, Xc = compress(X, Omega_L, Omega_R, q, orth)
    else:
        QL, QR, Xh, Xc = compress_lowp(X, Omega_L, Omega_R, q, fmt, refine, orth, lowp_sketches)
    W = np.array(W0, dtype=np.float64)
    Ht = np.array(H0t, dtype=np.float64)
    hist = []
    for _ in range(iters):
        W, Ht = fasthals_rp_iteration(W, Ht, Xh, Xc, QL, QR, normalize, alpha, beta)
        if record:
            hist.append(rel_error(X, W, Ht))
    return dict(QL=QL, QR=QR, Xh=Xh, Xc=Xc, W=W, Ht=Ht, e=rel_error(X, W, Ht), hist=hist)


def fasthals(X, W0, H0t, iters, normalize=1):
    W = np.array(W0, dtype=np.float64)
    Ht = np.array(H0t, dtype=np.float64)
    for _ in range(iters):
        W, Ht = fasthals_iteration(X, W, Ht, normalize)
    return W, Ht


def complexity_memory(d, n, k, kp):
    """Table 4.1 memory formulas in floats: non-RP d n + d k + n k and
    RP (2 k' + k)(d + n)."""
    return d * n + d * k + n * k, (2 * kp + k) * (d + n)
