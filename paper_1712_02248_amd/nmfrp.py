"""Thin ctypes binding of libnmfrp.so (declared in include/nmfrp.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  torch supplies device memory (workspace, inputs, outputs) and the
current HIP stream.  There is no CPU fallback: if the library is not built, or
the tensors are not on the GPU, the calls raise.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnmfrp.so")

NMF_FP32, NMF_BF16, NMF_FP8_E4M3 = 0, 1, 2
STATUS = {0: "NMF_OK", -1: "NMF_EINVAL", -2: "NMF_ENOMEM", -3: "NMF_EHIP", -4: "NMF_ESTATE",
          -5: "NMF_EBREAKDOWN", -6: "NMF_ENONFINITE"}

c_i64, c_i32, c_u32, c_u64, c_sz, c_vp = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p)
c_dbl_p = ctypes.POINTER(ctypes.c_double)
c_i32_p = ctypes.POINTER(ctypes.c_int32)


class Params(ctypes.Structure):
    _fields_ = [("m", c_i64), ("n", c_i64), ("r", c_i32), ("k_sketch", c_i32), ("q", c_i32),
                ("prec", c_i32), ("refine_fp32", c_i32), ("normalize", c_i32),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float), ("seed", c_u64),
                ("lowp_sketches", c_i32), ("update_prec", c_i32)]


# name -> (restype, argtypes)
_SIGS = {
    "nmf_workspace_bytes": (c_sz, [ctypes.POINTER(Params)]),
    "nmf_create": (c_i32, [ctypes.POINTER(Params), c_vp, c_sz, c_vp, ctypes.POINTER(c_vp)]),
    "nmf_destroy": (None, [c_vp]),
    "nmf_last_error": (ctypes.c_char_p, [c_vp]),
    "nmf_validate": (c_i32, [c_vp, c_vp, c_i64]),
    "nmf_compress": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp]),
    "nmf_init": (c_i32, [c_vp, c_vp, c_vp, ctypes.c_float]),
    "nmf_step": (c_i32, [c_vp, c_i32]),
    "nmf_fasthals_step": (c_i32, [c_vp, c_vp, c_i64, c_i32]),
    "nmf_residual": (c_i32, [c_vp, c_vp, c_i64, c_dbl_p]),
    "nmf_residual_check": (c_i32, [c_vp, c_vp, c_i64, ctypes.c_double, c_dbl_p, c_dbl_p, c_i32_p]),
    "nmf_proxy_residual": (c_i32, [c_vp, c_dbl_p]),
    "nmf_sketch_spectrum": (c_i32, [c_vp, c_dbl_p]),
    "nmf_fit": (c_i32, [c_vp, c_vp, c_i64, c_i32, ctypes.c_double, c_i32, c_i32_p, c_dbl_p]),
    "nmf_get_factors": (c_i32, [c_vp, c_vp, c_vp]),
    "nmf_get_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "nmf_set_state": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "nmf_sync": (c_i32, [c_vp, c_i32_p]),
    "nmf_stage_times": (c_i32, [c_vp, c_dbl_p, c_dbl_p, c_dbl_p]),
    "nmf_gaussian": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_u32, c_u64, c_vp]),
    "nmf_uniform": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_u32, c_u64, ctypes.c_float, c_vp]),
    "nmf_gemm_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64, c_i32]),
    "nmf_gemm": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_i64, c_vp,
                         c_sz, c_vp]),
    "nmf_gemm_noalloc": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_i64, c_vp]),
    "nmf_quantize_x": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_i32, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "nmf_gemm_lowp_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64]),
    "nmf_gemm_lowp": (c_i32, [c_i32, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64,
                              c_i64, c_i64, c_vp, c_sz, c_vp]),
    "nmf_lowp_prepare_thin": (c_i32, [c_i32, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "nmf_gemm_lowp_splits": (c_i32, [c_i64, c_i64, c_i64]),
    "nmf_gemm_lowp_prepared": (c_i32, [c_i32, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_i64,
                                       c_i64, c_i64, c_i32, c_vp]),
    "nmf_gemm_bf16_at_prepared": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_i32, c_vp]),
    "nmf_gemm_split_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64]),
    "nmf_gemm_split": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp, c_sz, c_vp]),
    "nmf_split_prepare_thin": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp]),
    "nmf_gemm_split_splits": (c_i32, [c_i64, c_i64, c_i64]),
    "nmf_gemm_split_prepared": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64,
                                        c_i32, c_vp]),
    "nmf_orth_workspace_bytes": (c_sz, [c_i64, c_i32]),
    "nmf_orth": (c_i32, [c_vp, c_i64, c_i64, c_i32, c_vp, c_sz, c_vp, c_i32_p]),
    "nmf_sym_eigvals": (c_i32, [c_vp, c_i64, c_i32, c_vp, c_vp, c_i32_p]),
    "nmf_gini_workspace_bytes": (c_sz, [c_i64, c_i64]),
    "nmf_gini": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_vp, c_sz, c_vp, c_dbl_p]),
    "nmf_mlp_n_params": (c_i64, [c_i32, c_i32, c_i32]),
    "nmf_mlp_workspace_bytes": (c_sz, [c_i32, c_i32, c_i32, c_i32]),
    "nmf_mlp_create": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_vp, c_vp, c_sz, c_vp, ctypes.POINTER(c_vp)]),
    "nmf_mlp_destroy": (None, [c_vp]),
    "nmf_mlp_last_error": (ctypes.c_char_p, [c_vp]),
    "nmf_mlp_get_params": (c_i32, [c_vp, c_vp]),
    "nmf_mlp_set_params": (c_i32, [c_vp, c_vp]),
    "nmf_mlp_loss_grad": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i64, c_i32, c_dbl_p, c_vp]),
    "nmf_mlp_train": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_i32, c_i32, ctypes.c_float,
                              c_dbl_p]),
    "nmf_mlp_infer": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_i64]),
    "nmf_nnls_rows": (c_i32, [c_vp, c_i64, c_i64, c_i32, c_vp, c_i32, c_i32, c_i32, c_vp, c_i64, c_vp]),
    "nmf_init_learned": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_float, c_i32,
                                 ctypes.POINTER(c_i64)]),
    "nmf_init_learned_ref": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, ctypes.c_float, c_i32,
                                     ctypes.POINTER(c_i64)]),
}

_lib = None


def load(path=LIB_PATH):
    """Loads the library (once) and declares every exported signature."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run python -m paper_1712_02248_amd.build")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class NmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status, ctx=None):
    if status != 0:
        msg = load().nmf_last_error(ctx)
        raise NmfError(status, msg.decode() if msg else "")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _f32(t, shape, name):
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous float32 device tensor of shape {shape}")
    return t


class NMF:
    """Context over a torch-allocated workspace.

    X (m x n) stays a borrowed torch tensor; W (m x r) and Ht (n x r) are the
    paper's A and B.
    """

    def __init__(self, m, n, r, k_sketch, q, seed=0, normalize=1, alpha=0.0, beta=0.0,
                 prec=NMF_FP32, refine_fp32=0, lowp_sketches=0, update_prec=0, device="cuda", stream=None):
        lib = load()
        self.p = Params(m, n, r, k_sketch, q, prec, refine_fp32, normalize, alpha, beta, seed,
                        lowp_sketches, update_prec)
        nbytes = lib.nmf_workspace_bytes(ctypes.byref(self.p))
        if nbytes == 0:
            _check(-1)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        self._wsptr = (base + 255) // 256 * 256
        self.stream = stream
        h = c_vp()
        _check(lib.nmf_create(ctypes.byref(self.p), self._wsptr, nbytes, _stream(stream), ctypes.byref(h)))
        self.h = h
        self.m, self.n, self.r, self.kp = m, n, r, k_sketch

    def close(self):
        if getattr(self, "h", None):
            load().nmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, status):
        _check(status, self.h)

    def validate(self, X):
        self._c(load().nmf_validate(self.h, _ptr(X), X.stride(0)))

    def compress(self, X, omega_L=None, omega_R=None):
        _f32(omega_L, (self.n, self.kp), "omega_L")
        _f32(omega_R, (self.m, self.kp), "omega_R")
        if X.dtype != torch.float32 or X.stride(1) != 1:
            raise ValueError("X: float32, unit column stride")
        self._c(load().nmf_compress(self.h, _ptr(X), X.stride(0), _ptr(omega_L), _ptr(omega_R)))

    def init(self, W0=None, Ht0=None, init_scale=1.0):
        _f32(W0, (self.m, self.r), "W0")
        _f32(Ht0, (self.n, self.r), "Ht0")
        self._c(load().nmf_init(self.h, _ptr(W0), _ptr(Ht0), float(init_scale)))

    def step(self, iters=1):
        self._c(load().nmf_step(self.h, int(iters)))

    def fasthals_step(self, X, iters=1):
        """Uncompressed FastHALS iterations (Sec 2.2) on X from the current factors."""
        if X.dtype != torch.float32 or X.stride(1) != 1:
            raise ValueError("X: float32, unit column stride")
        self._c(load().nmf_fasthals_step(self.h, _ptr(X), X.stride(0), int(iters)))

    def residual(self, X):
        e = ctypes.c_double()
        self._c(load().nmf_residual(self.h, _ptr(X), X.stride(0), ctypes.byref(e)))
        return e.value

    def residual_check(self, X, eps):
        """(e, bound, exact): e from FP32 products within `bound` of the exact
        value, or the exact value (exact = True, bound 0) when the FP32 one lies
        within its bound of eps."""
        e, b, x = ctypes.c_double(), ctypes.c_double(), c_i32()
        self._c(load().nmf_residual_check(self.h, _ptr(X), X.stride(0), float(eps), ctypes.byref(e),
                                          ctypes.byref(b), ctypes.byref(x)))
        return e.value, b.value, bool(x.value)

    def proxy_residual(self):
        """Sketch-only estimate of the relative error (see nmf_proxy_residual)."""
        e = ctypes.c_double()
        self._c(load().nmf_proxy_residual(self.h, ctypes.byref(e)))
        return e.value

    def sketch_spectrum(self):
        """Singular values of X-hat = Q_L^T X, descending (see nmf_sketch_spectrum)."""
        sig = (ctypes.c_double * self.kp)()
        self._c(load().nmf_sketch_spectrum(self.h, sig))
        return torch.tensor(sig[:], dtype=torch.float64)

    def fit(self, X, max_iters, eps=0.0, check_every=10):
        it = c_i32()
        e = ctypes.c_double()
        self._c(load().nmf_fit(self.h, _ptr(X), X.stride(0), int(max_iters), float(eps), int(check_every),
                               ctypes.byref(it), ctypes.byref(e)))
        return it.value, e.value

    def factors(self):
        W = torch.empty(self.m, self.r, dtype=torch.float32, device=self.ws.device)
        Ht = torch.empty(self.n, self.r, dtype=torch.float32, device=self.ws.device)
        self._c(load().nmf_get_factors(self.h, _ptr(W), _ptr(Ht)))
        return W, Ht

    def state(self):
        dev = self.ws.device
        QL = torch.empty(self.m, self.kp, dtype=torch.float32, device=dev)
        QR = torch.empty(self.n, self.kp, dtype=torch.float32, device=dev)
        Xh = torch.empty(self.n, self.kp, dtype=torch.float32, device=dev)
        Xc = torch.empty(self.m, self.kp, dtype=torch.float32, device=dev)
        self._c(load().nmf_get_state(self.h, _ptr(QL), _ptr(QR), _ptr(Xh), _ptr(Xc)))
        return QL, QR, Xh, Xc

    def left_basis(self, out=None):
        """Q_L (m x k') of the last compression, copied to a device tensor."""
        if out is None:
            out = torch.empty(self.m, self.kp, dtype=torch.float32, device=self.ws.device)
        _f32(out, (self.m, self.kp), "QL")
        self._c(load().nmf_get_state(self.h, _ptr(out), None, None, None))
        return out

    def set_state(self, QL, QR, Xh, Xc):
        _f32(QL, (self.m, self.kp), "QL")
        _f32(QR, (self.n, self.kp), "QR")
        _f32(Xh, (self.n, self.kp), "Xh")
        _f32(Xc, (self.m, self.kp), "Xc")
        self._c(load().nmf_set_state(self.h, _ptr(QL), _ptr(QR), _ptr(Xh), _ptr(Xc)))

    def init_learned(self, net, Wh_ref, align_M=None, W0=None, Ht_cold=None, init_scale=1.0, refine_sweeps=0,
                     count=True):
        """Warm start of H from `net` (an Mlp) with per-row rejection against
        Wh_ref (k' x r); returns the number of cold rows kept (None if count
        is False, in which case the call does not synchronise).  net=None: the
        same initialisation without a network (cold rows, then the sweeps)."""
        _f32(Wh_ref, (self.kp, self.r), "Wh_ref")
        _f32(align_M, (self.kp, self.kp), "align_M")
        _f32(W0, (self.m, self.r), "W0")
        _f32(Ht_cold, (self.n, self.r), "Ht_cold")
        nrej = ctypes.c_int64(-1)
        self._c(load().nmf_init_learned(self.h, net.h if net is not None else None, _ptr(align_M), _ptr(Wh_ref),
                                        _ptr(W0), _ptr(Ht_cold),
                                        float(init_scale), int(refine_sweeps),
                                        ctypes.byref(nrej) if count else None))
        return nrej.value if count else None

    def init_learned_ref(self, net, Q_train, W_ref, Ht_cold=None, init_scale=1.0, refine_sweeps=0, count=True):
        """Warm start from the reference fit (Q_train m x k', W_ref m x r): the
        library forms Q_train^T Q_L and Q_L^T W_ref itself; W = W_ref."""
        if Q_train.dtype != torch.float32 or Q_train.shape != (self.m, self.kp) or Q_train.stride(1) != 1:
            raise ValueError("Q_train: float32 m x k' with unit column stride")
        if W_ref.dtype != torch.float32 or W_ref.shape != (self.m, self.r) or W_ref.stride(1) != 1:
            raise ValueError("W_ref: float32 m x r with unit column stride")
        _f32(Ht_cold, (self.n, self.r), "Ht_cold")
        nrej = ctypes.c_int64(-1)
        self._c(load().nmf_init_learned_ref(self.h, net.h if net is not None else None, _ptr(Q_train),
                                            Q_train.stride(0), _ptr(W_ref),
                                            W_ref.stride(0), _ptr(Ht_cold), float(init_scale), int(refine_sweeps),
                                            ctypes.byref(nrej) if count else None))
        return nrej.value if count else None

    def sync(self):
        s = c_i32()
        self._c(load().nmf_sync(self.h, ctypes.byref(s)))
        return s.value

    def stage_times(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._c(load().nmf_stage_times(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(compress_ms=a.value, step_ms=b.value, residual_ms=c.value)


def gaussian(rows, cols, stream_id, seed, device="cuda", stream=None):
    out = torch.empty(rows, cols, dtype=torch.float32, device=device)
    _check(load().nmf_gaussian(_ptr(out), rows, cols, cols, stream_id, seed, _stream(stream)))
    return out


def uniform(rows, cols, stream_id, seed, scale=1.0, device="cuda", stream=None):
    out = torch.empty(rows, cols, dtype=torch.float32, device=device)
    _check(load().nmf_uniform(_ptr(out), rows, cols, cols, stream_id, seed, float(scale), _stream(stream)))
    return out


def gemm(A, B, a_trans=False, out=None, stream=None):
    """C = A @ B (a_trans=False) or A.T @ B (a_trans=True), FP32 MFMA."""
    lib = load()
    if a_trans:
        K, M = A.shape
    else:
        M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty(M, N, dtype=torch.float32, device=A.device)
    nb = lib.nmf_gemm_workspace_bytes(M, N, K, int(a_trans))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=A.device)
    _check(lib.nmf_gemm(_ptr(A), A.stride(0), int(a_trans), _ptr(B), B.stride(0), _ptr(out), out.stride(0),
                        M, N, K, _ptr(ws), ws.numel(), _stream(stream)))
    return out


def gemm_noalloc(A, B, a_trans=False, out=None, stream=None):
    """gemm() through the allocation-free entry point (split-K partials in the
    library's static per-GPU scratch; no workspace)."""
    lib = load()
    if a_trans:
        K, M = A.shape
    else:
        M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty(M, N, dtype=torch.float32, device=A.device)
    _check(lib.nmf_gemm_noalloc(_ptr(A), A.stride(0), int(a_trans), _ptr(B), B.stride(0), _ptr(out), out.stride(0),
                                M, N, K, _stream(stream)))
    return out


def gemm_split(X, at, B, stream=None):
    """op(X) B on split-BF16 operands (X FP32 contiguous rows, at = 1 for X^T B);
    returns C as a new FP32 device tensor."""
    lib = load()
    if X.dtype != torch.float32 or B.dtype != torch.float32 or X.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("X and B must be FP32 with unit column stride")
    rows, cols = X.shape
    M, K = (cols, rows) if at else (rows, cols)
    if B.shape[0] != K:
        raise ValueError("B must have op(X)'s inner dimension rows")
    N = B.shape[1]
    C = torch.empty((M, N), dtype=torch.float32, device=X.device)
    nb = lib.nmf_gemm_split_workspace_bytes(M, N, K)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=X.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    _check(lib.nmf_gemm_split(_ptr(X), X.stride(0), int(at), _ptr(B), B.stride(0), K, N, _ptr(C), C.stride(0), M,
                              base, nb, _stream(stream)))
    return C


class SplitProduct:
    """op(X) B on split-BF16 operands with the thin operand B (K x N) split once;
    run() launches only the product kernel (split-K partials, if any, land in
    self.part and are summed by result(), in ascending order)."""

    def __init__(self, X, at, B, stream=None):
        lib = load()
        if X.dtype != torch.float32 or B.dtype != torch.float32 or X.stride(1) != 1 or B.stride(1) != 1:
            raise ValueError("X and B must be FP32 with unit column stride")
        rows, cols = X.shape
        self.M, self.K = (cols, rows) if at else (rows, cols)
        if B.shape[0] != self.K:
            raise ValueError("B must have op(X)'s inner dimension rows")
        self.X, self.at, self.stream, self.N = X, int(at), stream, B.shape[1]
        self.ldbt = -(-self.K // 64) * 64
        self.Bh = torch.zeros(self.N, self.ldbt, dtype=torch.int16, device=X.device)
        self.Bl = torch.zeros(self.N, self.ldbt, dtype=torch.int16, device=X.device)
        _check(lib.nmf_split_prepare_thin(_ptr(B), B.stride(0), self.K, self.N, _ptr(self.Bh), _ptr(self.Bl),
                                          self.ldbt, _stream(stream)))
        self.splits = int(lib.nmf_gemm_split_splits(self.M, self.N, self.K))
        self.part = torch.empty(self.splits, self.M, self.N, dtype=torch.float32, device=X.device)

    def run(self):
        _check(load().nmf_gemm_split_prepared(_ptr(self.X), self.X.stride(0), self.at, _ptr(self.Bh), _ptr(self.Bl),
                                              self.ldbt, self.K, self.N, _ptr(self.part), self.N, self.M,
                                              self.splits, _stream(self.stream)))

    def result(self):
        out = self.part[0].clone()
        for z in range(1, self.splits):
            out += self.part[z]
        return out


def orth(Y, stream=None):
    """In-place CholeskyQR2 of Y (rows x k); returns the shifted flag."""
    lib = load()
    rows, k = Y.shape
    nb = lib.nmf_orth_workspace_bytes(rows, k)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=Y.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    sh = c_i32()
    _check(lib.nmf_orth(_ptr(Y), Y.stride(0), rows, k, base, nb, _stream(stream), ctypes.byref(sh)))
    return sh.value


def sym_eigvals(A, stream=None):
    """Eigenvalues (descending) of the symmetric FP64 device matrix A (k x k, lower
    triangle read); returns (device tensor of k values, Jacobi sweeps)."""
    lib = load()
    k = A.shape[0]
    if A.dtype != torch.float64 or A.dim() != 2 or A.shape[1] != k or A.stride(1) != 1:
        raise ValueError("A must be a row-major square float64 tensor")
    w = torch.empty(k, dtype=torch.float64, device=A.device)
    sw = c_i32()
    _check(lib.nmf_sym_eigvals(_ptr(A), A.stride(0), k, _ptr(w), _stream(stream), ctypes.byref(sw)))
    return w, sw.value


def gini(B, stream=None):
    """Gini coefficient (Sec 5.1) of the float32 device matrix B (rows x cols,
    row-major, unit column stride), sorted on the device; returns a float."""
    lib = load()
    if B.dtype != torch.float32 or B.dim() != 2 or not B.is_cuda or B.stride(1) != 1:
        raise ValueError("B must be a row-major float32 device matrix")
    rows, cols = B.shape
    nb = lib.nmf_gini_workspace_bytes(rows, cols)
    if nb == 0:
        _check(-1)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=B.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    g = ctypes.c_double()
    _check(lib.nmf_gini(_ptr(B), B.stride(0), rows, cols, base, nb, _stream(stream), ctypes.byref(g)))
    return g.value


def quantize_x(X, prec, stream=None):
    """Low-precision copies of X: returns (Xq, XqT, tile_exp or None) as raw device
    tensors (uint16 BF16 patterns or uint8 e4m3 codes), ld padded to 128."""
    lib = load()
    m, n = X.shape
    ldq, ldqt = -(-n // 128) * 128, -(-m // 128) * 128
    dt = torch.int16 if prec == NMF_BF16 else torch.uint8
    Xq = torch.empty(m, ldq, dtype=dt, device=X.device)
    XqT = torch.empty(n, ldqt, dtype=dt, device=X.device)
    E = torch.empty(-(-m // 128), -(-n // 128), dtype=torch.int32, device=X.device) if prec == NMF_FP8_E4M3 else None
    _check(lib.nmf_quantize_x(_ptr(X), X.stride(0), m, n, prec, _ptr(Xq), ldq, _ptr(XqT), ldqt, _ptr(E),
                              _stream(stream)))
    return Xq, XqT, E


def gemm_lowp(prec, A, K, B, E=None, ea=(0, 0), stream=None):
    """C = A[:, :K] @ B with A a low-precision copy (K-contiguous rows, ld % 128 == 0)."""
    lib = load()
    M, Kpad = A.shape
    N = B.shape[1]
    C = torch.empty(M, N, dtype=torch.float32, device=A.device)
    nb = lib.nmf_gemm_lowp_workspace_bytes(M, N, Kpad)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=A.device)
    base = (ws.data_ptr() + 255) // 256 * 256
    _check(lib.nmf_gemm_lowp(prec, _ptr(A), A.stride(0), _ptr(E), ea[0], ea[1], _ptr(B), B.stride(0), K, N,
                             _ptr(C), C.stride(0), M, Kpad, base, nb, _stream(stream)))
    return C


def mlp_n_params(k_in, hidden, r_out):
    return int(load().nmf_mlp_n_params(k_in, hidden, r_out))


class Mlp:
    """Warm-start network k_in -> hidden -> hidden -> r_out over a torch-allocated
    workspace; parameters are one flat float32 device vector (W1, b1, W2, b2,
    W3, b3, weights [fan_in][fan_out])."""

    def __init__(self, k_in, hidden, r_out, params, max_batch=4096, device="cuda", stream=None):
        lib = load()
        self.k, self.hdim, self.r, self.max_batch = k_in, hidden, r_out, max_batch
        self.np = mlp_n_params(k_in, hidden, r_out)
        _f32(params, (self.np,), "params")
        nbytes = lib.nmf_mlp_workspace_bytes(k_in, hidden, r_out, max_batch)
        if nbytes == 0:
            raise ValueError("invalid MLP sizes")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self._wsptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = stream
        h = c_vp()
        st = lib.nmf_mlp_create(k_in, hidden, r_out, max_batch, _ptr(params), self._wsptr, nbytes,
                                _stream(stream), ctypes.byref(h))
        if st != 0:
            msg = lib.nmf_mlp_last_error(None)
            raise NmfError(st, msg.decode() if msg else "")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().nmf_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, status):
        if status != 0:
            msg = load().nmf_mlp_last_error(self.h)
            raise NmfError(status, msg.decode() if msg else "")

    def params(self):
        out = torch.empty(self.np, dtype=torch.float32, device=self.ws.device)
        self._c(load().nmf_mlp_get_params(self.h, _ptr(out)))
        return out

    def set_params(self, flat):
        _f32(flat, (self.np,), "params")
        self._c(load().nmf_mlp_set_params(self.h, _ptr(flat)))

    def loss_grad(self, X, T):
        B = X.shape[0]
        if X.shape[1] != self.k or T.shape != (B, self.r):
            raise ValueError("shape mismatch")
        g = torch.empty(self.np, dtype=torch.float32, device=self.ws.device)
        L = ctypes.c_double()
        self._c(load().nmf_mlp_loss_grad(self.h, _ptr(X), X.stride(0), _ptr(T), T.stride(0), B,
                                         ctypes.byref(L), _ptr(g)))
        return L.value, g

    def train(self, X, T, epochs, batch, lr, order=None, report=True):
        """Adam passes over the pairs (X rows, T rows); order: int32 device
        tensor (epochs x npairs) of per-pass permutations or None.  Returns the
        mean batch loss per pass (None if report is False: asynchronous)."""
        npairs = X.shape[0]
        if X.shape[1] != self.k or T.shape != (npairs, self.r):
            raise ValueError("shape mismatch")
        if order is not None and (order.dtype != torch.int32 or order.numel() != epochs * npairs
                                  or not order.is_contiguous()):
            raise ValueError("order: contiguous int32, epochs x npairs")
        hist = (ctypes.c_double * max(epochs, 1))()
        self._c(load().nmf_mlp_train(self.h, _ptr(X), X.stride(0), _ptr(T), T.stride(0), npairs, _ptr(order),
                                     int(epochs), int(batch), float(lr), hist if report else None))
        return list(hist)[:epochs] if report else None

    def infer(self, X, out=None):
        rows = X.shape[0]
        if out is None:
            out = torch.empty(rows, self.r, dtype=torch.float32, device=X.device)
        self._c(load().nmf_mlp_infer(self.h, _ptr(X), X.stride(0), rows, _ptr(out), out.stride(0)))
        return out


def nnls_rows(Xr, Wh, sweeps, out=None, warm=False, stream=None):
    """Rows h = argmin_{h>=0} ||x - Wh h|| by `sweeps` H sweeps from h = 0, or
    from the rows already in `out` when warm."""
    rows, k = Xr.shape
    k2, r = Wh.shape
    if k2 != k or not Wh.is_contiguous():
        raise ValueError("Wh: contiguous k x r")
    if out is None:
        if warm:
            raise ValueError("warm start needs the starting rows in out")
        out = torch.empty(rows, r, dtype=torch.float32, device=Xr.device)
    _check(load().nmf_nnls_rows(_ptr(Xr), Xr.stride(0), rows, k, _ptr(Wh), r, int(sweeps), int(bool(warm)),
                                _ptr(out), out.stride(0), _stream(stream)))
    return out


class LowpProduct:
    """C = A[:, :K] @ B with the thin operand B (K x N) prepared once; A is a
    low-precision copy from quantize_x.  run() launches only the product kernel
    (split-K partials, if any, land in self.part and are summed by result())."""

    def __init__(self, prec, A, K, B, E=None, ea=(0, 0), stream=None, at=False, Kpad=None, M=None):
        """at=True (BF16): A is the row-major copy itself, C = A[:K, :M]^T B (M
        defaults to A's width), its tiles transposed by the product kernel; Kpad
        is then the thin operand's padded length (a multiple of 128, >= K)."""
        lib = load()
        self.prec, self.A, self.E, self.ea, self.stream, self.at, self.K = prec, A, E, ea, stream, at, K
        if at:
            self.M = A.shape[1] if M is None else M
            self.Kpad = Kpad if Kpad is not None else -(-K // 128) * 128
        else:
            self.M, self.Kpad = A.shape
        self.N = B.shape[1]
        dt = torch.int16 if prec == NMF_BF16 else torch.uint8
        self.Bt = torch.zeros(self.N, self.Kpad, dtype=dt, device=A.device)
        self.EB = torch.zeros(max(self.Kpad // 128, 1), dtype=torch.int32, device=A.device)
        _check(lib.nmf_lowp_prepare_thin(prec, _ptr(B), B.stride(0), K, self.N, _ptr(self.Bt), self.Kpad,
                                         _ptr(self.EB), _stream(stream)))
        self.splits = int(lib.nmf_gemm_lowp_splits(self.M, self.N, self.Kpad))
        self.part = torch.empty(self.splits, self.M, self.N, dtype=torch.float32, device=A.device)

    def run(self):
        if self.at:
            _check(load().nmf_gemm_bf16_at_prepared(_ptr(self.A), self.A.stride(0), self.K, _ptr(self.Bt), self.N,
                                                    _ptr(self.part), self.N, self.M, self.Kpad, self.splits,
                                                    _stream(self.stream)))
            return
        _check(load().nmf_gemm_lowp_prepared(self.prec, _ptr(self.A), self.A.stride(0), _ptr(self.E), self.ea[0],
                                             self.ea[1], _ptr(self.Bt), _ptr(self.EB), self.N, _ptr(self.part),
                                             self.N, self.M, self.Kpad, self.splits, _stream(self.stream)))

    def result(self):
        return self.part.sum(dim=0) if self.splits > 1 else self.part[0]
