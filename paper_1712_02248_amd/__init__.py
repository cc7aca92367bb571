"""MI355X-native compressed NMF with random projections (FastHALS-RP).

The method runs in hand-written HIP kernels for gfx950 behind the C ABI of
include/nmfrp.h (libnmfrp.so); `nmfrp` is its ctypes binding.
"""
from . import nmfrp  # noqa: F401
from .nmfrp import Mlp, NMF, NmfError, gaussian, gemm, load, mlp_n_params, nnls_rows, orth, uniform  # noqa: F401
