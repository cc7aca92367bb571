"""FP64 oracle of the spectrum of the compressed data (test infrastructure only).

The paper's parameter study relates the best power-iteration count w of the
range finder (eq 3.5) to how fast the singular values of X decay (Sec 5.2).
The compressed data X-hat = L^T X (Sec 4) carries the leading singular values:
for an orthonormal L, sigma_j(L^T X) <= sigma_j(X) for every j (interlacing of
singular values under projection), with equality for the j that L's span
captures exactly.

The decay law is printed garbled (a bare sigma_j(X)^{-p}); two readings are
kept, both fitted by least squares over a stated index range:
  power law    sigma_j ~ c j^{-p}    (slope of log sigma_j against log j)
  exponential  sigma_j ~ c e^{-p j}  (slope of log sigma_j against j)
"""
import numpy as np


def sym_eigvals(A):
    """Eigenvalues of the symmetric matrix A (lower triangle read), descending:
    the library's symmetric eigensolver as the definition."""
    A = np.tril(np.asarray(A, dtype=np.float64))
    A = A + np.tril(A, -1).T
    return np.linalg.eigvalsh(A)[::-1]


def sketch_singular_values(X, QL):
    """Singular values of X-hat = QL^T X (Sec 4), descending, from its SVD."""
    Xh = np.asarray(QL, np.float64).T @ np.asarray(X, np.float64)
    return np.linalg.svd(Xh, compute_uv=False)


def decay_power(sigma, j0=1, j1=None):
    """p of sigma_j ~ c j^{-p}, least squares over j = j0 .. j1 (1-based, inclusive)."""
    s = np.asarray(sigma, np.float64)
    j1 = len(s) if j1 is None else j1
    j = np.arange(j0, j1 + 1, dtype=np.float64)
    slope = np.polyfit(np.log(j), np.log(s[j0 - 1:j1]), 1)[0]
    return -slope


def decay_exp(sigma, j0=1, j1=None):
    """p of sigma_j ~ c e^{-p j}, least squares over j = j0 .. j1 (1-based, inclusive)."""
    s = np.asarray(sigma, np.float64)
    j1 = len(s) if j1 is None else j1
    j = np.arange(j0, j1 + 1, dtype=np.float64)
    slope = np.polyfit(j, np.log(s[j0 - 1:j1]), 1)[0]
    return -slope
