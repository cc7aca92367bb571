"""Pins of the spectrum oracle (eigenvalues, singular values of the compressed
data, decay fits) against closed forms and exact cases.  CPU only."""
import numpy as np

from oracle import spectrum


def householder(v):
    v = v / np.linalg.norm(v)
    return np.eye(len(v)) - 2.0 * np.outer(v, v)


def test_sym_eigvals_closed_forms():
    # 2 x 2: (a + c)/2 +- sqrt(((a - c)/2)^2 + b^2)
    a, b, c = 3.0, -1.25, 0.5
    h = np.hypot((a - c) / 2, b)
    assert np.allclose(spectrum.sym_eigvals([[a, b], [b, c]]), [(a + c) / 2 + h, (a + c) / 2 - h], rtol=0, atol=1e-15)
    # diagonal: the entries, sorted descending
    d = np.array([0.5, -2.0, 7.0, 0.0, 3.0])
    assert np.array_equal(spectrum.sym_eigvals(np.diag(d)), np.sort(d)[::-1])
    # Q diag(lam) Q^T with an orthogonal reflector: lam back
    g = np.random.default_rng(3)
    lam = np.array([9.0, 4.0, 4.0, 1.0, -0.5, -3.0])
    Q = householder(g.standard_normal(6))
    A = Q @ np.diag(lam) @ Q.T
    assert np.allclose(spectrum.sym_eigvals(A), lam, rtol=0, atol=1e-13)
    # only the lower triangle is read
    U = np.triu(g.standard_normal((6, 6)), 1)
    assert np.allclose(spectrum.sym_eigvals(np.tril(A) + 100 * U), lam, rtol=0, atol=1e-13)


def test_sym_eigvals_invariants():
    g = np.random.default_rng(4)
    B = g.standard_normal((40, 40))
    A = B + B.T
    w = spectrum.sym_eigvals(A)
    assert np.all(np.diff(w) <= 0)
    assert abs(w.sum() - np.trace(A)) <= 1e-12 * np.abs(A).sum()
    assert abs((w ** 2).sum() - (A ** 2).sum()) <= 1e-12 * (A ** 2).sum()


def test_sketch_singular_values_exact_on_captured_rank():
    """Rank rho <= k': the range finder's span holds range(X), so the compressed
    data keeps every singular value of X."""
    g = np.random.default_rng(5)
    m, n, rho, kp = 300, 120, 5, 8
    U = np.linalg.qr(g.standard_normal((m, rho)))[0]
    V = np.linalg.qr(g.standard_normal((n, rho)))[0]
    s = np.array([50.0, 20.0, 7.0, 2.0, 0.3])
    X = U @ np.diag(s) @ V.T
    QL = np.linalg.qr(X @ g.standard_normal((n, kp)))[0]
    sig = spectrum.sketch_singular_values(X, QL)
    assert sig.shape == (kp,)
    assert np.allclose(sig[:rho], s, rtol=1e-12, atol=0)
    assert np.all(sig[rho:] <= 1e-12 * s[0])
    # squares = eigenvalues of X-hat X-hat^T
    Xh = QL.T @ X
    assert np.allclose(sig ** 2, spectrum.sym_eigvals(Xh @ Xh.T), rtol=0, atol=1e-10 * s[0] ** 2)


def test_sketch_singular_values_interlace():
    """sigma_j(L^T X) <= sigma_j(X) for any orthonormal L, strictly below for a
    random L on a full-rank X."""
    g = np.random.default_rng(6)
    X = g.random((200, 90))
    Q = np.linalg.qr(g.standard_normal((200, 10)))[0]
    sig = spectrum.sketch_singular_values(X, Q)
    full = np.linalg.svd(X, compute_uv=False)[:10]
    assert np.all(sig <= full * (1 + 1e-12))
    assert sig[-1] < full[-1] * 0.99


def test_decay_fits_recover_exact_laws():
    j = np.arange(1, 65, dtype=np.float64)
    pw = 3.0 * j ** -0.7
    ex = 2.0 * np.exp(-0.05 * j)
    assert abs(spectrum.decay_power(pw) - 0.7) <= 1e-12
    assert abs(spectrum.decay_exp(ex) - 0.05) <= 1e-12
    # the readings differ: each law fitted by the other is off
    assert abs(spectrum.decay_exp(pw) - 0.7) > 0.5
    assert abs(spectrum.decay_power(ex) - 0.05) > 0.1
    # the index range: a perturbed head outside it changes nothing
    pw2 = pw.copy()
    pw2[:3] *= 5.0
    assert abs(spectrum.decay_power(pw2, j0=4) - 0.7) <= 1e-12
    assert abs(spectrum.decay_power(pw2[:40], j0=4, j1=40) - 0.7) <= 1e-12
