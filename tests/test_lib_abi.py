"""The C-ABI library loads and exports every symbol its header declares; host
logic that needs no GPU (parameter validation, workspace sizing)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmfrp.h")
LIB = os.path.join(ROOT, "paper_1712_02248_amd", "libnmfrp.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nmf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnmfrp.so is not built (python -m paper_1712_02248_amd.build)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1712_02248_amd import nmfrp
    assert set(nmfrp._SIGS) == set(declared_functions())


def _params(**kw):
    from paper_1712_02248_amd.nmfrp import Params
    d = dict(m=512, n=256, r=10, k_sketch=20, q=2, prec=0, refine_fp32=0, normalize=1, alpha=0.0,
             beta=0.0, seed=1)
    d.update(kw)
    return Params(**d)


def test_workspace_sizing_and_validation():
    from paper_1712_02248_amd import nmfrp
    lib = nmfrp.load()
    ok = lib.nmf_workspace_bytes(ctypes.byref(_params()))
    assert ok > 0 and ok % 256 == 0
    # the sketches dominate: at least the eight k'-wide buffers
    assert ok >= 4 * 20 * (3 * 256 + 5 * 512)
    bad = [dict(r=20), dict(r=25), dict(k_sketch=300), dict(n=254), dict(q=-1), dict(normalize=3),
           dict(m=0), dict(alpha=-1.0), dict(k_sketch=257, m=1000, n=1000), dict(lowp_sketches=1),
           dict(lowp_sketches=3, prec=1), dict(lowp_sketches=-1), dict(update_prec=2), dict(update_prec=-1),
           dict(update_prec=1)]   # split-BF16 update products need the wide-factor path
    assert lib.nmf_workspace_bytes(ctypes.byref(_params(lowp_sketches=1, prec=1))) > 0
    # split-BF16 sketches: any prec; the split thin operands add to the workspace
    for prec in (0, 1, 2):
        w2 = lib.nmf_workspace_bytes(ctypes.byref(_params(lowp_sketches=2, prec=prec)))
        assert w2 > lib.nmf_workspace_bytes(ctypes.byref(_params(prec=prec)))
    for b in bad:
        assert lib.nmf_workspace_bytes(ctypes.byref(_params(**b))) == 0, b
        assert lib.nmf_last_error(None)


def test_create_rejects_small_or_misaligned_workspace():
    from paper_1712_02248_amd import nmfrp
    lib = nmfrp.load()
    h = ctypes.c_void_p()
    p = _params()
    need = lib.nmf_workspace_bytes(ctypes.byref(p))
    assert lib.nmf_create(ctypes.byref(p), 4096, need - 1, None, ctypes.byref(h)) == -2
    assert lib.nmf_create(ctypes.byref(p), 4097, need, None, ctypes.byref(h)) == -1
    assert lib.nmf_create(ctypes.byref(_params(r=30)), 4096, need, None, ctypes.byref(h)) == -1
    assert not h.value


def test_gemm_workspace_sizing_on_empty_and_skinny_shapes():
    from paper_1712_02248_amd import nmfrp
    lib = nmfrp.load()
    for M, N, K, at in [(0, 8, 16, 0), (8, 0, 16, 1), (0, 0, 0, 0), (4096, 64, 65536, 1), (65536, 64, 4096, 0)]:
        assert lib.nmf_gemm_workspace_bytes(M, N, K, at) >= 256
    # empty products are no-ops that need no device pointers
    assert lib.nmf_gemm(None, 16, 0, None, 8, None, 8, 0, 8, 16, None, 0, None) == 0
