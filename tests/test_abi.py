"""The C-ABI library loads, exports every symbol include/bandops.h declares, and
rejects bad arguments before launching anything (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bandops.h")
LIBPATH = os.path.join(ROOT, "paper_1902_10078_amd", "libbandops.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIBPATH), reason="libbandops.so not built")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bo_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    from paper_1902_10078_amd import bandops
    assert set(declared_symbols()) == set(bandops.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIBPATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.fixture(scope="module")
def L():
    from paper_1902_10078_amd import bandops
    return bandops.lib()


def _band(n, l, u, ld, ptr=1, diag=None):
    from paper_1902_10078_amd.bandops import _Band
    return _Band(ctypes.c_void_p(ptr), ctypes.c_void_p(diag) if diag else None, n, l, u, ld, 0)


def test_status_strings(L):
    assert L.bo_status_string(0) == b"ok"
    assert L.bo_status_string(-1) == b"invalid argument"
    assert L.bo_status_string(-3) == b"workspace too small"


def test_workspace_query(L):
    assert L.bo_workspace_size(1000, 3) > 0
    assert L.bo_workspace_size(1000, 13) == 0      # beyond BO_KMAX
    assert L.bo_workspace_size(-1, 3) == 0
    # grows with n
    assert L.bo_workspace_size(10 ** 6, 5) > L.bo_workspace_size(10 ** 4, 5)


def test_argument_errors_return_before_launch(L):
    bp = ctypes.byref
    info = ctypes.c_void_p(8)
    Q = _band(100, 3, 0, 4)
    Lb = _band(100, 3, 0, 4)
    # null descriptor
    assert L.bo_chol(0, None, bp(Lb), None, None, None, info, None, 0, None) == -1
    assert b"null descriptor" in L.bo_last_error()
    # ld < l+u+1
    bad = _band(100, 3, 0, 3)
    assert L.bo_chol(0, bp(bad), bp(Lb), None, None, None, info, None, 0, None) == -1
    assert b"ld" in L.bo_last_error()
    # negative n
    neg = _band(-5, 3, 0, 4)
    assert L.bo_chol(0, bp(neg), bp(Lb), None, None, None, info, None, 0, None) == -1
    # upper width on a factor
    up = _band(100, 3, 1, 5)
    assert L.bo_chol(0, bp(up), bp(Lb), None, None, None, info, None, 0, None) == -1
    # mismatched shapes
    L2 = _band(99, 3, 0, 4)
    assert L.bo_chol(0, bp(Q), bp(L2), None, None, None, info, None, 0, None) == -1
    # y without z
    assert L.bo_chol(0, bp(Q), bp(Lb), ctypes.c_void_p(16), None, None, info, None, 0, None) == -1
    # missing info
    assert L.bo_chol(0, bp(Q), bp(Lb), None, None, None, None, None, 0, None) == -1
    # mixed without the FP64 diagonal; F64 with one
    assert L.bo_chol(1, bp(Q), bp(Lb), None, None, None, info, None, 0, None) == -1
    Qd = _band(100, 3, 0, 4, diag=64)
    assert L.bo_chol(0, bp(Qd), bp(Lb), None, None, None, info, None, 0, None) == -1
    # bandwidth beyond the compiled range
    wide = _band(100, 13, 0, 14)
    wideL = _band(100, 13, 0, 14)
    assert L.bo_chol(0, bp(wide), bp(wideL), None, None, None, info, None, 0, None) == -4
    # workspace too small
    assert L.bo_chol(0, bp(Q), bp(Lb), None, None, None, info, ctypes.c_void_p(4096), 16, None) == -3
    # unknown precision
    assert L.bo_trsv(7, bp(Q), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, 100, None, 0, None) == -1
    # null vectors
    assert L.bo_trsv(0, bp(Q), 0, None, None, 1, 100, None, 0, None) == -1
    # several right-hand sides with ldx < n; a negative count
    assert L.bo_trsv(0, bp(Q), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), 2, 99, None, 0, None) == -1
    assert L.bo_trsv(0, bp(Q), 0, ctypes.c_void_p(8), ctypes.c_void_p(8), -1, 100, None, 0, None) == -1
    # subset inverse: output narrower than L, too wide, or wider and not packed
    S2 = _band(100, 2, 0, 3)
    assert L.bo_subset_inv(0, bp(Q), bp(S2), None, 0, None) == -1
    S13 = _band(100, 13, 0, 14)
    assert L.bo_subset_inv(0, bp(Q), bp(S13), ctypes.c_void_p(4096), 1 << 30, None) == -4
    S7 = _band(100, 7, 0, 9)
    assert L.bo_subset_inv(0, bp(Q), bp(S7), ctypes.c_void_p(4096), 1 << 30, None) == -1
    S7p = _band(100, 7, 0, 8)
    assert L.bo_subset_inv(0, bp(Q), bp(S7p), ctypes.c_void_p(4096), 16, None) == -3
    assert L.bo_subset_inv_workspace_size(100, 3, 7) > L.bo_workspace_size(100, 7)
    assert L.bo_subset_inv_workspace_size(100, 3, 3) == L.bo_workspace_size(100, 3)
    assert L.bo_subset_inv_workspace_size(100, 3, 2) == 0


def test_plan_errors_and_stats(L):
    from paper_1902_10078_amd.bandops import _Problem
    h = ctypes.c_void_p()
    probs = (_Problem * 2)(_Problem(100, 3, 0, 0, 0), _Problem(50, 14, 0, 400, 100))
    assert L.bo_plan_create(probs, 2, 0, ctypes.byref(h)) == -4
    probs = (_Problem * 2)(_Problem(100, 3, 0, 0, 0), _Problem(-1, 1, 0, 400, 100))
    assert L.bo_plan_create(probs, 2, 0, ctypes.byref(h)) == -1
    assert L.bo_plan_create(probs, 0, 0, ctypes.byref(h)) == -1
    assert L.bo_plan_create(None, 1, 0, ctypes.byref(h)) == -1


def test_vi_kl_errors(L):
    """bo_plan_vi_kl refuses a missing plan, io or workspace before any launch."""
    from paper_1902_10078_amd.bandops import _KLIO
    io = _KLIO()
    assert L.bo_plan_vi_kl(None, 0, ctypes.byref(io), ctypes.c_void_p(1), None) == -1
    assert L.bo_plan_vi_kl(None, 0, None, ctypes.c_void_p(1), None) == -1
    assert b"bo_plan_vi_kl" in L.bo_last_error()


def test_marglik_errors(L):
    """bo_plan_marglik refuses a missing plan, io or workspace before any launch."""
    from paper_1902_10078_amd.bandops import _MLIO
    io = _MLIO()
    assert L.bo_plan_marglik(None, 0, ctypes.byref(io), ctypes.c_void_p(1), None) == -1
    assert L.bo_plan_marglik(None, 0, None, ctypes.c_void_p(1), None) == -1
    assert b"bo_plan_marglik" in L.bo_last_error()


def test_natgp_errors(L):
    """bo_plan_natgp refuses a missing plan, io or workspace before any launch."""
    from paper_1902_10078_amd.bandops import _NGIO
    io = _NGIO()
    assert L.bo_plan_natgp(None, 0, ctypes.byref(io), ctypes.c_void_p(1), None) == -1
    assert L.bo_plan_natgp(None, 0, None, ctypes.c_void_p(1), None) == -1
    assert b"bo_plan_natgp" in L.bo_last_error()


def test_whiten_errors(L):
    """bo_plan_whiten and its reverse refuse a missing plan, io or workspace
    before any launch."""
    from paper_1902_10078_amd.bandops import _WHIO
    io = _WHIO()
    assert L.bo_plan_whiten(None, 0, ctypes.byref(io), ctypes.c_void_p(1), None) == -1
    assert b"bo_plan_whiten" in L.bo_last_error()
    assert L.bo_plan_whiten_bwd(None, 0, ctypes.byref(io), ctypes.c_void_p(1), None) == -1
    assert b"bo_plan_whiten_bwd" in L.bo_last_error()


def test_wide_errors_and_workspace(L):
    """The wide (k = 64) entry points: argument errors before any launch, and
    the workspace size (problem and chunk tables, two FP32 64 x 64 blocks per
    block row, eleven per chunk and three doubles per chunk; here every block
    is a chunk of its own)."""
    from paper_1902_10078_amd.bandops import _BatchIO, _Problem
    sz = ctypes.c_size_t()
    probs = (_Problem * 2)(_Problem(130, 64, 0, 0, 0), _Problem(64, 64, 0, 130 * 65, 130))
    assert L.bo_wide_workspace_size(probs, 2, ctypes.byref(sz)) == 0
    blocks = chunks = 3 + 1
    al = lambda x: (x + 255) // 256 * 256
    assert sz.value == (al(2 * 40) + al(chunks * 24) + al(blocks * 2 * 64 * 64 * 4) + al(chunks * 11 * 64 * 64 * 4)
                        + al(chunks * 3 * 8))
    bad = (_Problem * 1)(_Problem(100, 5, 0, 0, 0))
    assert L.bo_wide_workspace_size(bad, 1, ctypes.byref(sz)) == -4
    assert b"k = 64" in L.bo_last_error()
    neg = (_Problem * 1)(_Problem(-3, 64, 0, 0, 0))
    assert L.bo_wide_workspace_size(neg, 1, ctypes.byref(sz)) == -1
    assert L.bo_wide_workspace_size(None, 1, ctypes.byref(sz)) == -1
    # a workspace that is too small is refused before any copy
    assert L.bo_wide_upload(probs, 2, ctypes.c_void_p(1), 16) == -3
    io = _BatchIO()
    # missing required arrays: refused before any launch
    assert L.bo_wide_forward(probs, 1, ctypes.byref(io), ctypes.c_void_p(1), 1 << 30, None) == -1
    assert L.bo_wide_gauss_loss(probs, 1, ctypes.byref(io), ctypes.c_void_p(1), 1 << 30, None) == -1
    assert L.bo_wide_forward(probs, 0, ctypes.byref(io), ctypes.c_void_p(1), 1 << 30, None) == -1
