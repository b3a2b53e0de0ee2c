"""C-ABI checks that need no GPU: the library loads, exports every function
include/linprim.h declares, and rejects bad arguments before touching a
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "linprim.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(linprim_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2501_16312_amd import linprim as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2501_16312_amd import build
        build.build()
    return L


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 10
    cdll = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(cdll, n), n
    assert set(lib.EXPORTS) <= set(names)


def test_workspace_sizes_and_validation(lib):
    from paper_2501_16312_amd import scenes
    cams = lib.cameras([scenes.make_camera(__import__("numpy").eye(3, 4, dtype="float32"), 64, 48)])
    t16 = lib.tuning(16)
    a = lib.linprim_view_workspace_size(0, 1000, cams, t16)
    b = lib.linprim_view_workspace_size(0, 2000, cams, t16)
    assert a > 0 and b > a and a % 256 == 0
    assert lib.linprim_view_workspace_size(7, 10, cams, t16) == 0          # unknown type
    assert lib.linprim_view_workspace_size(0, 10, cams, lib.tuning(12)) == 0  # bad tile
    assert lib.linprim_view_workspace_size(0, -1, cams, t16) == 0
    p1 = lib.linprim_pair_workspace_size(1000, cams, t16)
    p2 = lib.linprim_pair_workspace_size(100000, cams, t16)
    assert 0 < p1 < p2
    # pair workspace: keys x2 (8 B), values x2 (4 B), 20-float gradient records
    assert p2 >= 100000 * (8 + 8 + 4 + 4 + 80)
    assert lib.linprim_pair_workspace_size(1 << 31, cams, t16) == 0
    assert lib.linprim_pair_workspace_size(10, cams, lib.tuning(16, 9)) == 0
    # the anti-aliasing filter belongs to the ray-space model
    assert lib.linprim_view_workspace_size(0, 10, cams, lib.tuning(16, 8, lib.FLAG_ANTIALIAS)) > 0
    assert lib.linprim_view_workspace_size(0, 10, cams, lib.tuning(16, 8, lib.FLAG_EXACT_RAYS)) > 0
    assert lib.linprim_view_workspace_size(
        0, 10, cams, lib.tuning(16, 8, lib.FLAG_EXACT_RAYS | lib.FLAG_ANTIALIAS)) == 0


def test_null_arguments_rejected_without_device(lib):
    L = lib.load()
    cams = lib.cameras([])
    rc = L.linprim_preprocess(None, cams, 0, None, None, 0, None)
    assert rc == lib.ERR_INVALID_ARG
    rc = L.linprim_bin_sort(None, cams, 0, None, None, 0, None, 0, 0, None)
    assert rc == lib.ERR_INVALID_ARG
    n = ctypes.c_int64(0)
    assert L.linprim_pair_count(None, ctypes.byref(n), None) == lib.ERR_INVALID_ARG
    assert L.linprim_strerror(lib.ERR_WORKSPACE).decode() == "workspace too small"
    assert L.linprim_strerror(12345).decode() == "unknown error"


def test_product_path_has_no_cpu_fallback():
    """The binding fails loudly when the library is missing and never imports
    the oracle."""
    from paper_2501_16312_amd import linprim as L
    with pytest.raises(L.LinPrimError):
        saved = L._lib
        try:
            L._lib = None
            L.load(os.path.join(ROOT, "does-not-exist.so"))
        finally:
            L._lib = saved
    pkg = os.path.join(ROOT, "paper_2501_16312_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in src and "from oracle" not in src, fn
