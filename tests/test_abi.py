"""The C-ABI library loads and exports every entry point include/lcp.h declares
(no compute calls, so this runs without a GPU)."""
import ctypes
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lcp.h")
LIB = os.path.join(ROOT, "paper_2602_04936_amd", "liblcp.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lcp_[a-z_]+)\s*\(", src)))


def _ensure_built():
    if not os.path.exists(LIB):
        subprocess.run([sys.executable, os.path.join(ROOT, "paper_2602_04936_amd", "build_lib.py")], check=True)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lcp_index_build", "lcp_topk", "lcp_scan_topk", "lcp_index_free", "lcp_last_error",
              "lcp_topk_dev", "lcp_scan_topk_dev", "lcp_index_info", "lcp_index_views"):
        assert n in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_paths_without_gpu():
    """Argument checks run before any device call."""
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    lib.lcp_index_build.restype = ctypes.c_int
    lib.lcp_index_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.lcp_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.lcp_index_build(None, 10, 4, 16, None, ctypes.byref(h)) == -1
    assert b"tokens" in lib.lcp_last_error()
    dummy = ctypes.create_string_buffer(64)
    assert lib.lcp_index_build(dummy, 0, 4, 16, None, ctypes.byref(h)) == -1
    assert lib.lcp_index_build(dummy, 10, 256, 16, None, ctypes.byref(h)) == -1
    assert lib.lcp_index_build(dummy, 10, 4, 65537, None, ctypes.byref(h)) == -1
    # the row limit keeps positions (and the A window past the end) below 2^31
    assert lib.lcp_index_build(dummy, (1 << 31) - (1 << 16) + 1, 4, 16, None, ctypes.byref(h)) == -1
    assert b"2^31 - 2^16" in lib.lcp_last_error()
    assert h.value is None
    lib.lcp_topk.restype = ctypes.c_int
    lib.lcp_topk.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] + [ctypes.c_void_p] * 4
    assert lib.lcp_topk(None, None, 1, None, None, None, None) == -1
    lib.lcp_topk_persistent.restype = ctypes.c_int
    lib.lcp_topk_persistent.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_int64] + [ctypes.c_void_p] * 3 +
                                        [ctypes.c_int32] + [ctypes.c_void_p] * 2 + [ctypes.c_int32, ctypes.c_void_p])
    assert lib.lcp_topk_persistent(None, None, 8, None, None, None, 10, None, None, 0, None) == -1
    lib.lcp_index_append.restype = ctypes.c_int
    lib.lcp_index_append.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert lib.lcp_index_append(None, None, 1, None) == -1
    lib.lcp_index_reserve.restype = ctypes.c_int
    lib.lcp_index_reserve.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert lib.lcp_index_reserve(None, 10, None) == -1
    lib.lcp_index_set_search.restype = ctypes.c_int
    lib.lcp_index_set_search.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    assert lib.lcp_index_set_search(None, 1) == -1
    lib.lcp_index_generation.restype = ctypes.c_int
    lib.lcp_index_generation.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lcp_index_generation(None, None) == -1
    lib.lcp_topk_stats.restype = ctypes.c_int
    lib.lcp_topk_stats.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_int64] + [ctypes.c_void_p] * 5
    assert lib.lcp_topk_stats(None, None, 1, None, None, None, None, None) == -1
    lib.lcp_bucket_scan_topk.restype = ctypes.c_int
    lib.lcp_bucket_scan_topk.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_int64, ctypes.c_int32] +
                                         [ctypes.c_void_p] * 5)
    assert lib.lcp_bucket_scan_topk(None, None, 1, 2, None, None, None, None, None) == -1
    assert b"index is NULL" in lib.lcp_last_error()
    assert lib.lcp_bucket_scan_topk(None, None, 1, 2, None, None, None, 4, None) == -1  # bounds not 8-byte aligned
    assert b"aligned" in lib.lcp_last_error()
    lib.lcp_index_free(None)


def test_package_has_no_cpu_fallback():
    """The binding refuses to import without the HIP library and never imports the oracle."""
    src = open(os.path.join(ROOT, "paper_2602_04936_amd", "__init__.py")).read()
    assert "oracle" not in src
    assert "raise ImportError" in src
