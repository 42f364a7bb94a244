"""CPU oracle for exact top-k LCP retrieval.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the GPU path.

* ``lcp_oracle``: NumPy/pure-Python definitions (small inputs, structure).
* ``cpu_topk.c``: plain C brute force (OpenMP over queries) for large inputs;
  built into ``libcpu_topk.so`` next to this file by ``build()``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import lcp_oracle  # noqa: F401
from .lcp_oracle import csr_offsets

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_topk.c")
_LIB = os.path.join(_HERE, "libcpu_topk.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C oracle (gcc, OpenMP) into oracle/libcpu_topk.so."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _bind(lib):
    lib.oracle_topk.restype = ctypes.c_int
    lib.oracle_topk.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_threads.argtypes = [ctypes.c_int32]
    return lib


_native = None


def native_lib():
    """The same C source compiled for the host it runs on (-O3 -march=native),
    into a temporary directory (never shipped to another machine); used for the
    CPU-baseline timing.  Returns the loaded library."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="cpu_topk_native_")
        out = os.path.join(d, "libcpu_topk_native.so")
        subprocess.run(["gcc", "-O3", "-march=native", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", out],
                       check=True)
        _native = _bind(ctypes.CDLL(out))
    return _native


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def threads(nthreads: int = 0) -> int:
    return int(_load().oracle_threads(nthreads))


def c_topk(db: np.ndarray, queries: np.ndarray, ks, nthreads: int = 0, native: bool = False):
    """Brute-force top-k for a batch (C oracle).  Returns (ids, lcps, offsets).
    native=True runs the build made for this host (native_lib)."""
    lib = native_lib() if native else _load()
    db = np.ascontiguousarray(db)
    queries = np.ascontiguousarray(queries, dtype=db.dtype)
    if db.dtype not in (np.uint8, np.uint16):
        raise TypeError("tokens must be uint8 or uint16")
    ks = np.ascontiguousarray(np.broadcast_to(np.asarray(ks, dtype=np.int32), (queries.shape[0],)))
    off = csr_offsets(ks)
    ids = np.empty(int(off[-1]), dtype=np.int32)
    lcps = np.empty(int(off[-1]), dtype=np.int32)
    rc = lib.oracle_topk(db.ctypes.data, db.shape[0], db.shape[1], db.dtype.itemsize,
                         queries.ctypes.data, queries.shape[0], ks.ctypes.data, off.ctypes.data,
                         ids.ctypes.data, lcps.ctypes.data, int(nthreads))
    if rc != 0:
        raise ValueError("oracle_topk rejected its arguments")
    return ids, lcps, off
