"""Exact top-k retrieval under longest-common-prefix similarity on MI355X.

Thin Python binding over ``liblcp.so`` (C ABI in ``include/lcp.h``): it only
marshals arguments; every step of the computation runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.  There is no CPU
fallback: importing this package fails if the library has not been built
(``python paper_2602_04936_amd/build_lib.py``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Union

import numpy as np
import torch

__all__ = ["Index", "TopK", "LcpError", "LIB_PATH", "K_MAX", "L_MAX", "NOALLOC_SCRATCH_BYTES", "lib"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcp.so")
K_MAX = 1024
L_MAX = 255
NOALLOC_SCRATCH_BYTES = 32 << 20  # LCP_NOALLOC_SCRATCH_BYTES

_STATUS = {0: "LCP_OK", -1: "LCP_EINVAL", -2: "LCP_ENOMEM", -3: "LCP_EDEVICE", -4: "LCP_ERANGE",
           -5: "LCP_ENOTIMPL"}


class LcpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


def _load_lib() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2602_04936_amd/build_lib.py`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    sigs = {
        "lcp_index_build": [vp, i64, i32, i32, vp, ctypes.POINTER(vp)],
        "lcp_topk": [vp, vp, i64, vp, vp, vp, vp],
        "lcp_scan_topk": [vp, vp, i64, vp, vp, vp, vp],
        "lcp_bucket_scan_topk": [vp, vp, i64, i32, vp, vp, vp, vp, vp],
        "lcp_topk_stats": [vp, vp, i64, vp, vp, vp, vp, vp],
        "lcp_topk_dev": [vp, vp, i64, vp, vp, i32, vp, vp, vp],
        "lcp_scan_topk_dev": [vp, vp, i64, vp, vp, i32, vp, vp, vp],
        "lcp_scan_topk_dev_noalloc": [vp, vp, i64, vp, vp, i32, vp, vp, vp],
        "lcp_index_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                           ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lcp_index_views": [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)],
        "lcp_scan_info": [vp, i64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)],
        "lcp_index_append": [vp, vp, i64, vp],
        "lcp_topk_persistent": [vp, vp, i64, vp, vp, vp, i32, vp, vp, i32, vp],
        "lcp_index_generation": [vp, ctypes.POINTER(ctypes.c_uint64)],
        "lcp_index_set_search": [vp, i32],
        "lcp_index_reserve": [vp, i64, vp],
        "lcp_index_search_mode": [vp, ctypes.POINTER(i32)],
        "lcp_set_kernel_timing": [vp, i32],
        "lcp_kernel_time": [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.lcp_index_free.argtypes = [vp]
    L.lcp_index_free.restype = None
    L.lcp_last_error.argtypes = []
    L.lcp_last_error.restype = ctypes.c_char_p
    return L


lib = _load_lib()


def _check(status: int):
    if status != 0:
        raise LcpError(status, lib.lcp_last_error().decode(errors="replace"))


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _token_tensor(x: torch.Tensor, token_bytes: Optional[int] = None) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError("tokens must be a CUDA (HIP) tensor")
    if x.dim() != 2:
        raise ValueError("tokens must be 2-D [rows, L]")
    tb = x.element_size()
    if x.dtype not in (torch.uint8, torch.int16, torch.uint16):
        raise TypeError(f"tokens must be uint8, uint16 or int16 (got {x.dtype})")
    if token_bytes is not None and tb != token_bytes:
        raise TypeError(f"tokens must be {token_bytes}-byte (got {x.dtype})")
    return x.contiguous()


def to_device_tokens(arr: np.ndarray, device="cuda") -> torch.Tensor:
    """Host uint8/uint16 token matrix -> device tensor (uint16 travels as int16 bits)."""
    arr = np.ascontiguousarray(arr)
    if arr.dtype == np.uint16:
        arr = arr.view(np.int16)
    elif arr.dtype != np.uint8:
        raise TypeError("tokens must be uint8 or uint16")
    return torch.from_numpy(arr).to(device)


@dataclass
class TopK:
    """Answers in CSR layout: query i owns [offsets[i], offsets[i+1])."""
    ids: torch.Tensor       # int32 [sum k]
    lcps: torch.Tensor      # int32 [sum k]
    offsets: np.ndarray     # int64 [Q+1] (host)

    def query(self, i: int):
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.ids[a:b], self.lcps[a:b]


class Index:
    """Sorted index over N rows of L tokens (each < V), resident on the current device."""

    def __init__(self, tokens: Union[torch.Tensor, np.ndarray], V: int, stream=None):
        if isinstance(tokens, np.ndarray):
            tokens = to_device_tokens(tokens)
        t = _token_tensor(tokens)
        N, L = t.shape
        h = ctypes.c_void_p()
        _check(lib.lcp_index_build(t.data_ptr(), N, L, int(V), _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self._kcache = {}
        n, l, v, tb, w = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.lcp_index_info(h, ctypes.byref(n), ctypes.byref(l), ctypes.byref(v), ctypes.byref(tb),
                                  ctypes.byref(w)))
        self.N, self.L, self.V, self.token_bytes, self.row_words = n.value, l.value, v.value, tb.value, w.value
        self.device = t.device

    # ------------------------------------------------------------- queries
    def _prep(self, queries, k):
        if isinstance(queries, np.ndarray):
            queries = to_device_tokens(queries, self.device)
        q = _token_tensor(queries, self.token_bytes)
        if q.shape[1] != self.L:
            raise ValueError(f"queries have L={q.shape[1]}, index has L={self.L}")
        Q = q.shape[0]
        if isinstance(k, (int, np.integer)):
            # one k for every query: the k and offset arrays are built once per
            # (Q, k) and reused (read-only), keeping the per-call host work small
            key = (Q, int(k))
            hit = self._kcache.get(key)
            if hit is None:
                kk = np.full(Q, int(k), dtype=np.int32)
                off = np.arange(Q + 1, dtype=np.int64) * int(k)
                kk.flags.writeable = False
                off.flags.writeable = False
                if len(self._kcache) >= 64:
                    self._kcache.clear()
                hit = self._kcache[key] = (kk, off)
            return (q,) + hit
        kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (Q,)))
        off = np.zeros(Q + 1, dtype=np.int64)
        np.cumsum(kk, out=off[1:])
        return q, kk, off

    def _run(self, fn, queries, k, stream, out):
        q, kk, off = self._prep(queries, k)
        total = int(off[-1])
        if out is None:
            ids = torch.empty(total, dtype=torch.int32, device=self.device)
            lcps = torch.empty(total, dtype=torch.int32, device=self.device)
        else:
            ids, lcps = out
            if ids.numel() < total or lcps.numel() < total:
                raise ValueError("output tensors are too small")
        _check(fn(self._h, q.data_ptr(), q.shape[0], kk.ctypes.data, ids.data_ptr(), lcps.data_ptr(),
                  _stream_handle(stream)))
        return TopK(ids, lcps, off)

    def topk(self, queries, k: Union[int, Sequence[int], np.ndarray], stream=None, out=None) -> TopK:
        """Index path (lcp_topk)."""
        return self._run(lib.lcp_topk, queries, k, stream, out)

    def topk_stats(self, queries, k: Union[int, Sequence[int], np.ndarray], stream=None, out=None):
        """Index path with per-query work shape (lcp_topk_stats): returns (TopK, stats) where stats is
        an int32 [Q, 4] device tensor of (cutoff LCP c, rows above c, rows tied at c, tie selection)."""
        q, kk, off = self._prep(queries, k)
        total = int(off[-1])
        if out is None:
            ids = torch.empty(total, dtype=torch.int32, device=self.device)
            lcps = torch.empty(total, dtype=torch.int32, device=self.device)
        else:
            ids, lcps = out
            if ids.numel() < total or lcps.numel() < total:
                raise ValueError("output tensors are too small")
        stats = torch.empty((q.shape[0], 4), dtype=torch.int32, device=self.device)
        _check(lib.lcp_topk_stats(self._h, q.data_ptr(), q.shape[0], kk.ctypes.data, ids.data_ptr(),
                                  lcps.data_ptr(), stats.data_ptr(), _stream_handle(stream)))
        return TopK(ids, lcps, off), stats

    def scan_topk(self, queries, k: Union[int, Sequence[int], np.ndarray], stream=None, out=None) -> TopK:
        """Plain full-scan path (lcp_scan_topk)."""
        return self._run(lib.lcp_scan_topk, queries, k, stream, out)

    def bucket_scan_topk(self, queries, k: Union[int, Sequence[int], np.ndarray], depth: int, stream=None,
                         out=None, bounds: bool = False):
        """Prefix-bucket range scan (lcp_bucket_scan_topk): each query scans only the rows that share
        its first `depth` tokens.  With bounds=True returns (TopK, bounds), bounds an int32 [Q, 2]
        device tensor of each query's bucket [lo, hi) in sorted positions."""
        q, kk, off = self._prep(queries, k)
        total = int(off[-1])
        if out is None:
            ids = torch.empty(total, dtype=torch.int32, device=self.device)
            lcps = torch.empty(total, dtype=torch.int32, device=self.device)
        else:
            ids, lcps = out
            if ids.numel() < total or lcps.numel() < total:
                raise ValueError("output tensors are too small")
        b = torch.empty((q.shape[0], 2), dtype=torch.int32, device=self.device) if bounds else None
        _check(lib.lcp_bucket_scan_topk(self._h, q.data_ptr(), q.shape[0], int(depth), kk.ctypes.data,
                                        ids.data_ptr(), lcps.data_ptr(), b.data_ptr() if b is not None else None,
                                        _stream_handle(stream)))
        return (TopK(ids, lcps, off), b) if bounds else TopK(ids, lcps, off)

    def topk_dev(self, queries: torch.Tensor, k_dev: torch.Tensor, off_dev: torch.Tensor, k_max: int,
                 out_ids: torch.Tensor, out_lcp: torch.Tensor, stream=None, scan: bool = False,
                 noalloc: bool = False):
        """Device-k variant (lcp_topk_dev / lcp_scan_topk_dev): no host staging.  With scan=True and
        noalloc=True: lcp_scan_topk_dev_noalloc (fixed scratch, no allocation)."""
        q = _token_tensor(queries, self.token_bytes)
        if k_dev.dtype != torch.int32 or off_dev.dtype != torch.int64:
            raise TypeError("k_dev must be int32 and off_dev int64")
        if noalloc and not scan:
            raise ValueError("the allocation-free entry point is the full scan's (scan=True)")
        fn = (lib.lcp_scan_topk_dev_noalloc if noalloc else lib.lcp_scan_topk_dev) if scan else lib.lcp_topk_dev
        _check(fn(self._h, q.data_ptr(), q.shape[0], k_dev.data_ptr(), off_dev.data_ptr(), int(k_max),
                  out_ids.data_ptr(), out_lcp.data_ptr(), _stream_handle(stream)))

    def topk_persistent(self, queries: torch.Tensor, q_count_dev: torch.Tensor, k_dev: torch.Tensor,
                        off_dev: torch.Tensor, k_max: int, out_ids: torch.Tensor, out_lcp: torch.Tensor,
                        blocks: int = 0, stream=None):
        """Graph-capturable launch (lcp_topk_persistent); the batch size is *q_count_dev, at most
        the capacity queries.shape[0] (k_dev and off_dev hold at least that many entries)."""
        q = _token_tensor(queries, self.token_bytes)
        if q_count_dev.dtype != torch.int64 or k_dev.dtype != torch.int32 or off_dev.dtype != torch.int64:
            raise TypeError("q_count_dev and off_dev must be int64, k_dev int32")
        cap = int(q.shape[0])
        if k_dev.numel() < cap or off_dev.numel() < cap + 1:
            raise ValueError(f"k_dev and off_dev must hold {cap} and {cap + 1} entries")
        _check(lib.lcp_topk_persistent(self._h, q.data_ptr(), cap, q_count_dev.data_ptr(), k_dev.data_ptr(),
                                       off_dev.data_ptr(), int(k_max), out_ids.data_ptr(), out_lcp.data_ptr(),
                                       int(blocks), _stream_handle(stream)))

    def append(self, tokens, stream=None):
        """Append rows (ids N, N+1, ...); the index then equals a build over the concatenation."""
        if isinstance(tokens, np.ndarray):
            tokens = to_device_tokens(tokens, self.device)
        t = _token_tensor(tokens, self.token_bytes)
        if t.shape[1] != self.L:
            raise ValueError(f"rows have L={t.shape[1]}, index has L={self.L}")
        _check(lib.lcp_index_append(self._h, t.data_ptr(), t.shape[0], _stream_handle(stream)))
        n = ctypes.c_int64()
        _check(lib.lcp_index_info(self._h, ctypes.byref(n), None, None, None, None))
        self.N = n.value

    def set_search(self, mode: int):
        """Insertion-point search of the index path (lcp_index_set_search): 0 = 65-ary search tables,
        1 = first-token directory.  Answers are the same either way."""
        _check(lib.lcp_index_set_search(self._h, int(mode)))

    def search_mode(self) -> int:
        """The insertion-point search in use (lcp_index_search_mode): 0 tables, 1 directory."""
        m = ctypes.c_int32()
        _check(lib.lcp_index_search_mode(self._h, ctypes.byref(m)))
        return m.value

    def reserve(self, rows: int, stream=None):
        """Room for `rows` rows in total, so that later appends allocate nothing (lcp_index_reserve)."""
        _check(lib.lcp_index_reserve(self._h, int(rows), _stream_handle(stream)))

    def generation(self) -> int:
        """Changes of what queries read (lcp_index_generation); graphs captured at another value are stale."""
        g = ctypes.c_uint64()
        _check(lib.lcp_index_generation(self._h, ctypes.byref(g)))
        return g.value

    # ------------------------------------------------------------- tooling
    def views(self):
        """Copies of the index internals: perm, adjacent LCP, sorted key rows, id-order key rows."""
        p, a, s, r = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib.lcp_index_views(self._h, ctypes.byref(p), ctypes.byref(a), ctypes.byref(s), ctypes.byref(r)))
        dev = self.device
        perm = torch.empty(self.N, dtype=torch.int32, device=dev)
        A = torch.empty(self.N, dtype=torch.uint8, device=dev)
        srt = torch.empty((self.N, self.row_words), dtype=torch.int32, device=dev)
        rows = torch.empty((self.N, self.row_words), dtype=torch.int32, device=dev)
        torch.cuda.synchronize(dev)
        for dst, src, nbytes in ((perm, p, 4 * self.N), (A, a, self.N), (srt, s, 4 * self.N * self.row_words),
                                 (rows, r, 4 * self.N * self.row_words)):
            _hip_memcpy_d2d(dst.data_ptr(), src.value, nbytes)
        return {"perm": perm, "adj_lcp": A, "sorted_keys": srt, "id_keys": rows}

    def scan_info(self, Q: int, k_max: int):
        """Full-scan split for a batch: (query groups = passes over the rows, row chunks, seed rows)."""
        g, c, sr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib.lcp_scan_info(self._h, int(Q), int(k_max), ctypes.byref(g), ctypes.byref(c), ctypes.byref(sr)))
        return g.value, c.value, sr.value

    def set_kernel_timing(self, enable: bool):
        _check(lib.lcp_set_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time(self, which: int):
        """(total ms, launches) since the last read; which: 0 index kernel, 1 scan, 2 scan merge."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib.lcp_kernel_time(self._h, which, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib.lcp_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_hip = None


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(dst, src, nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")
