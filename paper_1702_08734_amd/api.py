"""Thin Python binding of the C ABI declared in include/mi_knn.h.

Every function here only checks and marshals arguments (torch tensors are
used for device memory and the current HIP stream) and calls the library of
the same name; all computation runs in the library's HIP kernels.  If the
library has not been built, the first call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmiknn.so")
_lib = None

MK_OK = 0
_STATUS = {-1: "invalid argument", -2: "unsupported", -3: "out of memory", -4: "device error",
           -5: "bad state"}
METRICS = {"l2": 0, "ip": 1}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float


class MKError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {_STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


# name -> argtypes (restype int32 status unless listed in _RESTYPE)
_SIGS = {
    "mk_last_error": [],
    "mk_version": [],
    "mk_norms": [_vp, _i64, _i32, _vp, _vp],
    "mk_rotate_rows": [_vp, _i64, _i32, _vp, _i32, _vp, _vp],
    "mk_kselect": [_vp, _i64, _i64, _i32, _i32, _vp, _vp, _vp],
    "mk_knn_search": [_vp, _i64, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp],
    "mk_knn_search_noalloc": [_vp, _i64, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp],
    "mk_knn_search_host": [_vp, _i64, _vp, _i64, _i32, _i32, _i32, _i64, _vp, _vp, _vp],
    "mk_knn_graph": [_vp, _i64, _i32, _i32, _i32, _i64, _i64, _vp, _vp, _vp],
    "mk_ivfpq_knn_graph": [_vp, _vp, _i64, _i64, _i32, _i32, _i32, _vp, _vp, _vp],
    "mk_knn_search_prenorm": [_vp, _i64, _vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp],
    "mk_kmeans_assign": [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp],
    "mk_kmeans_update": [_vp, _i64, _i32, _vp, _i32, _vp, _vp, _vp],
    "mk_pq_encode": [_vp, _i64, _i32, _i32, _vp, _vp, _vp],
    "mk_ivfpq_create": [_i32, _i32, _i32, ctypes.POINTER(_vp)],
    "mk_ivfpq_destroy": [_vp],
    "mk_ivfpq_train": [_vp, _vp, _i64, _i32, _vp, _vp, _vp],
    "mk_ivfpq_add": [_vp, _vp, _i64, _vp],
    "mk_ivfpq_ntotal": [_vp],
    "mk_ivfpq_search": [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp],
    "mk_ivfpq_search_rerank": [_vp, _vp, _i64, _i32, _i32, _i32, _vp, _i64, _vp, _vp, _vp],
    "mk_ivfpq_get_quantizers": [_vp, _vp, _vp],
    "mk_ivfpq_set_quantizers": [_vp, _vp, _vp, _vp],
    "mk_ivfpq_get_lists": [_vp, _vp, _vp, _vp],
    "mk_ivfpq_set_scan_options": [_vp, _i32, _i32],
    "mk_ivfpq_shape": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "mk_ivfpq_save": [_vp, ctypes.c_char_p],
    "mk_ivfpq_load": [ctypes.c_char_p, ctypes.POINTER(_vp)],
    "mk_mlp_save": [_vp, ctypes.c_char_p],
    "mk_mlp_shape": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "mk_mlp_load": [ctypes.c_char_p, ctypes.POINTER(_vp)],
    "mk_lowp_stride": [_i32],
    "mk_quantize_rows": [_vp, _i64, _i32, _i32, _vp, _vp, _vp],
    "mk_knn_search_lowp": [_vp, _i64, _vp, _vp, _vp, _vp, _i64, _i32, _i32, _i32, _i32, _i32,
                           _vp, _vp, _vp],
    "mk_mlp_create": [_i32, _i32, _i32, ctypes.POINTER(_vp)],
    "mk_mlp_destroy": [_vp],
    "mk_mlp_num_params": [_vp],
    "mk_mlp_set_params": [_vp, _vp],
    "mk_mlp_get_params": [_vp, _vp, _vp],
    "mk_mlp_fit_standardization": [_vp, _vp, _i64, _vp],
    "mk_mlp_get_standardization": [_vp, _vp, _vp],
    "mk_mlp_forward": [_vp, _vp, _i64, _vp, _vp],
    "mk_mlp_loss_grad": [_vp, _vp, _vp, _i64, _vp, _vp, _vp],
    "mk_mlp_train_epoch": [_vp, _vp, _i64, _vp, _vp, _i32, _f32, _vp, _vp],
    "mk_ivfpq_probe_features": [_vp, _vp, _i64, _vp, _vp],
    "mk_ivfpq_probe_labels": [_vp, _vp, _i64, _vp, _i32, _vp, _vp, _vp],
    "mk_ivfpq_search_learned": [_vp, _vp, _f32, _vp, _i64, _i32, _i32, _i32, _vp, _i64, _vp, _vp,
                                _vp, _vp],
    "mk_ivfpq_dim": [_vp],
    "mk_ivfpq_search_workspace_bytes": [_vp, _i64, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_size_t)],
    "mk_server_create": [_vp, _vp, ctypes.POINTER(_vp)],
    "mk_server_submit": [_vp, _vp, _i64, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)],
    "mk_server_wait": [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)],
    "mk_server_stats": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "mk_server_destroy": [_vp],
    "mk_debug_pool_drops": [ctypes.POINTER(_i64)],
    "mk_profile_enable": [_i32],
    "mk_profile_read": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)],
}
_RESTYPE = {"mk_last_error": ctypes.c_char_p, "mk_ivfpq_destroy": None, "mk_mlp_destroy": None,
            "mk_mlp_num_params": ctypes.c_int64, "mk_ivfpq_dim": ctypes.c_int32,
            "mk_server_destroy": None,
            "mk_ivfpq_ntotal": ctypes.c_int64, "mk_lowp_stride": ctypes.c_int32}
PRECISIONS = {"bf16": 1, "fp8": 2}


def lib():
    """Open the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1702_08734_amd.build` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = _RESTYPE.get(name, ctypes.c_int32)
    _lib = L
    return L


def _call(name: str, *args) -> None:
    st = getattr(lib(), name)(*args)
    if st != MK_OK:
        msg = lib().mk_last_error()
        raise MKError(name, st, msg.decode() if msg else "")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None or t.numel() == 0 else t.data_ptr()


def _out(shape, dtype, like: torch.Tensor) -> torch.Tensor:
    return torch.empty(shape, dtype=dtype, device=like.device)


def norms(x: torch.Tensor) -> torch.Tensor:
    _dev(x, torch.float32, "x")
    out = _out((x.shape[0],), torch.float32, x)
    _call("mk_norms", _ptr(x), x.shape[0], x.shape[1], _ptr(out), _stream())
    return out


def rotate_rows(x: torch.Tensor, rot: torch.Tensor) -> torch.Tensor:
    """out[i][j] = sum_t rot[j][t] x[i][t] (an OPQ rotation or projection)."""
    _dev(x, torch.float32, "x")
    _dev(rot, torch.float32, "rot")
    if rot.dim() != 2 or rot.shape[1] != x.shape[1]:
        raise ValueError("rot must be [dout, d] with d = x.shape[1]")
    out = _out((x.shape[0], rot.shape[0]), torch.float32, x)
    _call("mk_rotate_rows", _ptr(x), x.shape[0], x.shape[1], _ptr(rot), rot.shape[0], _ptr(out),
          _stream())
    return out


def kselect(a: torch.Tensor, k: int, largest: bool = False):
    """Row-wise k smallest (or largest) values and their column indices."""
    _dev(a, torch.float32, "a")
    nrows, length = a.shape
    vals = _out((nrows, k), torch.float32, a)
    idx = _out((nrows, k), torch.int64, a)
    _call("mk_kselect", _ptr(a), nrows, length, k, int(bool(largest)), _ptr(vals), _ptr(idx),
          _stream())
    return vals, idx


def knn_search(xq: torch.Tensor, xb: torch.Tensor, k: int, metric: str = "l2",
               yn: torch.Tensor | None = None):
    """Exact k-NN: (D [nq, k] float32, I [nq, k] int64)."""
    _dev(xq, torch.float32, "xq")
    _dev(xb, torch.float32, "xb")
    nq, d = xq.shape
    nb = xb.shape[0]
    if nb and xb.shape[1] != d:
        raise ValueError("xq and xb dimensions differ")
    D = _out((nq, k), torch.float32, xq)
    I = _out((nq, k), torch.int64, xq)
    if yn is None:
        _call("mk_knn_search", _ptr(xq), nq, _ptr(xb), nb, d, k, METRICS[metric], _ptr(D),
              _ptr(I), _stream())
    else:
        _dev(yn, torch.float32, "yn")
        _call("mk_knn_search_prenorm", _ptr(xq), nq, _ptr(xb), _ptr(yn), nb, d, k,
              METRICS[metric], _ptr(D), _ptr(I), _stream())
    return D, I


def knn_search_host(xq: torch.Tensor, xb_host: torch.Tensor, k: int, metric: str = "l2",
                    chunk_rows: int = 1 << 20):
    """Exact k-NN against a host-resident (ideally pinned) database streamed
    to the device in chunks of chunk_rows rows; synchronises the stream."""
    _dev(xq, torch.float32, "xq")
    if not isinstance(xb_host, torch.Tensor) or xb_host.is_cuda:
        raise ValueError("xb_host must be a CPU tensor")
    if xb_host.dtype != torch.float32 or not xb_host.is_contiguous():
        raise ValueError("xb_host must be contiguous float32")
    nq, d = xq.shape
    nb = xb_host.shape[0]
    if nb and xb_host.shape[1] != d:
        raise ValueError("xq and xb_host dimensions differ")
    D = _out((nq, k), torch.float32, xq)
    I = _out((nq, k), torch.int64, xq)
    _call("mk_knn_search_host", _ptr(xq), nq, _ptr(xb_host), nb, d, k, METRICS[metric],
          chunk_rows, _ptr(D), _ptr(I), _stream())
    return D, I


def knn_graph(xb: torch.Tensor, k: int, metric: str = "l2", node0: int = 0,
              nnodes: int | None = None):
    """Rows node0 .. node0 + nnodes - 1 of the exact k-NN graph of xb (a node
    is not its own neighbour): (D [nnodes, k], I [nnodes, k])."""
    _dev(xb, torch.float32, "xb")
    nb, d = xb.shape
    nnodes = nb - node0 if nnodes is None else nnodes
    D = _out((nnodes, k), torch.float32, xb)
    I = _out((nnodes, k), torch.int64, xb)
    _call("mk_knn_graph", _ptr(xb), nb, d, k, METRICS[metric], node0, nnodes, _ptr(D), _ptr(I),
          _stream())
    return D, I


def knn_search_noalloc(xq: torch.Tensor, xb: torch.Tensor, k: int, metric: str = "l2",
                       D: torch.Tensor | None = None, I: torch.Tensor | None = None):
    """Exact k-NN through the allocation-free entry point (the library's fixed
    scratch array); D and I may be passed in preallocated."""
    _dev(xq, torch.float32, "xq")
    _dev(xb, torch.float32, "xb")
    nq, d = xq.shape
    nb = xb.shape[0]
    if nb and xb.shape[1] != d:
        raise ValueError("xq and xb dimensions differ")
    D = _out((nq, k), torch.float32, xq) if D is None else _dev(D, torch.float32, "D")
    I = _out((nq, k), torch.int64, xq) if I is None else _dev(I, torch.int64, "I")
    if tuple(D.shape) != (nq, k) or tuple(I.shape) != (nq, k):
        raise ValueError("D and I must be [nq, k]")
    _call("mk_knn_search_noalloc", _ptr(xq), nq, _ptr(xb), nb, d, k, METRICS[metric], _ptr(D),
          _ptr(I), _stream())
    return D, I


def quantize_rows(x: torch.Tensor, prec: str):
    """Low-precision copy of the rows of x: (uint8 tensor [n, ld * bytes],
    float32 1/scale per row)."""
    _dev(x, torch.float32, "x")
    n, d = x.shape
    ld = int(lib().mk_lowp_stride(d))
    nbytes = 2 if prec == "bf16" else 1
    out = _out((n, ld * nbytes), torch.uint8, x)
    inv = _out((n,), torch.float32, x)
    _call("mk_quantize_rows", _ptr(x), n, d, PRECISIONS[prec], _ptr(out), _ptr(inv), _stream())
    return out, inv


def knn_search_lowp(xq: torch.Tensor, xb: torch.Tensor, xb_lp: torch.Tensor, xb_inv: torch.Tensor,
                    k: int, rerank: int, prec: str, metric: str = "l2",
                    yn: torch.Tensor | None = None):
    """Low-precision brute force + exact FP32 re-rank of `rerank` candidates."""
    _dev(xq, torch.float32, "xq")
    _dev(xb, torch.float32, "xb")
    _dev(xb_lp, torch.uint8, "xb_lp")
    _dev(xb_inv, torch.float32, "xb_inv")
    nq, d = xq.shape
    nb = xb.shape[0]
    D = _out((nq, k), torch.float32, xq)
    I = _out((nq, k), torch.int64, xq)
    if yn is not None:
        _dev(yn, torch.float32, "yn")
    _call("mk_knn_search_lowp", _ptr(xq), nq, _ptr(xb), _ptr(xb_lp), _ptr(xb_inv), _ptr(yn), nb,
          d, k, rerank, METRICS[metric], PRECISIONS[prec], _ptr(D), _ptr(I), _stream())
    return D, I


def kmeans_assign(x: torch.Tensor, c: torch.Tensor):
    _dev(x, torch.float32, "x")
    _dev(c, torch.float32, "c")
    n, d = x.shape
    a = _out((n,), torch.int64, x)
    dist = _out((n,), torch.float32, x)
    _call("mk_kmeans_assign", _ptr(x), n, d, _ptr(c), c.shape[0], _ptr(a), _ptr(dist), _stream())
    return a, dist


def kmeans_update(x: torch.Tensor, assign: torch.Tensor, c: torch.Tensor):
    """Returns (new centroids, counts); c itself is left unchanged."""
    _dev(x, torch.float32, "x")
    _dev(assign, torch.int64, "assign")
    _dev(c, torch.float32, "c")
    n, d = x.shape
    cn = c.clone()
    counts = _out((c.shape[0],), torch.int64, x)
    _call("mk_kmeans_update", _ptr(x), n, d, _ptr(assign), c.shape[0], _ptr(cn), _ptr(counts),
          _stream())
    return cn, counts


def pq_encode(r: torch.Tensor, codebooks: torch.Tensor) -> torch.Tensor:
    _dev(r, torch.float32, "r")
    _dev(codebooks, torch.float32, "codebooks")
    n, d = r.shape
    M = codebooks.shape[0]
    codes = _out((n, M), torch.uint8, r)
    _call("mk_pq_encode", _ptr(r), n, d, M, _ptr(codebooks), _ptr(codes), _stream())
    return codes


class IVFPQ:
    """Resident IVFADC index (coarse k-means + 8-bit PQ on residuals, L2)."""

    def __init__(self, d: int, nlist: int, M: int, _handle=None):
        self.d, self.nlist, self.M = d, nlist, M
        if _handle is not None:
            self._h = _handle
            return
        h = _vp()
        _call("mk_ivfpq_create", d, nlist, M, ctypes.byref(h))
        self._h = h

    def set_scan_options(self, lut: str = "fp32", lists_per_group: int = 0) -> None:
        """List-scan options: lookup tables in "fp32" or "fp16"; probed lists
        per workgroup (0 automatic, -1 all of a query's lists, or a count)."""
        _call("mk_ivfpq_set_scan_options", self._h, {"fp32": 0, "fp16": 3}[lut],
              int(lists_per_group))

    def save(self, path: str) -> None:
        """Write the trained index (quantizers and lists) to `path`."""
        _call("mk_ivfpq_save", self._h, os.fsencode(path))

    @classmethod
    def load(cls, path: str) -> "IVFPQ":
        """An index read from a file written by save()."""
        h = _vp()
        _call("mk_ivfpq_load", os.fsencode(path), ctypes.byref(h))
        d, nlist, M = _i32(), _i32(), _i32()
        _call("mk_ivfpq_shape", h, ctypes.byref(d), ctypes.byref(nlist), ctypes.byref(M))
        return cls(d.value, nlist.value, M.value, _handle=h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mk_ivfpq_destroy(h)
            self._h = None

    @property
    def ntotal(self) -> int:
        return int(lib().mk_ivfpq_ntotal(self._h))

    def train(self, xt: torch.Tensor, niter: int, coarse_init_rows, pq_init_rows) -> None:
        import numpy as np
        _dev(xt, torch.float32, "xt")
        ci = np.ascontiguousarray(coarse_init_rows, np.int64)
        pi = np.ascontiguousarray(pq_init_rows, np.int64)
        if ci.shape != (self.nlist,) or pi.shape != (self.M, 256):
            raise ValueError("init rows must be [nlist] and [M, 256]")
        _call("mk_ivfpq_train", self._h, _ptr(xt), xt.shape[0], niter, ci.ctypes.data,
              pi.ctypes.data, _stream())

    def add(self, xb: torch.Tensor) -> None:
        _dev(xb, torch.float32, "xb")
        _call("mk_ivfpq_add", self._h, _ptr(xb), xb.shape[0], _stream())

    def search(self, xq: torch.Tensor, k: int, nprobe: int):
        _dev(xq, torch.float32, "xq")
        nq = xq.shape[0]
        D = _out((nq, k), torch.float32, xq)
        I = _out((nq, k), torch.int64, xq)
        _call("mk_ivfpq_search", self._h, _ptr(xq), nq, k, nprobe, _ptr(D), _ptr(I), _stream())
        return D, I

    def knn_graph(self, xb: torch.Tensor, k: int, nprobe: int, node0: int = 0,
                  nnodes: int | None = None, R: int = 0):
        """Rows node0 .. node0 + nnodes - 1 of the IVFADC k-NN graph of the
        added vectors xb (ids 0 .. ntotal - 1); a node is not its own
        neighbour.  R > 0 re-ranks an R-entry ADC short list exactly."""
        _dev(xb, torch.float32, "xb")
        if xb.dim() != 2 or xb.shape[1] != self.d or xb.shape[0] < self.ntotal:
            raise ValueError(f"xb must be the [ntotal, {self.d}] added vectors")
        nnodes = self.ntotal - node0 if nnodes is None else nnodes
        D = _out((nnodes, k), torch.float32, xb)
        I = _out((nnodes, k), torch.int64, xb)
        _call("mk_ivfpq_knn_graph", self._h, _ptr(xb), node0, nnodes, k, nprobe, R, _ptr(D),
              _ptr(I), _stream())
        return D, I

    def search_rerank(self, xq: torch.Tensor, k: int, nprobe: int, R: int, xb: torch.Tensor):
        """ADC short list of R entries, re-ranked exactly against xb[id]."""
        _dev(xq, torch.float32, "xq")
        _dev(xb, torch.float32, "xb")
        if xb.dim() != 2 or xb.shape[1] != self.d or xq.dim() != 2 or xq.shape[1] != self.d:
            raise ValueError(f"xq and xb must be [n, {self.d}]")
        nq = xq.shape[0]
        D = _out((nq, k), torch.float32, xq)
        I = _out((nq, k), torch.int64, xq)
        _call("mk_ivfpq_search_rerank", self._h, _ptr(xq), nq, k, nprobe, R, _ptr(xb),
              xb.shape[0], _ptr(D), _ptr(I), _stream())
        return D, I

    def workspace_bytes(self, nq: int, k: int, nprobe: int, R: int = 0) -> int:
        b = ctypes.c_size_t()
        _call("mk_ivfpq_search_workspace_bytes", self._h, nq, k, nprobe, R, ctypes.byref(b))
        return int(b.value)

    def probe_features(self, xq: torch.Tensor) -> torch.Tensor:
        """[xq ; its 32 smallest squared coarse distances] per query."""
        _dev(xq, torch.float32, "xq")
        F = _out((xq.shape[0], self.d + 32), torch.float32, xq)
        _call("mk_ivfpq_probe_features", self._h, _ptr(xq), xq.shape[0], _ptr(F), _stream())
        return F

    def probe_labels(self, xq: torch.Tensor, nn_ids: torch.Tensor, cap: int):
        """(target = log2(label), label): rank of the list of each query's
        nearest neighbour in its coarse order, at most cap."""
        _dev(xq, torch.float32, "xq")
        _dev(nn_ids, torch.int64, "nn_ids")
        nq = xq.shape[0]
        target = _out((nq,), torch.float32, xq)
        label = _out((nq,), torch.int32, xq)
        _call("mk_ivfpq_probe_labels", self._h, _ptr(xq), nq, _ptr(nn_ids), cap, _ptr(target),
              _ptr(label), _stream())
        return target, label

    def search_learned(self, net: "MLP", delta: float, xq: torch.Tensor, k: int, cap: int,
                       R: int = 0, xb: torch.Tensor | None = None):
        """Search with the predicted per-query probe count; (D, I, tau)."""
        _dev(xq, torch.float32, "xq")
        if xb is not None:
            _dev(xb, torch.float32, "xb")
        nq = xq.shape[0]
        D = _out((nq, k), torch.float32, xq)
        I = _out((nq, k), torch.int64, xq)
        tau = _out((nq,), torch.int32, xq)
        _call("mk_ivfpq_search_learned", self._h, net._h, delta, _ptr(xq), nq, k, cap, R,
              _ptr(xb), xb.shape[0] if xb is not None else 0, _ptr(D), _ptr(I), _ptr(tau),
              _stream())
        return D, I, tau

    def get_quantizers(self):
        import numpy as np
        coarse = np.empty((self.nlist, self.d), np.float32)
        books = np.empty((self.M, 256, self.d // self.M), np.float32)
        _call("mk_ivfpq_get_quantizers", self._h, coarse.ctypes.data, books.ctypes.data)
        return coarse, books

    def set_quantizers(self, coarse, books) -> None:
        import numpy as np
        c = np.ascontiguousarray(coarse, np.float32)
        b = np.ascontiguousarray(books, np.float32)
        _call("mk_ivfpq_set_quantizers", self._h, c.ctypes.data, b.ctypes.data, _stream())

    def get_lists(self):
        import numpy as np
        n = self.ntotal
        offs = np.empty(self.nlist + 1, np.int64)
        codes = np.empty((max(n, 1), self.M), np.uint8)
        ids = np.empty(max(n, 1), np.int64)
        _call("mk_ivfpq_get_lists", self._h, offs.ctypes.data, codes.ctypes.data, ids.ctypes.data)
        return offs, codes[:n], ids[:n]


def debug_pool_drops() -> int:
    """Candidates dropped by full candidate pools so far (must be 0)."""
    n = _i64()
    _call("mk_debug_pool_drops", ctypes.byref(n))
    return n.value


def profile_enable(on: bool = True) -> None:
    """Start (clearing earlier records) or stop per-launch kernel timing."""
    _call("mk_profile_enable", int(bool(on)))


def profile_read(name: str):
    """(total device milliseconds, launches) recorded for kernel `name`."""
    ms = ctypes.c_double()
    n = _i64()
    _call("mk_profile_read", name.encode(), ctypes.byref(ms), ctypes.byref(n))
    return ms.value, n.value


class MLP:
    """Probe-count predictor: din -> hidden (ReLU) -> hidden (ReLU) -> 1."""

    def __init__(self, din: int, hidden: int, prec: str = "fp32", _handle=None):
        self.din, self.hidden = din, hidden
        h = _handle
        if h is None:
            h = _vp()
            _call("mk_mlp_create", din, hidden, {"fp32": 0, "bf16": 1}[prec], ctypes.byref(h))
        self._h = h
        self.n_params = int(lib().mk_mlp_num_params(h))

    def save(self, path: str) -> None:
        """Write parameters, Adam state and standardisation to `path`."""
        _call("mk_mlp_save", self._h, os.fsencode(path))

    @classmethod
    def load(cls, path: str) -> "MLP":
        h = _vp()
        _call("mk_mlp_load", os.fsencode(path), ctypes.byref(h))
        din, hidden, prec = _i32(), _i32(), _i32()
        _call("mk_mlp_shape", h, ctypes.byref(din), ctypes.byref(hidden), ctypes.byref(prec))
        return cls(din.value, hidden.value, {0: "fp32", 1: "bf16"}[prec.value], _handle=h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mk_mlp_destroy(h)
            self._h = None

    def set_params(self, theta) -> None:
        import numpy as np
        t = np.ascontiguousarray(theta, np.float32)
        if t.shape != (self.n_params,):
            raise ValueError(f"theta must have {self.n_params} entries")
        _call("mk_mlp_set_params", self._h, t.ctypes.data)

    def get_params(self):
        """(theta, last gradient) as float32 numpy arrays."""
        import numpy as np
        t = np.empty(self.n_params, np.float32)
        g = np.empty(self.n_params, np.float32)
        _call("mk_mlp_get_params", self._h, t.ctypes.data, g.ctypes.data)
        return t, g

    def fit_standardization(self, F: torch.Tensor) -> None:
        _dev(F, torch.float32, "F")
        _call("mk_mlp_fit_standardization", self._h, _ptr(F), F.shape[0], _stream())

    def get_standardization(self):
        import numpy as np
        m = np.empty(self.din, np.float32)
        s = np.empty(self.din, np.float32)
        _call("mk_mlp_get_standardization", self._h, m.ctypes.data, s.ctypes.data)
        return m, s

    def forward(self, F: torch.Tensor) -> torch.Tensor:
        _dev(F, torch.float32, "F")
        y = _out((F.shape[0],), torch.float32, F)
        _call("mk_mlp_forward", self._h, _ptr(F), F.shape[0], _ptr(y), _stream())
        return y

    def loss_grad(self, F: torch.Tensor, y: torch.Tensor, rows: torch.Tensor | None = None):
        """Batch loss (device scalar); the gradient stays in the network."""
        _dev(F, torch.float32, "F")
        _dev(y, torch.float32, "y")
        if rows is not None:
            _dev(rows, torch.int64, "rows")
        B = rows.shape[0] if rows is not None else F.shape[0]
        loss = _out((1,), torch.float32, F)
        _call("mk_mlp_loss_grad", self._h, _ptr(F), _ptr(rows), B, _ptr(y), _ptr(loss),
              _stream())
        return loss

    def train_epoch(self, F: torch.Tensor, y: torch.Tensor, perm: torch.Tensor, batch: int,
                    lr: float = 1e-3) -> torch.Tensor:
        _dev(F, torch.float32, "F")
        _dev(y, torch.float32, "y")
        _dev(perm, torch.int64, "perm")
        n = F.shape[0]
        losses = _out(((n + batch - 1) // batch,), torch.float32, F)
        _call("mk_mlp_train_epoch", self._h, _ptr(F), n, _ptr(y), _ptr(perm), batch, lr,
              _ptr(losses), _stream())
        return losses


class _ServerConfig(ctypes.Structure):
    _fields_ = [("k", _i32), ("nprobe", _i32), ("R", _i32), ("max_batch", _i32),
                ("nstreams", _i32), ("cap", _i32), ("delta", _f32), ("net", _vp), ("xb", _vp),
                ("nb", _i64), ("workspace_budget", _i64)]


class Server:
    """Continuous-batching search loop over a resident IVFPQ index.

    submit() takes host float32 query rows and returns a ticket; wait(ticket)
    blocks until the request is done and returns (D, I, latency seconds)."""

    def __init__(self, index: IVFPQ, k: int, nprobe: int = 1, R: int = 0, max_batch: int = 1024,
                 nstreams: int = 2, net: MLP | None = None, delta: float = 0.0, cap: int = 0,
                 xb: torch.Tensor | None = None, workspace_budget: int = 0):
        if xb is not None:
            _dev(xb, torch.float32, "xb")
        self.index, self.k, self.d = index, k, index.d
        self._keep = (index, net, xb)
        cfg = _ServerConfig(k, nprobe, R, max_batch, nstreams, cap, delta,
                            net._h.value if net is not None else None,
                            _ptr(xb), xb.shape[0] if xb is not None else 0, workspace_budget)
        h = _vp()
        _call("mk_server_create", index._h, ctypes.byref(cfg), ctypes.byref(h))
        self._h = h
        self._pending = {}

    def submit(self, xq) -> int:
        import numpy as np
        q = np.ascontiguousarray(xq, np.float32)
        if q.ndim != 2 or q.shape[1] != self.d:
            raise ValueError(f"xq must be [n, {self.d}]")
        D = np.empty((q.shape[0], self.k), np.float32)
        I = np.empty((q.shape[0], self.k), np.int64)
        t = ctypes.c_uint64()
        _call("mk_server_submit", self._h, q.ctypes.data, q.shape[0], D.ctypes.data,
              I.ctypes.data, ctypes.byref(t))
        self._pending[t.value] = (q, D, I)  # keeps the host buffers alive
        return t.value

    def wait(self, ticket: int):
        lat = ctypes.c_double()
        try:
            _call("mk_server_wait", self._h, ticket, ctypes.byref(lat))
        finally:
            bufs = self._pending.pop(ticket, None)
        _, D, I = bufs
        return D, I, lat.value

    def stats(self):
        b, r = _i64(), _i64()
        _call("mk_server_stats", self._h, ctypes.byref(b), ctypes.byref(r))
        return b.value, r.value

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mk_server_destroy(h)
            self._h = None

    def __del__(self):
        self.close()
