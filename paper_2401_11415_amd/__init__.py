"""MI355X (gfx950) neighbourhood-based link prediction: Python binding of liblp.so.

Argument marshalling only: every step of the prediction runs in the HIP
kernels of ``csrc/`` behind the C ABI of ``include/lp.h``.  PyTorch provides
device memory for outputs and the HIP stream.  The binding fails loudly when
the native library is missing; there is no CPU fallback.

Method: Sahu, "A Fast Parallel Approach for Neighborhood-based Link Prediction
by Disregarding Large Hubs" (arXiv 2401.11415): two-hop common-neighbour
accumulation per source (Section 4.1), hub limit L_H on intermediates
(Section 4.2), the nine measures of Section 3.1, top-N_P prediction
(Algorithm 1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["MEASURES", "HUB_NONE", "LpError", "Graph", "predict", "predict_multi", "query",
           "query_static", "fingerprint", "set_tuning", "last_stats", "Server", "library_path", "load",
           "BUCKET_MAX_DEFAULT"]

MEASURES = ("CN", "JC", "SI", "SC", "HP", "HD", "LHN", "AA", "RA")
HUB_NONE = (1 << 63) - 1  # L_H = infinity: IBase
# scheduling buckets of the accumulation, by wedges per source (lp_stats order),
# then the row of the 12-byte-table launch for AA / RA sources whose sums do
# not fit a packed slot
BUCKETS = ("tiny", "small", "mid1", "mid2", "mid3", "large", "global", "split")
LP_VALIDATE = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liblp.so")
_lib = None


class LpError(RuntimeError):
    def __init__(self, status: int, name: str, detail: str):
        super().__init__(f"{name}: {detail}")
        self.status = status
        self.name = name
        self.detail = detail


class _Tuning(ctypes.Structure):
    _fields_ = [("lds_wedge_cap", ctypes.c_int64), ("global_slots", ctypes.c_int64),
                ("sample_budget", ctypes.c_int64), ("bucket_max", ctypes.c_int64 * 5),
                ("batch_sources", ctypes.c_int64 * 2), ("kernel_shape", ctypes.c_int64 * 2),
                ("scratch_limit", ctypes.c_int64)]


class _BucketStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("sources", ctypes.c_uint64),
                ("first_order", ctypes.c_uint64), ("arcs", ctypes.c_uint64),
                ("wedges", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("ms", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("wedges", ctypes.c_uint64), ("sources", ctypes.c_uint64),
                ("bucket_sources", ctypes.c_uint64 * 8), ("appended", ctypes.c_uint64),
                ("retries", ctypes.c_uint64), ("ms_plan", ctypes.c_double),
                ("ms_accumulate", ctypes.c_double), ("ms_select", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("bucket", _BucketStats * 8),
                ("sampled", _BucketStats * 8)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch_sources", ctypes.c_int64),
                ("max_batch_paths", ctypes.c_int64), ("max_batch_bytes", ctypes.c_int64),
                ("host_launches", ctypes.c_int64)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("batch", ctypes.c_uint64),
                ("batch_requests", ctypes.c_uint32), ("replayed", ctypes.c_uint32),
                ("batch_sources", ctypes.c_uint64),
                ("batch_bytes", ctypes.c_uint64),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]


def library_path() -> str:
    return _LIB


def load():
    """Load liblp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise ImportError(f"{_LIB} is missing: build it with paper_2401_11415_amd/build.py")
    lib = ctypes.CDLL(_LIB)
    vp, i64, i32, u32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_float
    st = ctypes.c_int
    lib.lp_graph_create.restype = st
    lib.lp_graph_create.argtypes = [i64, vp, vp, u32, ctypes.POINTER(vp)]
    lib.lp_graph_destroy.restype = st
    lib.lp_graph_destroy.argtypes = [vp]
    lib.lp_graph_info.restype = st
    lib.lp_graph_info.argtypes = [vp, vp, vp, vp, vp]
    lib.lp_predict.restype = st
    lib.lp_predict.argtypes = [vp, ctypes.c_int, i64, i64, f32, vp, vp, vp, vp, vp]
    lib.lp_predict_multi.restype = st
    lib.lp_predict_multi.argtypes = [vp, i64, vp, vp, ctypes.c_int, i64, f32, vp, vp, vp, vp, vp]
    lib.lp_query.restype = st
    lib.lp_query.argtypes = [vp, vp, i64, ctypes.c_int, i64, i32, f32, vp, vp, vp, vp]
    lib.lp_query_static.restype = st
    lib.lp_query_static.argtypes = [vp, vp, i64, ctypes.c_int, i64, i32, f32, vp, vp, vp, vp]
    lib.lp_fingerprint.restype = st
    lib.lp_fingerprint.argtypes = [vp, i64, vp, vp]
    lib.lp_set_tuning.restype = st
    lib.lp_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.lp_last_stats.restype = st
    lib.lp_last_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
    lib.lp_server_create.restype = st
    lib.lp_server_create.argtypes = [vp, ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
    lib.lp_server_destroy.restype = st
    lib.lp_server_destroy.argtypes = [vp]
    lib.lp_server_submit.restype = st
    lib.lp_server_submit.argtypes = [vp, vp, i64, ctypes.c_int, i64, i32, f32, vp, vp, vp,
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.lp_server_wait.restype = st
    lib.lp_server_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(_RequestInfo)]
    lib.lp_status_string.restype = ctypes.c_char_p
    lib.lp_status_string.argtypes = [ctypes.c_int]
    lib.lp_last_error.restype = ctypes.c_char_p
    lib.lp_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        lib = load()
        raise LpError(status, lib.lp_status_string(status).decode(), lib.lp_last_error().decode())


def _measure(m) -> int:
    if isinstance(m, str):
        return MEASURES.index(m.upper())
    return int(m)


def _hub(L) -> int:
    return HUB_NONE if L is None else int(L)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(x):
    """Data pointer of a numpy array or torch tensor (host or device)."""
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    return ctypes.c_void_p(x.data_ptr())


class Graph:
    """A CSR graph resident on the current HIP device (lp_graph)."""

    def __init__(self, offsets, indices, validate: bool = False):
        lib = load()
        off = offsets
        idx = indices
        if isinstance(off, np.ndarray):
            off = np.ascontiguousarray(off, dtype=np.int64)
        if isinstance(idx, np.ndarray):
            idx = np.ascontiguousarray(idx, dtype=np.int32)
            if idx.size == 0:
                idx = np.zeros(1, np.int32)
        n = int(off.shape[0]) - 1
        h = ctypes.c_void_p()
        _check(lib.lp_graph_create(n, _ptr(off), _ptr(idx), LP_VALIDATE if validate else 0,
                                   ctypes.byref(h)))
        self._h = h
        self.n = n

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph is closed")
        return self._h

    def info(self):
        n, arcs, dmax, nbytes = (ctypes.c_int64() for _ in range(4))
        _check(load().lp_graph_info(self.handle, ctypes.byref(n), ctypes.byref(arcs),
                                    ctypes.byref(dmax), ctypes.byref(nbytes)))
        return {"n": n.value, "arcs": arcs.value, "max_degree": dmax.value,
                "device_bytes": nbytes.value}

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().lp_graph_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def predict(g: Graph, measure, hub_limit, k: int, score_threshold: float = 0.0, out=None,
            stream=None):
    """Top-k predicted edges: (a, c, score) int32/int32/float32 CUDA tensors of
    length k' = min(k, candidates), sorted by (score desc, a asc, c asc)."""
    import torch
    lib = load()
    k = int(k)
    if out is None:
        dev = torch.device("cuda", torch.cuda.current_device())
        out = (torch.empty(max(k, 1), dtype=torch.int32, device=dev),
               torch.empty(max(k, 1), dtype=torch.int32, device=dev),
               torch.empty(max(k, 1), dtype=torch.float32, device=dev))
    a, c, s = out
    cnt = ctypes.c_int64(0)
    _check(lib.lp_predict(g.handle, _measure(measure), _hub(hub_limit), k, float(score_threshold),
                          _ptr(a), _ptr(c), _ptr(s), ctypes.byref(cnt), _stream(stream)))
    n = cnt.value
    return a[:n], c[:n], s[:n]


def predict_multi(g: Graph, vstart, ks, measure, hub_limit, score_threshold: float = 0.0,
                  stream=None):
    """Several graphs in one call (lp_predict_multi).  vstart: ngraphs + 1
    original-id boundaries; ks: per-graph k.  Returns a list of per-graph
    (a, c, score) CUDA tensors of length k'_i."""
    import torch
    lib = load()
    vs = np.ascontiguousarray(np.asarray(vstart, dtype=np.int64))
    kk = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    ng = int(kk.shape[0])
    tot = int(kk.sum())
    dev = torch.device("cuda", torch.cuda.current_device())
    a = torch.empty(max(tot, 1), dtype=torch.int32, device=dev)
    c = torch.empty(max(tot, 1), dtype=torch.int32, device=dev)
    s = torch.empty(max(tot, 1), dtype=torch.float32, device=dev)
    cnt = np.zeros(ng, dtype=np.int64)
    _check(lib.lp_predict_multi(g.handle, ng, _ptr(vs), _ptr(kk), _measure(measure), _hub(hub_limit),
                                float(score_threshold), _ptr(a), _ptr(c), _ptr(s), _ptr(cnt),
                                _stream(stream)))
    out, off = [], 0
    for i in range(ng):
        n = int(cnt[i])
        out.append((a[off:off + n], c[off:off + n], s[off:off + n]))
        off += int(kk[i])
    return out


def query(g: Graph, sources, measure, hub_limit, k_q: int, score_threshold: float = 0.0,
          stream=None):
    """Per-source top-k_q recommendations: (c [ns, k_q] int32, score [ns, k_q]
    float32, count [ns] int32) CUDA tensors; row i holds count[i] entries."""
    import torch
    lib = load()
    dev = torch.device("cuda", torch.cuda.current_device())
    if isinstance(sources, np.ndarray) or isinstance(sources, (list, tuple)):
        src = torch.as_tensor(np.asarray(sources, dtype=np.int32), device=dev)
    else:
        src = sources.to(device=dev, dtype=torch.int32).contiguous()
    ns = int(src.shape[0])
    k_q = int(k_q)
    oc = torch.empty((max(ns, 1), k_q), dtype=torch.int32, device=dev)
    os_ = torch.empty((max(ns, 1), k_q), dtype=torch.float32, device=dev)
    on = torch.zeros(max(ns, 1), dtype=torch.int32, device=dev)
    _check(lib.lp_query(g.handle, _ptr(src), ns, _measure(measure), _hub(hub_limit), k_q,
                        float(score_threshold), _ptr(oc), _ptr(os_), _ptr(on), _stream(stream)))
    return oc[:ns], os_[:ns], on[:ns]


def query_static(g: Graph, sources, measure, hub_limit, k_q: int, score_threshold: float = 0.0,
                 out=None, stream=None):
    """lp_query_static: query() with every piece of device scratch taken from
    the library's fixed per-device array (no device allocation in the call).
    out = (c [ns, k_q] int32, score [ns, k_q] float32, count [ns] int32) CUDA
    tensors to fill; with out and sources given as CUDA int32 tensors the
    binding allocates nothing either.  Returns (c, score, count)."""
    import torch
    lib = load()
    dev = torch.device("cuda", torch.cuda.current_device())
    if isinstance(sources, np.ndarray) or isinstance(sources, (list, tuple)):
        src = torch.as_tensor(np.asarray(sources, dtype=np.int32), device=dev)
    elif sources.dtype == torch.int32 and sources.is_cuda and sources.is_contiguous():
        src = sources
    else:
        src = sources.to(device=dev, dtype=torch.int32).contiguous()
    ns = int(src.shape[0])
    k_q = int(k_q)
    if out is None:
        out = (torch.empty((max(ns, 1), k_q), dtype=torch.int32, device=dev),
               torch.empty((max(ns, 1), k_q), dtype=torch.float32, device=dev),
               torch.zeros(max(ns, 1), dtype=torch.int32, device=dev))
    oc, os_, on = out
    if ns > 0 and (oc.dtype != torch.int32 or os_.dtype != torch.float32 or on.dtype != torch.int32 or
                   oc.numel() < ns * k_q or os_.numel() < ns * k_q or on.numel() < ns or
                   not (oc.is_contiguous() and os_.is_contiguous() and on.is_contiguous())):
        raise ValueError("out must be contiguous (int32 [ns, k_q], float32 [ns, k_q], int32 [ns]) tensors")
    _check(lib.lp_query_static(g.handle, _ptr(src), ns, _measure(measure), _hub(hub_limit), k_q,
                               float(score_threshold), _ptr(oc), _ptr(os_), _ptr(on), _stream(stream)))
    return oc[:ns], os_[:ns], on[:ns]


def fingerprint(g: Graph, hub_limit, stream=None):
    """(|C_L|, sum h, sum mix64(a, c, h) mod 2^64, wedges) over all candidates."""
    out = (ctypes.c_uint64 * 4)()
    _check(load().lp_fingerprint(g.handle, _hub(hub_limit), out, _stream(stream)))
    return tuple(int(x) for x in out)


# default upper bounds of T = U + d_a for the buckets tiny .. mid3
BUCKET_MAX_DEFAULT = (32, 256, 1024, 2048, 4096)


# kernel shapes of the small and mid1 buckets (lp_tuning.kernel_shape)
SHAPES = {"batch": 1, "wave": 2, "workgroup128": 3, "workgroup256": 4}


def set_tuning(g: Graph, lds_wedge_cap: int = 0, global_slots: int = 0, sample_budget: int = 0,
               bucket_max=None, tiny_batch: int = 0, small_batch: int = 0, small_shape=0,
               mid1_shape=0, scratch_limit: int = 0):
    """Scheduler knobs of g (lp_set_tuning); 0 keeps a knob's default.
    bucket_max: up to five T bounds for tiny .. mid3, each at most its
    default (BUCKET_MAX_DEFAULT); tiny_batch / small_batch: sources per
    workgroup in the tiny (48 or 32) and small (8 or 4) buckets;
    small_shape / mid1_shape: the kernel of those buckets, a key of SHAPES
    or its number ("wave" is for the small bucket only); scratch_limit:
    largest single scratch allocation of a call, in bytes (forces
    LP_ERR_OUT_OF_MEMORY above it)."""
    bm = list(bucket_max or [])
    if len(bm) > 5:
        raise ValueError("bucket_max holds at most 5 bounds")
    bm += [0] * (5 - len(bm))
    shape = [SHAPES[x] if isinstance(x, str) else int(x) for x in (small_shape, mid1_shape)]
    t = _Tuning(lds_wedge_cap, global_slots, sample_budget, (ctypes.c_int64 * 5)(*bm),
                (ctypes.c_int64 * 2)(tiny_batch, small_batch), (ctypes.c_int64 * 2)(*shape),
                scratch_limit)
    _check(load().lp_set_tuning(g.handle, ctypes.byref(t)))


def last_stats(g: Graph) -> dict:
    s = _Stats()
    _check(load().lp_last_stats(g.handle, ctypes.byref(s)))
    launches, sampled = {}, {}
    for name, b, x in zip(BUCKETS, s.bucket, s.sampled):
        launches[name] = {f: getattr(b, f) for f, _ in _BucketStats._fields_}
        sampled[name] = {f: getattr(x, f) for f, _ in _BucketStats._fields_}
    return {"wedges": s.wedges, "sources": s.sources,
            "buckets": dict(zip(BUCKETS, list(s.bucket_sources))), "appended": s.appended,
            "retries": s.retries, "ms_plan": s.ms_plan, "ms_accumulate": s.ms_accumulate,
            "ms_select": s.ms_select, "ms_total": s.ms_total, "launches": launches,
            "sampled": sampled}


class Server:
    """Request loop over the per-source query (lp_server_*): submit() queues a
    request and returns a ticket; wait() returns (c [n, k_q], score [n, k_q],
    count [n]) numpy arrays and the request's timing / batch record."""

    def __init__(self, g: Graph, slots: int = 0, max_batch_sources: int = 0,
                 max_batch_paths: int = 0, max_batch_bytes: int = 0, host_launches: bool = False):
        lib = load()
        cfg = _ServerConfig(slots, max_batch_sources, max_batch_paths, max_batch_bytes,
                            1 if host_launches else 0)
        h = ctypes.c_void_p()
        _check(lib.lp_server_create(g.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._g = g  # the graph must outlive the server
        self._pending = {}

    def submit(self, sources, measure, hub_limit, k_q: int, score_threshold: float = 0.0) -> int:
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
        ns, k_q = int(src.shape[0]), int(k_q)
        out = (np.zeros((ns, k_q), np.int32), np.zeros((ns, k_q), np.float32),
               np.zeros(ns, np.int32))
        t = ctypes.c_uint64(0)
        _check(load().lp_server_submit(self._h, _ptr(src), ns, _measure(measure), _hub(hub_limit),
                                       k_q, float(score_threshold), _ptr(out[0]), _ptr(out[1]),
                                       _ptr(out[2]), ctypes.byref(t)))
        self._pending[t.value] = (src, out)  # keep the buffers alive until wait()
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        info = _RequestInfo()
        _check(load().lp_server_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(info)))
        _, out = self._pending.pop(int(ticket))
        rec = {f: getattr(info, f) for f, _ in _RequestInfo._fields_}
        return out, rec

    def close(self):
        if getattr(self, "_h", None) is not None:
            load().lp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
