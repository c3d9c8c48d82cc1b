"""CPU oracle for neighbourhood-based link prediction (IBase / DLH), FP64.

TEST INFRASTRUCTURE ONLY: the product path never imports this package.  Only
``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may use it.  It shares no code with the GPU implementation.

Two routes over the same definition (Sahu, arXiv 2401.11415):

* ``bruteforce`` / ``pair`` (O0): every pair a < c, h by merge intersection of
  sorted neighbour lists restricted to explored intermediates d_b <= L
  (Section 3.3 baseline + Section 4.2.1 hub limit).
* ``source`` / ``predict`` / ``query`` / ``fingerprint`` (O1): the paper's
  two-hop accumulation per source into a dense per-thread table (Section 4.1,
  Algorithm 1), first-order neighbours cleared, scores from Section 3.1,
  per-thread top-N_P heaps merged, ties ordered (fp32 score desc, a asc, c asc).

``pybrute.py`` holds a third, pure-Python route for tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

MEASURES = ("CN", "JC", "SI", "SC", "HP", "HD", "LHN", "AA", "RA")
HUB_NONE = np.iinfo(np.int64).max  # L = infinity: IBase

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", src,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("LP_ORACLE_LIB", _LIB_PATH)  # tests may point at a mutated build
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(path)
    vp, i64, i32, f32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_float, ctypes.c_double)
    lib.oracle_weight.restype = dbl
    lib.oracle_weight.argtypes = [ctypes.c_int, i64]
    lib.oracle_score.restype = dbl
    lib.oracle_score.argtypes = [ctypes.c_int, i64, dbl, i64, i64]
    lib.oracle_pair.restype = ctypes.c_int
    lib.oracle_pair.argtypes = [i64, vp, vp, i64, ctypes.c_int, i64, i64, vp, vp]
    lib.oracle_pairs.restype = None
    lib.oracle_pairs.argtypes = [i64, vp, vp, i64, ctypes.c_int, vp, vp, i64, ctypes.c_int, vp, vp, vp]
    lib.oracle_bruteforce.restype = i64
    lib.oracle_bruteforce.argtypes = [i64, vp, vp, i64, ctypes.c_int, vp, vp, vp, vp, i64]
    lib.oracle_source.restype = i64
    lib.oracle_source.argtypes = [i64, vp, vp, i64, ctypes.c_int, i64, ctypes.c_int, vp, vp, vp, i64]
    lib.oracle_predict.restype = i64
    lib.oracle_predict.argtypes = [i64, vp, vp, i64, ctypes.c_int, i64, f32, ctypes.c_int,
                                   vp, vp, vp, vp]
    lib.oracle_predict_sources.restype = i64
    lib.oracle_predict_sources.argtypes = [i64, vp, vp, i64, ctypes.c_int, i64, f32, ctypes.c_int,
                                           vp, i64, vp, vp, vp, vp]
    lib.oracle_query.restype = ctypes.c_int
    lib.oracle_query.argtypes = [i64, vp, vp, i64, ctypes.c_int, vp, i64, i32, f32,
                                 ctypes.c_int, vp, vp, vp, vp]
    lib.oracle_fingerprint.restype = ctypes.c_int
    lib.oracle_fingerprint.argtypes = [i64, vp, vp, i64, ctypes.c_int, vp]
    _lib = lib
    return lib


def measure_id(m) -> int:
    if isinstance(m, str):
        return MEASURES.index(m.upper())
    return int(m)


def _hub(L) -> int:
    return HUB_NONE if L is None else int(L)


def _arrays(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    if idx.shape[0] == 0:
        idx = np.zeros(1, dtype=np.int32)
    return off, idx


def score(m, h: int, w: float, da: int, dc: int) -> float:
    return _load().oracle_score(measure_id(m), h, w, da, dc)


def weight(m, db: int) -> float:
    return _load().oracle_weight(measure_id(m), db)


def pair(g, L, m, a: int, c: int):
    """(is_candidate, h, fp64 score) for one unordered pair, by definition."""
    off, idx = _arrays(g)
    h = ctypes.c_int64(0)
    s = ctypes.c_double(0)
    ok = _load().oracle_pair(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m),
                             a, c, ctypes.addressof(h), ctypes.addressof(s))
    return bool(ok), h.value, s.value


def pairs(g, L, m, a, c, threads: int = 0):
    """``pair`` for many unordered pairs: (is_candidate bool[], h int64[], fp64 score[])."""
    off, idx = _arrays(g)
    a = np.ascontiguousarray(a, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    assert a.shape == c.shape
    npairs = a.shape[0]
    ok = np.zeros(max(npairs, 1), np.int8)
    h = np.zeros(max(npairs, 1), np.int64)
    s = np.zeros(max(npairs, 1), np.float64)
    if npairs:
        _load().oracle_pairs(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m),
                             a.ctypes.data, c.ctypes.data, npairs, int(threads), ok.ctypes.data,
                             h.ctypes.data, s.ctypes.data)
    return ok[:npairs].astype(bool), h[:npairs], s[:npairs]


def bruteforce(g, L, m):
    """All candidates a < c by definition: dict with arrays a, c, h, s (fp64)."""
    lib = _load()
    off, idx = _arrays(g)
    args = (g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m))
    total = lib.oracle_bruteforce(*args, None, None, None, None, 0)
    a = np.zeros(max(total, 1), np.int32)
    c = np.zeros(max(total, 1), np.int32)
    h = np.zeros(max(total, 1), np.int64)
    s = np.zeros(max(total, 1), np.float64)
    lib.oracle_bruteforce(*args, a.ctypes.data, c.ctypes.data, h.ctypes.data, s.ctypes.data, total)
    return {"a": a[:total], "c": c[:total], "h": h[:total], "s": s[:total]}


def source(g, L, m, a: int, mode: str = "predict"):
    """Candidates of one source via the two-hop algorithm, sorted by c."""
    lib = _load()
    off, idx = _arrays(g)
    md = 0 if mode == "predict" else 1
    cap = max(g.n, 1)
    c = np.zeros(cap, np.int32)
    h = np.zeros(cap, np.int64)
    s = np.zeros(cap, np.float64)
    r = lib.oracle_source(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m), a, md,
                          c.ctypes.data, h.ctypes.data, s.ctypes.data, cap)
    if r < 0:
        raise MemoryError("oracle_source")
    o = np.argsort(c[:r], kind="stable")
    return {"c": c[:r][o], "h": h[:r][o], "s": s[:r][o]}


def predict(g, L, m, k: int, s_th: float = 0.0, threads: int = 0):
    """Top-k prediction: dict with a, c (a < c), s32 (fp32), s64 (fp64)."""
    lib = _load()
    off, idx = _arrays(g)
    kk = max(int(k), 0)
    a = np.zeros(max(kk, 1), np.int32)
    c = np.zeros(max(kk, 1), np.int32)
    s32 = np.zeros(max(kk, 1), np.float32)
    s64 = np.zeros(max(kk, 1), np.float64)
    r = lib.oracle_predict(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m), kk,
                           float(s_th), int(threads), a.ctypes.data, c.ctypes.data,
                           s32.ctypes.data, s64.ctypes.data)
    if r < 0:
        raise MemoryError("oracle_predict")
    return {"a": a[:r], "c": c[:r], "s32": s32[:r], "s64": s64[:r]}


def predict_sources(g, L, m, k: int, sources, s_th: float = 0.0, threads: int = 0):
    """Top-k among the candidates owned by the given sources (pairs a < c with
    a in sources): dict with a, c, s32, s64."""
    lib = _load()
    off, idx = _arrays(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    kk = max(int(k), 0)
    a = np.zeros(max(kk, 1), np.int32)
    c = np.zeros(max(kk, 1), np.int32)
    s32 = np.zeros(max(kk, 1), np.float32)
    s64 = np.zeros(max(kk, 1), np.float64)
    r = lib.oracle_predict_sources(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m),
                                   kk, float(s_th), int(threads), src.ctypes.data, src.shape[0],
                                   a.ctypes.data, c.ctypes.data, s32.ctypes.data, s64.ctypes.data)
    if r < 0:
        raise MemoryError("oracle_predict_sources")
    return {"a": a[:r], "c": c[:r], "s32": s32[:r], "s64": s64[:r]}


def query(g, L, m, sources, kq: int, s_th: float = 0.0, threads: int = 0):
    """Per-source top-kq recommendation: list of dicts (c, s32, s64) per source."""
    lib = _load()
    off, idx = _arrays(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    ns = src.shape[0]
    kq = int(kq)
    c = np.zeros(max(ns * kq, 1), np.int32)
    s32 = np.zeros(max(ns * kq, 1), np.float32)
    s64 = np.zeros(max(ns * kq, 1), np.float64)
    cnt = np.zeros(max(ns, 1), np.int32)
    r = lib.oracle_query(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), measure_id(m),
                         src.ctypes.data if ns else None, ns, kq, float(s_th), int(threads),
                         c.ctypes.data, s32.ctypes.data, s64.ctypes.data, cnt.ctypes.data)
    if r < 0:
        raise MemoryError("oracle_query")
    out = []
    for i in range(ns):
        n_i = int(cnt[i])
        sl = slice(i * kq, i * kq + n_i)
        out.append({"c": c[sl].copy(), "s32": s32[sl].copy(), "s64": s64[sl].copy()})
    return out


def fingerprint(g, L, threads: int = 0):
    """(|C_L|, sum h, sum mix64(a, c, h) mod 2^64, wedges with c > a)."""
    off, idx = _arrays(g)
    out = np.zeros(4, np.uint64)
    r = _load().oracle_fingerprint(g.n, off.ctypes.data, idx.ctypes.data, _hub(L), int(threads),
                                   out.ctypes.data)
    if r < 0:
        raise MemoryError("oracle_fingerprint")
    return tuple(int(x) for x in out)


def mix64(a, c, h):
    """The digest term used by ``fingerprint`` (SplitMix64 finaliser), numpy u64."""
    a = np.asarray(a, dtype=np.uint64)
    c = np.asarray(c, dtype=np.uint64)
    h = np.asarray(h, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = ((a << np.uint64(32)) | (c & np.uint64(0xFFFFFFFF))) ^ (h * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def wedges(g, L) -> int:
    """W_L = sum over explored b of C(d_b, 2): the wedges with c > a (closed form)."""
    d = np.diff(g.offsets).astype(np.int64)
    Lh = _hub(L)
    d = d[d <= Lh]
    return int((d * (d - 1) // 2).sum())
