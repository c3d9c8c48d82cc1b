"""Comparison helpers for GPU-vs-oracle parity (no link-prediction arithmetic)."""
from __future__ import annotations

import sys

import numpy as np

EXACT_MEASURES = ("CN", "JC", "SI", "SC", "HP", "HD", "LHN")
REL_TOL = 1e-6  # FP32 scores against the FP64 oracle


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_np(t):
    return t.detach().cpu().numpy()


def order_key(s32, a, c):
    """Rows sorted by (score desc, a asc, c asc)."""
    return np.lexsort((c, a, -s32.astype(np.float64)))


def assert_sorted_unique(a, c, s):
    assert np.all(a < c), "pairs must be (min, max)"
    o = order_key(s, a, c)
    assert np.array_equal(o, np.arange(len(a))), "rows are not in (score desc, a, c) order"
    pairs = a.astype(np.int64) << 32 | c.astype(np.int64)
    assert np.unique(pairs).shape[0] == pairs.shape[0], "duplicate pairs"


def assert_same_list(gpu, ref, measure, label="", graph=None, L=None, s_th=0.0):
    """gpu: (a, c, s32) numpy; ref: oracle.predict dict (a, c, s32, s64).
    graph / L / s_th: the graph and call the lists came from; needed to check
    GPU pairs that the oracle's list does not hold (AA / RA ties)."""
    ga, gc, gs = gpu
    assert_sorted_unique(ga, gc, gs)
    ra, rc, r32, r64 = ref["a"], ref["c"], ref["s32"], ref["s64"]
    assert ga.shape[0] == ra.shape[0], f"{label}: count {ga.shape[0]} != {ra.shape[0]}"
    if measure in EXACT_MEASURES:
        # exact integers in, one correctly rounded FP64 evaluation, one rounding to FP32
        assert np.array_equal(ga, ra) and np.array_equal(gc, rc), f"{label}: pair lists differ"
        assert np.array_equal(gs, r32), f"{label}: FP32 scores differ"
    else:
        assert_topk_acceptance(gpu, ref, label, graph=graph, L=L, measure=measure, s_th=s_th)


def check_off_list(graph, L, measure, a, c, s_gpu, sk, s_th, label):
    """Pairs a GPU list holds that the oracle's list does not: each must be a
    candidate by definition (non-adjacent, an explored common neighbour), have
    its FP64 score (recomputed pair by pair) within REL_TOL of the GPU's, pass
    the score threshold, and not lie clearly below the k-th score sk."""
    a = np.asarray(a, np.int32)
    c = np.asarray(c, np.int32)
    s_gpu = np.asarray(s_gpu, np.float64)
    if a.shape[0] == 0:
        return
    assert graph is not None, f"{label}: {a.shape[0]} GPU pairs outside the oracle's list and no graph to check them"
    import oracle
    ok, _, s64 = oracle.pairs(graph, L, measure, a, c)
    bad = np.nonzero(~ok)[0]
    assert bad.shape[0] == 0, f"{label}: {(int(a[bad[0]]), int(c[bad[0]]))} is not a candidate"
    err = np.abs(s_gpu - s64) > REL_TOL * np.abs(s64)
    i = np.nonzero(err)[0]
    assert i.shape[0] == 0, f"{label}: score {s_gpu[i[0]]} vs {s64[i[0]]} at {(int(a[i[0]]), int(c[i[0]]))}"
    low = np.nonzero(~(s64.astype(np.float32) > np.float32(s_th)))[0]
    assert low.shape[0] == 0, f"{label}: {(int(a[low[0]]), int(c[low[0]]))} not above S_th"
    below = np.nonzero(s64 < sk * (1 - REL_TOL))[0]
    assert below.shape[0] == 0, \
        f"{label}: {(int(a[below[0]]), int(c[below[0]]))} clearly below the k-th score ({s64[below[0]]} < {sk})"


def assert_topk_acceptance(gpu, ref, label="", graph=None, L=None, measure=None, s_th=0.0):
    """Several top-k sets are correct when scores tie within the tolerance:
    the GPU list must hold every pair clearly above the k-th score and only
    candidates not clearly below it; its scores must match within REL_TOL.
    Pairs outside the oracle's list are checked one by one (check_off_list)."""
    ga, gc, gs = gpu
    ra, rc, r64 = ref["a"], ref["c"], ref["s64"]
    assert ga.shape[0] == ra.shape[0], f"{label}: count differs"
    if ga.shape[0] == 0:
        return
    sk = float(r64[-1])
    ref_map = dict(zip(zip(ra.tolist(), rc.tolist()), r64.tolist()))
    gpu_pairs = list(zip(ga.tolist(), gc.tolist()))
    off_a, off_c, off_s = [], [], []
    for (a, c), s in zip(gpu_pairs, gs.tolist()):
        if (a, c) in ref_map:
            sr = ref_map[(a, c)]
            assert abs(s - sr) <= REL_TOL * abs(sr), f"{label}: score {s} vs {sr} at {(a, c)}"
            assert sr >= sk * (1 - REL_TOL), f"{label}: {(a, c)} clearly below the k-th score"
        else:
            off_a.append(a)
            off_c.append(c)
            off_s.append(s)
    check_off_list(graph, L, measure, off_a, off_c, off_s, sk, s_th, label)
    gset = set(gpu_pairs)
    for (a, c), sr in zip(zip(ra.tolist(), rc.tolist()), r64.tolist()):
        if sr > sk * (1 + REL_TOL):
            assert (a, c) in gset, f"{label}: missing {(a, c)} (score {sr} > k-th {sk})"


def assert_same_candidates(gpu, bf, measure, label=""):
    """All candidates: gpu (a, c, s32) with k >= |C|; bf = oracle.bruteforce dict."""
    ga, gc, gs = gpu
    assert_sorted_unique(ga, gc, gs)
    g = {(int(a), int(c)): float(s) for a, c, s in zip(ga, gc, gs)}
    r = {(int(a), int(c)): float(s) for a, c, s in zip(bf["a"], bf["c"], bf["s"])}
    assert set(g) == set(r), f"{label}: candidate sets differ ({len(g)} vs {len(r)})"
    for p, sr in r.items():
        if measure in EXACT_MEASURES:
            assert g[p] == float(np.float32(sr)), f"{label}: {p} {g[p]} vs {sr}"
        else:
            assert abs(g[p] - sr) <= REL_TOL * abs(sr), f"{label}: {p} {g[p]} vs {sr}"


def assert_same_query(gpu_row, ref_row, measure, label="", graph=None, L=None, src=None, s_th=0.0):
    """One source's ranked list: gpu (c, s32) numpy vs oracle.query row.
    graph / L / src: the query, to check entries outside the oracle's row."""
    gc, gs = gpu_row
    rc, r32, r64 = ref_row["c"], ref_row["s32"], ref_row["s64"]
    assert gc.shape[0] == rc.shape[0], f"{label}: count {gc.shape[0]} != {rc.shape[0]}"
    assert np.unique(gc).shape[0] == gc.shape[0], f"{label}: duplicate entries"
    if measure in EXACT_MEASURES:
        assert np.array_equal(gc, rc), f"{label}: lists differ"
        assert np.array_equal(gs, r32), f"{label}: scores differ"
        return
    if gc.shape[0] == 0:
        return
    order = np.lexsort((gc, -gs.astype(np.float64)))
    assert np.array_equal(order, np.arange(gc.shape[0])), f"{label}: not in (score desc, c asc) order"
    sk = float(r64[-1])
    ref = dict(zip(rc.tolist(), r64.tolist()))
    off_c, off_s = [], []
    for c, s in zip(gc.tolist(), gs.tolist()):
        if c in ref:
            assert abs(s - ref[c]) <= REL_TOL * abs(ref[c]), f"{label}: c={c}"
            assert ref[c] >= sk * (1 - REL_TOL), f"{label}: c={c} clearly below the k_q-th score"
        else:
            off_c.append(c)
            off_s.append(s)
    if off_c:
        assert src is not None, f"{label}: entries outside the oracle's row and no source to check them"
        check_off_list(graph, L, measure, [int(src)] * len(off_c), off_c, off_s, sk, s_th, label)
    gset = set(gc.tolist())
    for c, sr in ref.items():
        if sr > sk * (1 + REL_TOL):
            assert c in gset, f"{label}: missing c={c}"


def assert_query_rows(c, s, cnt, src, refq, measure, label, graph=None, L=None, s_th=0.0):
    """Every row of an lp_query result (c, s: [n, k_q]; cnt: [n]) against the
    oracle's rows."""
    for i in range(len(src)):
        n = int(cnt[i])
        assert_same_query((c[i][:n], s[i][:n]), refq[i], measure, f"{label} src={src[i]}",
                          graph=graph, L=L, src=src[i], s_th=s_th)
