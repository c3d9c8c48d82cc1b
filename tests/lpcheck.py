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


def assert_same_list(gpu, ref, measure, label=""):
    """gpu: (a, c, s32) numpy; ref: oracle.predict dict (a, c, s32, s64)."""
    ga, gc, gs = gpu
    assert_sorted_unique(ga, gc, gs)
    ra, rc, r32, r64 = ref["a"], ref["c"], ref["s32"], ref["s64"]
    assert ga.shape[0] == ra.shape[0], f"{label}: count {ga.shape[0]} != {ra.shape[0]}"
    if measure in EXACT_MEASURES:
        # exact integers in, one correctly rounded FP64 evaluation, one rounding to FP32
        assert np.array_equal(ga, ra) and np.array_equal(gc, rc), f"{label}: pair lists differ"
        assert np.array_equal(gs, r32), f"{label}: FP32 scores differ"
    else:
        assert_topk_acceptance(gpu, ref, label)


def assert_topk_acceptance(gpu, ref, label="", full=None):
    """Several top-k sets are correct when scores tie within the tolerance:
    the GPU list must hold every pair clearly above the k-th score and only
    pairs not clearly below it; its scores must match within REL_TOL.
    `full`: optional dict pair -> s64 over all candidates (else ref only)."""
    ga, gc, gs = gpu
    ra, rc, r64 = ref["a"], ref["c"], ref["s64"]
    assert ga.shape[0] == ra.shape[0], f"{label}: count differs"
    if ga.shape[0] == 0:
        return
    sk = float(r64[-1])
    ref_map = dict(zip(zip(ra.tolist(), rc.tolist()), r64.tolist()))
    if full is not None:
        ref_map = full
    gpu_pairs = list(zip(ga.tolist(), gc.tolist()))
    for (a, c), s in zip(gpu_pairs, gs.tolist()):
        if (a, c) in ref_map:
            sr = ref_map[(a, c)]
            assert abs(s - sr) <= REL_TOL * abs(sr), f"{label}: score {s} vs {sr} at {(a, c)}"
            assert sr >= sk * (1 - REL_TOL), f"{label}: {(a, c)} clearly below the k-th score"
        else:
            # not in the oracle's list: must tie with its boundary
            assert abs(s - sk) <= 2 * REL_TOL * abs(sk), f"{label}: {(a, c)} not a top-k pair"
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


def assert_same_query(gpu_row, ref_row, measure, label=""):
    """One source's ranked list: gpu (c, s32) numpy vs oracle.query row."""
    gc, gs = gpu_row
    rc, r32, r64 = ref_row["c"], ref_row["s32"], ref_row["s64"]
    assert gc.shape[0] == rc.shape[0], f"{label}: count {gc.shape[0]} != {rc.shape[0]}"
    if measure in EXACT_MEASURES:
        assert np.array_equal(gc, rc), f"{label}: lists differ"
        assert np.array_equal(gs, r32), f"{label}: scores differ"
    else:
        if gc.shape[0] == 0:
            return
        sk = float(r64[-1])
        ref = dict(zip(rc.tolist(), r64.tolist()))
        for c, s in zip(gc.tolist(), gs.tolist()):
            if c in ref:
                assert abs(s - ref[c]) <= REL_TOL * abs(ref[c]), f"{label}: c={c}"
            else:
                assert abs(s - sk) <= 2 * REL_TOL * abs(sk), f"{label}: c={c} not in top"
        gset = set(gc.tolist())
        for c, sr in ref.items():
            if sr > sk * (1 + REL_TOL):
                assert c in gset, f"{label}: missing c={c}"
