"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every case prints its name before touching the device.  Inputs are seeded
synthetic graphs from ``synth``; expected values come from ``oracle`` only."""
import itertools
import os

import numpy as np
import pytest

import oracle
import synth
from lpcheck import (assert_query_rows, assert_same_candidates, assert_same_list, assert_same_query,
                     say, to_np)

pytestmark = pytest.mark.gpu

MEAS = oracle.MEASURES
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2401_11415_amd as m
    m.load()
    return m


def run_predict(lp, g, m, L, k, s_th=0.0, host=False):
    if host:
        out = (np.zeros(max(k, 1), np.int32), np.zeros(max(k, 1), np.int32),
               np.zeros(max(k, 1), np.float32))
        a, c, s = lp.predict(g, m, L, k, s_th, out=out)
        return a, c, s
    a, c, s = lp.predict(g, m, L, k, s_th)
    return to_np(a), to_np(c), to_np(s)


def total_candidates(gr, L):
    return oracle.fingerprint(gr, L)[0]


CLOSED = {
    "star": (6, [(0, i) for i in range(1, 6)]),
    "path": (6, [(i, i + 1) for i in range(5)]),
    "k34": (7, [(a, b) for a in range(3) for b in range(3, 7)]),
    "c4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "k5": (5, list(itertools.combinations(range(5), 2))),
}


@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_forms(lp, name):
    n, edges = CLOSED[name]
    gr = synth.from_edges(n, edges)
    say(f"[gpu] closed form {name}")
    with lp.Graph(gr.offsets, gr.indices, validate=True) as g:
        for m in MEAS:
            for L in (None, 1, 2, 3, 4, 5):
                bf = oracle.bruteforce(gr, L, m)
                got = run_predict(lp, g, m, L, 100)
                assert_same_candidates(got, bf, m, f"{name}/{m}/L={L}")


def test_worked_example(lp):
    path = os.path.join(HERE, "golden", "worked_example_dlh.txt")
    n, edges, sets = None, [], {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        t = line.split()
        if t[0] == "n":
            n = int(t[1])
        elif t[0] == "edges":
            edges = [tuple(int(x) for x in e.split("-")) for e in t[1:]]
        elif t[0] == "second_order":
            sets[None if t[1] == "inf" else int(t[1])] = {int(x) for x in t[2:]}
    gr = synth.from_edges(n, edges)
    say("[gpu] worked example")
    with lp.Graph(gr.offsets, gr.indices, validate=True) as g:
        for L, want in sets.items():
            c, s, cnt = lp.query(g, [1], "CN", L, 100)
            got = set(to_np(c)[0][: int(cnt[0])].tolist())
            assert got == want, (L, got, want)


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("kind", ["er", "cl"])
def test_random_graphs_all_candidates(lp, seed, kind):
    gr = synth.random_graph(150, 0.06, seed) if kind == "er" else synth.chung_lu(3000, 10.0, 2.2, seed)
    say(f"[gpu] random {kind} seed={seed} n={gr.n} m={gr.m}")
    with lp.Graph(gr.offsets, gr.indices, validate=True) as g:
        for L in (2, 8, 64, None):
            tot = total_candidates(gr, L)
            for m in MEAS:
                ref = oracle.predict(gr, L, m, tot + 5)
                got = run_predict(lp, g, m, L, tot + 5)
                assert_same_list(got, ref, m, f"{kind}{seed}/{m}/L={L}", graph=gr, L=L)


@pytest.fixture(scope="module")
def config1():
    g = synth.chung_lu_10k(1)
    obs, held = synth.holdout(g, 0.1, 1)
    return obs, held.shape[0]


@pytest.mark.parametrize("L", [256, None])
def test_config1_jaccard_topk(lp, config1, L):
    gr, k = config1
    say(f"[gpu] config1 JC L={L} k={k}")
    ref = oracle.predict(gr, L, "JC", k)
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, "JC", L, k)
        assert_same_list(got, ref, "JC", f"config1/JC/L={L}", graph=gr, L=L)
        st = lp.last_stats(g)
        assert st["wedges"] == oracle.wedges(gr, L)


@pytest.mark.parametrize("m", MEAS)
def test_config1_measures(lp, config1, m):
    gr, k = config1
    say(f"[gpu] config1 {m} L=256")
    with lp.Graph(gr.offsets, gr.indices) as g:
        for L in (32, 256):
            ref = oracle.predict(gr, L, m, k)
            got = run_predict(lp, g, m, L, k)
            assert_same_list(got, ref, m, f"config1/{m}/L={L}", graph=gr, L=L)


@pytest.mark.parametrize("L", [0, 1, 2, 16, 256, None])
def test_config1_fingerprint(lp, config1, L):
    gr, _ = config1
    say(f"[gpu] config1 fingerprint L={L}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, L) == oracle.fingerprint(gr, L)


def test_global_path_and_partitions(lp, config1):
    """Force the dense global accumulator (tiny LDS cap), and exercise hash
    partitions with a graph whose sources can reach more distinct keys than
    one LDS table holds (K_{4,12000}: a leaf reaches up to 12,003 others)."""
    gr, k = config1
    say("[gpu] forced global path")
    with lp.Graph(gr.offsets, gr.indices) as g:
        for cap in (1, 40, 300):
            lp.set_tuning(g, lds_wedge_cap=cap)
            for m in ("JC", "RA"):
                ref = oracle.predict(gr, 256, m, k)
                got = run_predict(lp, g, m, 256, k)
                assert_same_list(got, ref, m, f"cap={cap}/{m}", graph=gr, L=256)
            assert lp.fingerprint(g, None) == oracle.fingerprint(gr, None)
            st = lp.last_stats(g)
            assert st["buckets"]["global"] > 0
    say("[gpu] hash partitions K_{4,12000}")
    kb = synth.from_edges(12004, [(h, 4 + i) for h in range(4) for i in range(12000)])
    with lp.Graph(kb.offsets, kb.indices) as g:
        for m in ("JC", "AA", "CN"):
            ref = oracle.predict(kb, None, m, 3000)
            got = run_predict(lp, g, m, None, 3000)
            assert_same_list(got, ref, m, f"K4,12000/{m}", graph=kb, L=None)
        assert lp.fingerprint(g, None) == oracle.fingerprint(kb, None)
        st = lp.last_stats(g)
        assert st["buckets"]["large"] > 0


def _launch_sums(st):
    tot = {f: 0 for f in ("launches", "sources", "wedges", "candidates")}
    for b in list(st["launches"].values()) + list(st["sampled"].values()):
        for f in tot:
            tot[f] += b[f]
        assert (b["ms"] > 0) == (b["launches"] > 0)
    return tot


@pytest.mark.parametrize("L", [2, 256, None])
def test_launch_work_counters(lp, config1, L):
    """Per-launch work counters: over a call, the wedges and the distinct
    candidates the accumulation kernels report add up to W_L and |C_L|."""
    gr, k = config1
    say(f"[gpu] launch work counters L={L}")
    ref = oracle.fingerprint(gr, L)
    with lp.Graph(gr.offsets, gr.indices) as g:
        for cap in (0, 40):
            lp.set_tuning(g, lds_wedge_cap=cap)
            assert lp.fingerprint(g, L) == ref
            st = lp.last_stats(g)
            tot = _launch_sums(st)
            assert tot["wedges"] == ref[3] == st["wedges"]
            assert tot["candidates"] == ref[0]
            assert tot["sources"] == st["sources"]
            assert st["launches"]["global"]["sources"] >= st["buckets"]["global"]
            if cap == 40 and L is None:
                assert st["buckets"]["global"] > 0
        lp.set_tuning(g, sample_budget=20000)
        run_predict(lp, g, "JC", L, 50)
        st = lp.last_stats(g)
        tot = _launch_sums(st)
        if st["retries"] == 0:
            assert tot["wedges"] == ref[3]
            # with a threshold, pairs beyond a source's degree cutoff are not
            # accumulated at all
            assert tot["candidates"] <= ref[0]


def test_sampled_threshold_path(lp, config1):
    """The top-k threshold estimated from a sample, including its retries."""
    gr, k = config1
    say("[gpu] sampled threshold")
    with lp.Graph(gr.offsets, gr.indices) as g:
        for budget in (20000, 200000):
            lp.set_tuning(g, sample_budget=budget)
            for m in (MEAS if budget == 20000 else ("JC", "CN", "AA", "LHN")):
                for kk in (50, k, 3 * k):
                    ref = oracle.predict(gr, 256, m, kk)
                    got = run_predict(lp, g, m, 256, kk)
                    assert_same_list(got, ref, m, f"budget={budget}/{m}/k={kk}", graph=gr, L=256)


@pytest.mark.parametrize("m", ["JC", "SC", "AA", "RA", "HP"])
def test_query(lp, config1, m):
    gr, _ = config1
    src = synth.sample_sources(gr, 60, seed=3, top=6)
    src = np.concatenate([src, src[:3]])  # repeats are allowed
    say(f"[gpu] query {m} ns={src.shape[0]}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        for L, kq in ((256, 10), (None, 7), (256, 20000), (None, 1)):
            ref = oracle.query(gr, L, m, src, kq)
            c, s, cnt = lp.query(g, src, m, L, kq)
            c, s, cnt = to_np(c), to_np(s), to_np(cnt)
            for i in range(src.shape[0]):
                row = (c[i][: cnt[i]], s[i][: cnt[i]])
                assert_same_query(row, ref[i], m, f"query {m} L={L} src={src[i]}", graph=gr, L=L,
                                  src=src[i])


def test_query_global_path(lp, config1):
    gr, _ = config1
    src = synth.sample_sources(gr, 20, seed=5, top=4)
    say("[gpu] query global path")
    with lp.Graph(gr.offsets, gr.indices) as g:
        lp.set_tuning(g, lds_wedge_cap=64)
        for m in ("JC", "AA"):
            ref = oracle.query(gr, None, m, src, 50)
            c, s, cnt = lp.query(g, src, m, None, 50)
            c, s, cnt = to_np(c), to_np(s), to_np(cnt)
            assert_query_rows(c, s, cnt, src, ref, m, f"q-global {m}", graph=gr, L=None)


def test_determinism(lp, config1):
    gr, k = config1
    say("[gpu] determinism")
    with lp.Graph(gr.offsets, gr.indices) as g:
        for m in ("JC", "AA"):
            r1 = run_predict(lp, g, m, 256, k)
            r2 = run_predict(lp, g, m, 256, k)
            for x, y in zip(r1, r2):
                assert np.array_equal(x, y)


def test_edge_cases(lp, config1):
    gr, k = config1
    say("[gpu] edge cases")
    with lp.Graph(gr.offsets, gr.indices) as g:
        a, c, s = run_predict(lp, g, "JC", 256, 0)
        assert a.shape[0] == 0
        for L in (0, 1):
            a, c, s = run_predict(lp, g, "CN", L, 100)
            assert a.shape[0] == 0
        # threshold: strictly above
        ref = oracle.predict(gr, 256, "JC", k, 0.25)
        got = run_predict(lp, g, "JC", 256, k, 0.25)
        assert_same_list(got, ref, "JC", "s_th=0.25", graph=gr, L=256, s_th=0.25)
        assert np.all(got[2] > 0.25)
        # host output pointers
        ref = oracle.predict(gr, 256, "SC", 500)
        got = run_predict(lp, g, "SC", 256, 500, host=True)
        assert_same_list(got, ref, "SC", "host outputs")
        # more than all candidates
        tot = total_candidates(gr, 16)
        ref = oracle.predict(gr, 16, "HD", tot + 1000)
        got = run_predict(lp, g, "HD", 16, tot + 1000)
        assert got[0].shape[0] == tot
        assert_same_list(got, ref, "HD", "k > |C|")
    # graphs with nothing to predict
    for n, edges in ((0, []), (5, []), (3, [(0, 1)]), (4, [(0, 1), (2, 3)])):
        gr0 = synth.from_edges(n, edges) if n else synth.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
        with lp.Graph(gr0.offsets, gr0.indices, validate=True) as g:
            a, c, s = run_predict(lp, g, "JC", None, 10)
            assert a.shape[0] == 0
            assert lp.fingerprint(g, None) == (0, 0, 0, 0)


def test_graph_usable_after_out_of_memory(lp, config1):
    """Scratch allocations above the graph's scratch_limit fail as the device
    running out would (LP_ERR_OUT_OF_MEMORY, no partial output); with the
    limit lifted the same graph answers every call correctly."""
    gr, k = config1
    say("[gpu] out of memory, then usable")
    with lp.Graph(gr.offsets, gr.indices) as g:
        lp.set_tuning(g, scratch_limit=1 << 16)
        for call in (lambda: lp.predict(g, "JC", 256, k), lambda: lp.query(g, [0, 1, 2], "AA", 256, 5),
                     lambda: lp.fingerprint(g, 256), lambda: lp.predict(g, "RA", 32, k)):
            with pytest.raises(lp.LpError) as e:
                call()
            assert e.value.name == "LP_ERR_OUT_OF_MEMORY"
        lp.set_tuning(g)
        for m in ("JC", "RA"):
            ref = oracle.predict(gr, 256, m, k)
            assert_same_list(run_predict(lp, g, m, 256, k), ref, m, f"after OOM {m}", graph=gr, L=256)
        assert lp.fingerprint(g, 256) == oracle.fingerprint(gr, 256)
        src = synth.sample_sources(gr, 20, seed=2, top=2)
        refq = oracle.query(gr, 256, "AA", src, 5)
        c, s, cnt = (to_np(x) for x in lp.query(g, src, "AA", 256, 5))
        assert_query_rows(c, s, cnt, src, refq, "AA", "after OOM query", graph=gr, L=256)


def test_busy_from_two_threads(lp, config1):
    """Two threads calling into one graph: a call that finds the graph in use
    returns LP_ERR_BUSY at once; every call that runs gives the right digest."""
    import threading
    import time
    gr, _ = config1
    ref = oracle.fingerprint(gr, 256)
    say("[gpu] busy from two threads")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, 256) == ref  # buffers at their working size
        lock = threading.Lock()
        seen = {"ok": 0, "busy": 0, "wrong": 0, "other": 0}
        stop = threading.Event()

        def worker():
            while not stop.is_set():
                try:
                    key = "ok" if lp.fingerprint(g, 256) == ref else "wrong"
                except lp.LpError as e:
                    key = "busy" if e.name == "LP_ERR_BUSY" else "other"
                with lock:
                    seen[key] += 1

        threads = [threading.Thread(target=worker) for _ in range(2)]
        for t in threads:
            t.start()
        t0 = time.time()
        while time.time() - t0 < 20:
            time.sleep(0.05)
            with lock:
                if seen["busy"] > 0 and seen["ok"] >= 20:
                    break
        stop.set()
        for t in threads:
            t.join()
        assert seen["wrong"] == 0 and seen["other"] == 0, seen
        assert seen["busy"] > 0 and seen["ok"] > 0, seen
        assert lp.fingerprint(g, 256) == ref


def test_invalid_inputs(lp):
    say("[gpu] invalid inputs")
    good = synth.from_edges(4, [(0, 1), (1, 2), (2, 3)])

    def create(off, idx, validate=True):
        return lp.Graph(np.asarray(off, np.int64), np.asarray(idx, np.int32), validate=validate)

    with pytest.raises(lp.LpError) as e:
        create([0, 2, 1, 3], [1, 2, 0], validate=False)  # offsets decrease
    assert e.value.name == "LP_ERR_INVALID_GRAPH"
    with pytest.raises(lp.LpError):
        create([0, 1, 2], [1, 7], validate=False)  # index out of range
    with pytest.raises(lp.LpError):
        create([0, 1, 3], [1, 0, 1])  # self loop 1-1
    with pytest.raises(lp.LpError):
        create([0, 2, 4, 6], [2, 1, 0, 2, 0, 1])  # unsorted row
    with pytest.raises(lp.LpError):
        create([0, 2, 3, 4], [1, 1, 0, 0])  # duplicate edge
    with pytest.raises(lp.LpError):
        create([0, 1, 1, 2], [1, 0])  # asymmetric: 0->1 but 1 has no arcs
    with lp.Graph(good.offsets, good.indices, validate=True) as g:
        for bad in (dict(m=9), dict(L=-1), dict(k=-1), dict(s=-0.5), dict(s=float("nan"))):
            with pytest.raises(lp.LpError) as e:
                lp.predict(g, bad.get("m", 1), bad.get("L", 2), bad.get("k", 5), bad.get("s", 0.0))
            assert e.value.name == "LP_ERR_INVALID_ARGUMENT"
        with pytest.raises(lp.LpError):
            lp.query(g, [0, 9], "JC", 2, 5)
        with pytest.raises(lp.LpError):
            lp.query(g, [0], "JC", 2, 0)
        # the graph stays usable after errors
        a, c, s = lp.predict(g, "CN", None, 10)
        assert to_np(a).tolist() == [0, 1] and to_np(c).tolist() == [2, 3]


def test_weighted_precision_bound(lp):
    """AA / RA sums are fixed point with as many fraction bits as the largest
    degree allows.  With an explored intermediate of degree 3,000,000 an RA
    term (1/d_b) cannot keep 2^-24 of its value, so the call refuses with
    LP_ERR_INVALID_ARGUMENT instead of rounding terms away; with a hub limit
    below that degree the same graph runs (and, on a star, has no wedges)."""
    say("[gpu] weighted fixed-point bound")
    leaves = 3_000_000
    n = leaves + 1
    off = np.concatenate([[0], leaves + np.arange(0, n, dtype=np.int64)]).astype(np.int64)
    idx = np.concatenate([np.arange(1, n, dtype=np.int32), np.zeros(leaves, np.int32)])
    with lp.Graph(off, idx) as g:
        with pytest.raises(lp.LpError) as e:
            lp.predict(g, "RA", None, 10)
        assert e.value.name == "LP_ERR_INVALID_ARGUMENT" and "hub limit" in e.value.detail
        a, c, s = lp.predict(g, "RA", 1000, 10)
        assert len(to_np(a)) == 0


@pytest.fixture(scope="module")
def rmat22():
    """The benchmark workload: R-MAT scale 22, edge factor 16, seed 1, 10% holdout."""
    full = synth.rmat22(seed=1)
    obs, held = synth.holdout(full, 0.1, seed=1)
    return obs, int(held.shape[0])


def test_full_size_rmat22_digest(lp, rmat22):
    """Parity at the benchmark's full size (R-MAT-22, L = 256): the
    candidate-set digest (|C_L|, sum h, sum mix64, W_L) is exact."""
    gr, k = rmat22
    say(f"[gpu] R-MAT-22 fingerprint n={gr.n}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, 256) == oracle.fingerprint(gr, 256)


def test_full_size_rmat22_topk(lp, rmat22):
    """The benchmark's own call (DLH JC, L = 256, k = |held out|, sampled
    threshold): identical FP32 top-k list to the oracle's."""
    gr, k = rmat22
    say(f"[gpu] R-MAT-22 predict JC k={k}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, "JC", 256, k)
        st = lp.last_stats(g)
        assert st["launches"]["mid3"]["launches"] > 0 and st["launches"]["large"]["launches"] > 0
    ref = oracle.predict(gr, 256, "JC", k)
    assert_same_list(got, ref, "JC", "R-MAT-22/JC/L=256")


def test_full_size_rmat22_digest_l64(lp, rmat22):
    """The R-MAT-22 candidate-set digest at the smallest hub limit of the
    sweep's main range (L = 64)."""
    gr, _ = rmat22
    say(f"[gpu] R-MAT-22 fingerprint L=64 n={gr.n}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, 64) == oracle.fingerprint(gr, 64)


@pytest.mark.parametrize("m", ["AA", "RA", "CN"])
def test_full_size_rmat22_topk_measures(lp, rmat22, m):
    """The benchmark graph with the unnormalised measures (DLH, L = 256,
    k = |held out|): CN exact, AA / RA by the acceptance rule, every pair
    outside the oracle's list checked by definition."""
    gr, k = rmat22
    say(f"[gpu] R-MAT-22 predict {m} L=256 k={k}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, m, 256, k)
    ref = oracle.predict(gr, 256, m, k)
    assert_same_list(got, ref, m, f"R-MAT-22/{m}/L=256", graph=gr, L=256)


def test_full_size_rmat22_topk_global(lp, rmat22):
    """The benchmark's call with the LDS cap lowered to 2048, so that sources
    above it (and above the key bound that keeps hubs on LDS tables) run on
    the dense global accumulator at full size: the same list as the oracle."""
    gr, k = rmat22
    say(f"[gpu] R-MAT-22 predict JC k={k}, lds_wedge_cap 2048")
    with lp.Graph(gr.offsets, gr.indices) as g:
        lp.set_tuning(g, lds_wedge_cap=2048)
        got = run_predict(lp, g, "JC", 256, k)
        st = lp.last_stats(g)
    assert st["launches"]["global"]["sources"] > 0
    ref = oracle.predict(gr, 256, "JC", k)
    assert_same_list(got, ref, "JC", "R-MAT-22/JC/L=256, dense accumulator")


@pytest.mark.parametrize("L", [32, 64])
def test_full_size_rmat22_cn_ties(lp, rmat22, L):
    """CN at small hub limits on the benchmark graph: counts are small
    integers, so the keys tied with the sampled threshold's count number many
    times k.  The list is still exact, and the call needs one pass (the
    sampled key with its ids bounds the ties)."""
    gr, k = rmat22
    say(f"[gpu] R-MAT-22 predict CN L={L} k={k}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, "CN", L, k)
        st = lp.last_stats(g)
    assert st["retries"] == 0, st["retries"]
    assert st["appended"] < 4 * k, st["appended"]
    ref = oracle.predict(gr, L, "CN", k)
    assert_same_list(got, ref, "CN", f"R-MAT-22/CN/L={L}")


@pytest.mark.parametrize("L", [1024, None])
@pytest.mark.parametrize("m", ["JC", "AA"])
def test_full_size_rmat22_query_wide(lp, rmat22, m, L):
    """Ranked lists on R-MAT-22 at L = 1024 and IBase (every intermediate,
    hubs included) for seeded sources plus the 4 of highest degree: the
    sources whose wedges go through the global accumulator."""
    gr, _ = rmat22
    src = synth.sample_sources(gr, 128, seed=29, top=4)
    say(f"[gpu] R-MAT-22 query {m} L={L} ns={src.shape[0]}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        c, s, cnt = (to_np(x) for x in lp.query(g, src, m, L, 10))
    refq = oracle.query(gr, L, m, src, 10)
    assert_query_rows(c, s, cnt, src, refq, m, f"R-MAT-22 query {m} L={L}", graph=gr, L=L)


@pytest.mark.parametrize("m", ["JC", "RA"])
def test_full_size_rmat22_query(lp, rmat22, m):
    """Per-source ranked lists on R-MAT-22 for a seeded sample of sources,
    including the 16 of highest degree."""
    gr, _ = rmat22
    src = synth.sample_sources(gr, 512, seed=7, top=16)
    say(f"[gpu] R-MAT-22 query {m} ns={src.shape[0]}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        c, s, cnt = lp.query(g, src, m, 256, 10)
        c, s, cnt = to_np(c), to_np(s), to_np(cnt)
    refq = oracle.query(gr, 256, m, src, 10)
    assert_query_rows(c, s, cnt, src, refq, m, f"R-MAT-22 query {m}", graph=gr, L=256)


@pytest.mark.parametrize("host_launches", [False, True])
def test_server_mix_equals_alone(lp, config1, host_launches):
    """Serving loop: requests of uneven size and two kinds, submitted together
    and batched by the server across three slots, each get exactly what
    lp_query returns for that request alone (and what the oracle returns).
    By default batches replay captured HIP graphs (the device-count query
    path); host_launches runs every batch as lp_query does."""
    gr, _ = config1
    rng = np.random.default_rng(11)
    deg = gr.degrees()
    nz = np.nonzero(deg > 0)[0]
    kinds = [("JC", 256, 10), ("AA", None, 5)]
    reqs = []
    for i in range(40):
        size = int(np.exp(rng.uniform(0, np.log(400))))
        p = deg[nz] / deg[nz].sum()  # degree-biased sources, repeats allowed
        reqs.append((rng.choice(nz, size=size, p=p).astype(np.int32), kinds[i % 2]))
    say(f"[gpu] server mix of {len(reqs)} requests, host_launches={host_launches}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        with lp.Server(g, slots=3, max_batch_sources=300, host_launches=host_launches) as srv:
            tickets = [srv.submit(src, m, L, kq) for src, (m, L, kq) in reqs]
            results = [srv.wait(t) for t in tickets]
            # a second round of the same requests: batches of shapes seen
            # before replay the graphs recorded then
            tickets = [srv.submit(src, m, L, kq) for src, (m, L, kq) in reqs]
            again = [srv.wait(t) for t in tickets]
        batches = {}
        for (out, rec) in results:
            assert rec["status"] == 0
            batches.setdefault(rec["batch"], rec["batch_requests"])
            assert rec["total_ms"] >= rec["run_ms"] >= 0
        assert max(batches.values()) > 1, "no request was batched with another"
        assert sum(batches.values()) == len(reqs)
        first = [rec["replayed"] for _, rec in results]
        second = [rec["replayed"] for _, rec in again]
        if host_launches:
            assert not any(first + second)
        else:
            # 1: replayed; 2: a batch outgrew the candidate capacity recorded
            # for its kind so far and ran on host launches (batches form by
            # timing, so a second-round batch can still be the largest); a
            # failed capture or replay (3) never happens
            assert first.count(1) > 0 and second.count(1) > len(second) // 2, (first, second)
            assert set(first + second) <= {1, 2}, (first, second)
        for (out, _), (out2, _) in zip(results, again):
            assert np.array_equal(out[2], out2[2])
            for i in range(out[2].shape[0]):
                n = out[2][i]
                assert np.array_equal(out[0][i][:n], out2[0][i][:n])
                assert np.array_equal(out[1][i][:n], out2[1][i][:n])
        for (src, (m, L, kq)), (out, rec) in zip(reqs, results):
            c, s, cnt = lp.query(g, src, m, L, kq)
            assert np.array_equal(out[2], to_np(cnt))
            for i in range(src.shape[0]):
                n = out[2][i]
                assert np.array_equal(out[0][i][:n], to_np(c)[i][:n])
                assert np.array_equal(out[1][i][:n], to_np(s)[i][:n])
        for (src, (m, L, kq)), (out, rec) in list(zip(reqs, results))[:6]:
            ref = oracle.query(gr, L, m, src, kq)
            assert_query_rows(out[0], out[1], out[2], src, ref, m, f"server {m}", graph=gr, L=L)


def test_server_invalid_requests(lp, config1):
    gr, _ = config1
    say("[gpu] server invalid requests")
    with lp.Graph(gr.offsets, gr.indices) as g:
        with lp.Server(g) as srv:
            for bad in (lambda: srv.submit([gr.n], "JC", 256, 10),
                        lambda: srv.submit([-1], "JC", 256, 10),
                        lambda: srv.submit([0], "JC", 256, 0),
                        lambda: srv.submit([0], "JC", -1, 10),
                        lambda: srv.submit([], "JC", 256, 10)):
                with pytest.raises(lp.LpError):
                    bad()
            t = srv.submit([0, 1, 2], "CN", 256, 3)
            out, rec = srv.wait(t)
            assert rec["status"] == 0
            with pytest.raises(lp.LpError):
                srv.wait(t)


def test_server_scratch_budget(lp, config1):
    """Admission by device scratch: with a budget below any two requests'
    need every batch holds one request; with the default budget requests
    share batches; both give lp_query's results.  Each request reports its
    batch's scratch bound."""
    gr, _ = config1
    rng = np.random.default_rng(5)
    deg = gr.degrees()
    nz = np.nonzero(deg > 0)[0]
    reqs = [rng.choice(nz, size=int(rng.integers(5, 60))).astype(np.int32) for _ in range(16)]
    say("[gpu] server scratch budget")
    with lp.Graph(gr.offsets, gr.indices) as g:
        ref = [tuple(to_np(x) for x in lp.query(g, r, "RA", 256, 5)) for r in reqs]
        for budget, batched in ((1, False), (0, True)):
            with lp.Server(g, slots=1, max_batch_bytes=budget) as srv:
                tickets = [srv.submit(r, "RA", 256, 5) for r in reqs]
                res = [srv.wait(t) for t in tickets]
            sizes = {rec["batch"]: rec["batch_requests"] for _, rec in res}
            assert all(rec["batch_bytes"] > 0 for _, rec in res)
            if batched:
                assert max(sizes.values()) > 1
                assert any(rec["replayed"] == 1 for _, rec in res)
                assert all(rec["replayed"] in (1, 2) for _, rec in res)
            else:
                assert set(sizes.values()) == {1}
                # no replayed shape fits a budget below one request's need
                assert not any(rec["replayed"] for _, rec in res)
            for (out, _), (c, s, n) in zip(res, ref):
                assert np.array_equal(out[2], n)
                for i in range(n.shape[0]):
                    assert np.array_equal(out[0][i][: n[i]], c[i][: n[i]])
                    assert np.array_equal(out[1][i][: n[i]], s[i][: n[i]])


@pytest.fixture(scope="module")
def chung_lu_8m():
    """The AA / RA workload: Chung-Lu, 8M vertices, exponent 2.1, weights capped
    at 2e5, seed 1, 10% holdout; k = 10% of the edges."""
    full = synth.chung_lu_8m(seed=1)
    obs, held = synth.holdout(full, 0.1, seed=1)
    return obs, int(held.shape[0])


def test_full_size_chung_lu_8m_digest(lp, chung_lu_8m):
    gr, _ = chung_lu_8m
    say(f"[gpu] Chung-Lu 8M fingerprint L=32 n={gr.n}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, 32) == oracle.fingerprint(gr, 32)


def test_full_size_chung_lu_8m_aa_topk(lp, chung_lu_8m):
    """DLH Adamic-Adar at L = 32 (the paper's choice for AA), k = |held out|:
    the top-k meets the acceptance rule against the oracle's FP64 list."""
    gr, k = chung_lu_8m
    say(f"[gpu] Chung-Lu 8M predict AA L=32 k={k}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, "AA", 32, k)
    ref = oracle.predict(gr, 32, "AA", k)
    assert_same_list(got, ref, "AA", "Chung-Lu 8M/AA/L=32", graph=gr, L=32)


def test_full_size_chung_lu_8m_digest_l256(lp, chung_lu_8m):
    gr, _ = chung_lu_8m
    say(f"[gpu] Chung-Lu 8M fingerprint L=256 n={gr.n}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        assert lp.fingerprint(g, 256) == oracle.fingerprint(gr, 256)


def test_full_size_chung_lu_8m_ra_topk(lp, chung_lu_8m):
    """DLH resource allocation at L = 256 (the paper's choice for RA),
    k = |held out|, as bench.py times it."""
    gr, k = chung_lu_8m
    say(f"[gpu] Chung-Lu 8M predict RA L=256 k={k}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        got = run_predict(lp, g, "RA", 256, k)
        st = lp.last_stats(g)
    ref = oracle.predict(gr, 256, "RA", k)
    assert_same_list(got, ref, "RA", "Chung-Lu 8M/RA/L=256", graph=gr, L=256)
    # the batched buckets skipped, whole, the sources whose arcs' weights sum
    # below the threshold (about 3 of their 7.7 million sources here)
    batched = ("tiny", "small", "mid1")
    listed = sum(st["buckets"][b] for b in batched)
    run = sum(st["launches"][b]["sources"] + st["sampled"][b]["sources"] for b in batched)
    handed = st["launches"]["split"]["sources"] + st["sampled"]["split"]["sources"]
    say(f"[gpu]   batched sources {listed}, accumulated {run}, handed to 12-byte tables {handed}")
    assert st["retries"] > 0 or run + handed < 0.8 * listed


@pytest.mark.parametrize("m", ["RA", "AA", "JC"])
def test_full_size_chung_lu_8m_query(lp, chung_lu_8m, m):
    """Ranked lists at L = 256 for seeded sources including the 16 of highest
    degree, whose wedges exceed the LDS tables."""
    gr, _ = chung_lu_8m
    src = synth.sample_sources(gr, 256, seed=5, top=16)
    say(f"[gpu] Chung-Lu 8M query {m} L=256 ns={src.shape[0]}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        c, s, cnt = lp.query(g, src, m, 256, 10)
        c, s, cnt = to_np(c), to_np(s), to_np(cnt)
    ref = oracle.query(gr, 256, m, src, 10)
    assert_query_rows(c, s, cnt, src, ref, m, f"Chung-Lu 8M query {m}", graph=gr, L=256)


def test_full_size_rmat24_server(lp):
    """The serving graph (R-MAT scale 24, full): requests of degree-biased
    sources through the server, DLH AA L = 32 top-10, against the oracle."""
    gr = synth.rmat24(seed=1)
    say(f"[gpu] R-MAT-24 server n={gr.n} m={gr.m}")
    rng = np.random.default_rng(17)
    deg = gr.degrees().astype(np.float64)
    nz = np.nonzero(deg > 0)[0]
    cdf = np.cumsum(deg[nz])
    reqs = [nz[np.minimum(np.searchsorted(cdf, rng.uniform(0, cdf[-1], n)), nz.shape[0] - 1)]
            .astype(np.int32) for n in (1, 37, 512, 200)]
    with lp.Graph(gr.offsets, gr.indices) as g:
        with lp.Server(g, slots=2) as srv:
            # twice: the second round replays graphs recorded in the first
            rounds = []
            for rnd in range(2):
                tickets = [srv.submit(r, "AA", 32, 10) for r in reqs]
                rounds.append([srv.wait(t) for t in tickets])
    flags = [[rec["replayed"] for _, rec in res] for res in rounds]
    say(f"replayed per round: {flags}")
    for j, r in enumerate(reqs):
        ref = oracle.query(gr, 32, "AA", r, 10)
        for rnd, res in enumerate(rounds):
            out = res[j][0]
            assert_query_rows(out[0], out[1], out[2], r, ref, "AA",
                              f"R-MAT-24 server, request {j}, round {rnd}, replayed {flags[rnd][j]}",
                              graph=gr, L=32)
    assert all(f in (1, 2) for f in flags[0] + flags[1]) and flags[1].count(1) >= 2, flags


@pytest.mark.parametrize("budget", [-1, 3000])
def test_predict_multi_equals_alone(lp, budget):
    """Several graphs in one call: each graph's top-k equals lp_predict on that
    graph alone and the oracle's list (ids shifted by the graph's start), with
    and without per-graph thresholds from a sample."""
    gs = synth.chung_lu_batch(24, 60, 6000, seed=9)
    u, vs = synth.disjoint_union(gs)
    ks = [max(0, gr.m // 10) for gr in gs]
    ks[3] = 0
    say(f"[gpu] predict_multi {len(gs)} graphs n={u.n} budget={budget}")
    with lp.Graph(u.offsets, u.indices) as g:
        lp.set_tuning(g, sample_budget=budget)
        sampled = 0
        for m, L in (("JC", 256), ("AA", None), ("CN", 8)):
            res = lp.predict_multi(g, vs, ks, m, L)
            st = lp.last_stats(g)
            for i, gr in enumerate(gs):
                a, c, s = (to_np(x) for x in res[i])
                got = (a - vs[i], c - vs[i], s)
                ref = oracle.predict(gr, L, m, ks[i])
                assert_same_list(got, ref, m, f"multi graph {i} {m} L={L}", graph=gr, L=L)
                if m != "AA":
                    with lp.Graph(gr.offsets, gr.indices) as gi:
                        alone = run_predict(lp, gi, m, L, ks[i])
                    assert np.array_equal(got[0], alone[0]) and np.array_equal(got[1], alone[1])
                    assert np.array_equal(got[2], alone[2])
            sampled += sum(b["launches"] for b in st["sampled"].values())
        assert (sampled > 0) == (budget > 0)


def test_predict_multi_invalid(lp):
    gs = synth.chung_lu_batch(3, 50, 200, seed=4)
    u, vs = synth.disjoint_union(gs)
    say("[gpu] predict_multi invalid")
    with lp.Graph(u.offsets, u.indices) as g:
        with pytest.raises(lp.LpError):
            lp.predict_multi(g, [0, 10, u.n - 1], [1, 1], "JC", 256)  # does not end at n
        with pytest.raises(lp.LpError):
            lp.predict_multi(g, [0, 30, 20, u.n], [1, 1, 1], "JC", 256)  # decreasing
        with pytest.raises(lp.LpError):
            lp.predict_multi(g, vs, [1, -1, 1], "JC", 256)
        with pytest.raises(lp.LpError) as e:
            cut = int(vs[1]) + int(np.argmax(gs[1].degrees())) + 1  # a hub of graph 1 left behind
            lp.predict_multi(g, [0, cut, u.n], [5, 5], "JC", 256)
        assert e.value.name == "LP_ERR_INVALID_GRAPH"


BUCKET_SETTINGS = [
    {"bucket_max": (16, 64, 512, 1536, 3072)},
    {"bucket_max": (32, 33, 34, 35, 36)},
    {"bucket_max": (1, 1, 1, 1, 1)},  # nearly every source in the 1024-lane kernel
    {"bucket_max": (1, 1, 1, 1, 1), "lds_wedge_cap": 200},
    {"tiny_batch": 32, "small_batch": 4},
    {"bucket_max": (16, 128), "tiny_batch": 32, "small_batch": 4, "lds_wedge_cap": 3000},
    {"small_shape": "wave", "mid1_shape": "workgroup128"},
    {"small_shape": "workgroup128", "mid1_shape": "batch"},
    {"small_shape": "workgroup256", "mid1_shape": "workgroup256"},
]


@pytest.mark.parametrize("which", range(len(BUCKET_SETTINGS)))
def test_bucket_bounds_same_result(lp, config1, which):
    """The bucket bounds only move sources between kernels: lists, digests,
    queries and the several-graph call are bit-identical to the defaults."""
    gr, k = config1
    setting = BUCKET_SETTINGS[which]
    say(f"[gpu] bucket bounds {setting}")
    src = synth.sample_sources(gr, 40, seed=8, top=4)
    gs = synth.chung_lu_batch(8, 60, 3000, seed=13)
    u, vs = synth.disjoint_union(gs)
    ks = [gr_i.m // 10 for gr_i in gs]
    with lp.Graph(gr.offsets, gr.indices) as g, lp.Graph(u.offsets, u.indices) as gu:
        base = {}
        for m in ("JC", "AA", "CN"):
            base[m] = (run_predict(lp, g, m, 256, k), lp.fingerprint(g, 256),
                       tuple(to_np(x) for x in lp.query(g, src, m, 256, 10)))
        base_multi = [tuple(to_np(x) for x in r) for r in lp.predict_multi(gu, vs, ks, "JC", 256)]
        lp.set_tuning(g, **setting)
        lp.set_tuning(gu, **setting)
        for m in ("JC", "AA", "CN"):
            got = run_predict(lp, g, m, 256, k)
            st = lp.last_stats(g)
            for x, y in zip(got, base[m][0]):
                assert np.array_equal(x, y), f"{setting} {m}"
            assert lp.fingerprint(g, 256) == base[m][1]
            q = tuple(to_np(x) for x in lp.query(g, src, m, 256, 10))
            for x, y in zip(q, base[m][2]):
                assert np.array_equal(x, y), f"query {setting} {m}"
        if len(setting.get("bucket_max", ())) == 5 and setting["bucket_max"][4] == 1:
            nb = st["buckets"]
            assert nb["small"] == nb["mid1"] == nb["mid2"] == nb["mid3"] == 0
            assert nb["large"] + nb["global"] > nb["tiny"]
        for r, b in zip(lp.predict_multi(gu, vs, ks, "JC", 256), base_multi):
            for x, y in zip((to_np(x) for x in r), b):
                assert np.array_equal(x, y), f"multi {setting}"
        ref = oracle.predict(gr, 256, "JC", k)
        assert_same_list(run_predict(lp, g, "JC", 256, k), ref, "JC", f"oracle {setting}")


def test_tuning_invalid(lp, config1):
    gr, k = config1
    say("[gpu] tuning invalid")
    with lp.Graph(gr.offsets, gr.indices) as g:
        before = run_predict(lp, g, "JC", 256, k)
        lp.set_tuning(g, bucket_max=(8, 8, 8, 8, 8))
        for bad in ((33, 0, 0, 0, 0), (0, 0, 0, 0, 4097), (-1, 0, 0, 0, 0)):
            with pytest.raises(lp.LpError):
                lp.set_tuning(g, bucket_max=bad)
        with pytest.raises(lp.LpError):
            lp.set_tuning(g, lds_wedge_cap=-5)
        with pytest.raises(lp.LpError):
            lp.set_tuning(g, tiny_batch=40)
        with pytest.raises(lp.LpError):
            lp.set_tuning(g, small_batch=16)
        with pytest.raises(lp.LpError):
            lp.set_tuning(g, mid1_shape="wave")
        with pytest.raises(lp.LpError):
            lp.set_tuning(g, small_shape=7)
        with pytest.raises(ValueError):
            lp.set_tuning(g, bucket_max=(1, 1, 1, 1, 1, 1))
        run_predict(lp, g, "JC", 256, k)
        assert lp.last_stats(g)["buckets"]["small"] == 0  # the valid knobs stayed
        after = run_predict(lp, g, "JC", 256, k)
        for x, y in zip(before, after):
            assert np.array_equal(x, y)


def test_autotune_keeps_results(lp):
    """The autotuner over a small space on a several-graph call: it leaves the
    graph at the best setting it measured, and the lists do not change."""
    from paper_2401_11415_amd import tune
    import torch
    gs = synth.chung_lu_batch(16, 100, 20000, seed=21)
    u, vs = synth.disjoint_union(gs)
    ks = [gr_i.m // 10 for gr_i in gs]
    say(f"[gpu] autotune n={u.n}")
    with lp.Graph(u.offsets, u.indices) as g:
        base = [tuple(to_np(x) for x in r) for r in lp.predict_multi(g, vs, ks, "JC", 256)]

        def run():
            lp.predict_multi(g, vs, ks, "JC", 256)
            torch.cuda.synchronize()

        space = {"bucket_max0": (32, 16), "tiny_batch": (48, 32), "lds_wedge_cap": (65536, 512)}
        res = tune.autotune(g, run, space=space, repeats=1)
        assert len(res["trials"]) == 4
        assert res["ms"] <= res["default_ms"]
        assert set(res["setting"]) == set(space)
        for r, b in zip(lp.predict_multi(g, vs, ks, "JC", 256), base):
            for x, y in zip((to_np(x) for x in r), b):
                assert np.array_equal(x, y)


@pytest.fixture(scope="module")
def batch512():
    """The batched workload: 512 Chung-Lu graphs of 1,000-1,000,000 vertices
    (log-uniform), mean degree 8-32, exponent 2.3, graph i seeded 1000 + i,
    sizes drawn with seed 5; k_i = m_i / 10."""
    gs = synth.chung_lu_batch(512, 1000, 1_000_000, seed=5)
    u, vs = synth.disjoint_union(gs)
    return gs, u, vs, [gr.m // 10 for gr in gs]


def test_full_size_batch512(lp, batch512):
    """The several-graph call at the batched workload's full size (71.8 M
    vertices in one union, DLH JC L = 256, default knobs, as bench.py --multi
    times it): the lists of a seeded sample of graphs, and of the largest
    one, equal the oracle's on each graph alone.  The union has more than
    2^26 vertices, so its tiny sources run 32 per workgroup."""
    gs, u, vs, ks = batch512
    rng = np.random.default_rng(17)
    order = np.argsort([gr.n for gr in gs])
    picks = sorted(set(rng.choice(order[:384], size=10, replace=False).tolist()) | {int(order[-1])})
    say(f"[gpu] batch of 512 graphs n={u.n} picks={picks}")
    assert u.n > (1 << 26)
    with lp.Graph(u.offsets, u.indices) as g:
        res = lp.predict_multi(g, vs, ks, "JC", 256)
        st = lp.last_stats(g)
        got = {i: tuple(to_np(x) for x in res[i]) for i in picks}
        sizes = [int(r[0].shape[0]) for r in res]
    assert st["launches"]["tiny"]["launches"] > 0
    assert all(sz <= k for sz, k in zip(sizes, ks))
    for i in picks:
        a, c, s = got[i]
        ref = oracle.predict(gs[i], 256, "JC", ks[i])
        assert_same_list((a - vs[i], c - vs[i], s), ref, "JC", f"batch graph {i} n={gs[i].n}")


@pytest.mark.parametrize("slots", [1, 3, 0, 1 << 20])
def test_global_path_forms(lp, config1, slots):
    """The global accumulator runs one workgroup per source when there are
    more than two rounds of slabs and splits each source over all workgroups
    otherwise; the workgroup count decides which.  Both forms, for predict
    and for weighted queries (with their per-source floors), match the
    oracle."""
    gr, k = config1
    src = synth.sample_sources(gr, 30, seed=23, top=6)
    say(f"[gpu] global path, {slots} slabs")
    with lp.Graph(gr.offsets, gr.indices) as g:
        lp.set_tuning(g, lds_wedge_cap=40, global_slots=slots)
        for m in ("JC", "RA"):
            ref = oracle.predict(gr, 256, m, k)
            got = run_predict(lp, g, m, 256, k)
            assert_same_list(got, ref, m, f"slots={slots}/{m}", graph=gr, L=256)
            assert lp.last_stats(g)["launches"]["global"]["sources"] > 0
        assert lp.fingerprint(g, None) == oracle.fingerprint(gr, None)
        for m, kq in (("AA", 5), ("RA", 40)):
            refq = oracle.query(gr, None, m, src, kq)
            c, s, cnt = (to_np(x) for x in lp.query(g, src, m, None, kq))
            assert_query_rows(c, s, cnt, src, refq, m, f"slots={slots} query {m}", graph=gr, L=None)


def test_predict_multi_empty_graphs(lp):
    """Graphs without vertices or without edges inside a union: they return
    no rows, and their neighbours in the union are unaffected."""
    gs = synth.chung_lu_batch(3, 200, 2000, seed=31)
    empty = synth.Graph(np.zeros(1, np.int64), np.zeros(0, np.int32))
    isolated = synth.Graph(np.zeros(6, np.int64), np.zeros(0, np.int32))  # 5 vertices, no edges
    parts = [empty, gs[0], isolated, empty, gs[1], gs[2], empty]
    u, vs = synth.disjoint_union(parts)
    ks = [0, gs[0].m // 10, 3, 5, gs[1].m // 10, 7, 0]
    say(f"[gpu] predict_multi with empty graphs n={u.n}")
    with lp.Graph(u.offsets, u.indices) as g:
        for budget in (-1, 500):
            lp.set_tuning(g, sample_budget=budget)
            res = lp.predict_multi(g, vs, ks, "JC", 256)
            for i, gr in enumerate(parts):
                a, c, sc = (to_np(x) for x in res[i])
                if gr.m == 0:
                    assert a.shape[0] == 0
                    continue
                ref = oracle.predict(gr, 256, "JC", ks[i])
                assert_same_list((a - vs[i], c - vs[i], sc), ref, "JC", f"graph {i} budget={budget}")


def test_predict_multi_many_graphs(lp):
    """More graphs than the per-graph histograms hold in LDS (2,500 small
    graphs): the global-memory counters give the same lists."""
    gs = synth.chung_lu_batch(2500, 12, 60, seed=41, d_min=3.0, d_max=8.0)
    u, vs = synth.disjoint_union(gs)
    ks = [max(1, gr.m // 4) for gr in gs]
    say(f"[gpu] predict_multi {len(gs)} graphs n={u.n}")
    rng = np.random.default_rng(43)
    picks = rng.choice(len(gs), size=150, replace=False)
    with lp.Graph(u.offsets, u.indices) as g:
        for budget in (-1, 2000):
            lp.set_tuning(g, sample_budget=budget)
            res = lp.predict_multi(g, vs, ks, "JC", 256)
            for i in picks:
                a, c, sc = (to_np(x) for x in res[i])
                ref = oracle.predict(gs[i], 256, "JC", ks[i])
                assert_same_list((a - vs[i], c - vs[i], sc), ref, "JC", f"graph {i} budget={budget}")
