"""Pins for the CPU oracle: closed forms, the paper's worked example, brute
force on tiny inputs, library identities and invariants.  CPU only."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import pybrute as pybf
import synth

MEAS = oracle.MEASURES
HERE = os.path.dirname(os.path.abspath(__file__))


def cands_c(g, L, m):
    r = oracle.bruteforce(g, L, m)
    return {(int(a), int(c)): (int(h), float(s)) for a, c, h, s in zip(r["a"], r["c"], r["h"], r["s"])}


def cands_o1(g, L, m):
    out = {}
    for a in range(g.n):
        r = oracle.source(g, L, m, a, "predict")
        for c, h, s in zip(r["c"], r["h"], r["s"]):
            out[(a, int(c))] = (int(h), float(s))
    return out


# --------------------------------------------------------------------------
# Closed forms: every value below is worked out by hand from Section 3.1
# --------------------------------------------------------------------------

LN = math.log

CLOSED = {
    # star K_{1,5}: centre 0 (degree 5), leaves 1..5; every leaf pair has h = 1
    "star": dict(
        n=6, edges=[(0, i) for i in range(1, 6)],
        pairs={(i, j): 1 for i in range(1, 6) for j in range(i + 1, 6)},
        vals={"CN": 1, "JC": 1, "SI": 0.5, "SC": 1, "HP": 1, "HD": 1, "LHN": 1,
              "AA": 1 / LN(5), "RA": 0.2}),
    # path 0-1-2-3-4-5: degrees 1,2,2,2,2,1
    "path": dict(
        n=6, edges=[(i, i + 1) for i in range(5)],
        pairs={(0, 2): 1, (1, 3): 1, (2, 4): 1, (3, 5): 1},
        vals_by_pair={
            (0, 2): {"CN": 1, "JC": 0.5, "SI": 1 / 3, "SC": 1 / math.sqrt(2), "HP": 1, "HD": 0.5,
                     "LHN": 0.5, "AA": 1 / LN(2), "RA": 0.5},
            (1, 3): {"CN": 1, "JC": 1 / 3, "SI": 0.25, "SC": 0.5, "HP": 0.5, "HD": 0.5,
                     "LHN": 0.25, "AA": 1 / LN(2), "RA": 0.5},
        }),
    # K_{3,4}: A = {0,1,2} (degree 4), B = {3,4,5,6} (degree 3)
    "k34": dict(
        n=7, edges=[(a, b) for a in range(3) for b in range(3, 7)],
        pairs={**{(a, c): 4 for a in range(3) for c in range(a + 1, 3)},
               **{(a, c): 3 for a in range(3, 7) for c in range(a + 1, 7)}},
        vals_by_pair={
            (0, 1): {"CN": 4, "JC": 1, "SI": 0.5, "SC": 1, "HP": 1, "HD": 1, "LHN": 0.25,
                     "AA": 4 / LN(3), "RA": 4 / 3},
            (3, 4): {"CN": 3, "JC": 1, "SI": 0.5, "SC": 1, "HP": 1, "HD": 1, "LHN": 1 / 3,
                     "AA": 3 / LN(4), "RA": 0.75},
        }),
    # 4-cycle 0-1-2-3-0
    "c4": dict(
        n=4, edges=[(0, 1), (1, 2), (2, 3), (3, 0)],
        pairs={(0, 2): 2, (1, 3): 2},
        vals={"CN": 2, "JC": 1, "SI": 0.5, "SC": 1, "HP": 1, "HD": 1, "LHN": 0.5,
              "AA": 2 / LN(2), "RA": 1.0}),
    # complete graph: no candidate at all
    "k5": dict(n=5, edges=list(itertools.combinations(range(5), 2)), pairs={}, vals={}),
}


@pytest.mark.parametrize("name", sorted(CLOSED))
@pytest.mark.parametrize("m", MEAS)
def test_closed_forms(name, m):
    spec = CLOSED[name]
    g = synth.from_edges(spec["n"], spec["edges"])
    for route in (cands_c, cands_o1):
        got = route(g, None, m)
        assert set(got) == set(spec["pairs"]), (route.__name__, name)
        for p, h in spec["pairs"].items():
            assert got[p][0] == h
            if "vals" in spec:
                want = spec["vals"][m]
            elif p in spec["vals_by_pair"]:
                want = spec["vals_by_pair"][p][m]
            else:
                continue
            assert got[p][1] == pytest.approx(want, rel=1e-15, abs=0), (name, m, p)


def test_hub_limit_boundary():
    """d_b <= L explores b, d_b > L skips it (Section 4.2.1)."""
    star = synth.from_edges(6, [(0, i) for i in range(1, 6)])
    assert len(cands_c(star, 5, "CN")) == 10      # centre degree 5 <= 5
    assert len(cands_c(star, 4, "CN")) == 0       # 5 > 4: a large hub
    k34 = synth.from_edges(7, CLOSED["k34"]["edges"])
    got = cands_c(k34, 3, "CN")                   # only B (degree 3) explored
    assert set(got) == {(0, 1), (0, 2), (1, 2)} and all(v[0] == 4 for v in got.values())
    got = cands_c(k34, 2, "CN")
    assert got == {}


# --------------------------------------------------------------------------
# The paper's worked example (Section 4.2.2)
# --------------------------------------------------------------------------

def load_worked_example():
    path = os.path.join(HERE, "golden", "worked_example_dlh.txt")
    n, edges, src, sets = None, [], None, {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "n":
            n = int(tok[1])
        elif tok[0] == "edges":
            edges = [tuple(int(x) for x in t.split("-")) for t in tok[1:]]
        elif tok[0] == "source":
            src = int(tok[1])
        elif tok[0] == "second_order":
            L = None if tok[1] == "inf" else int(tok[1])
            sets[L] = {int(x) for x in tok[2:]}
    return synth.from_edges(n, edges), src, sets


def test_worked_example_second_order_sets():
    g, a, sets = load_worked_example()
    assert set(sets) == {None, 8, 4}
    for L, want in sets.items():
        for mode in ("predict", "query"):
            got = oracle.source(g, L, "CN", a, mode)
            assert set(int(c) for c in got["c"]) == want, (L, mode)
        assert set(pybf.second_order(g, L, a)) == want
        assert set(c for (x, c) in cands_c(g, L, "CN") if x == a) == {c for c in want if c > a}


# --------------------------------------------------------------------------
# Brute force on tiny inputs: every labelled graph on 5 vertices
# --------------------------------------------------------------------------

def all_graphs(nv):
    pairs = list(itertools.combinations(range(nv), 2))
    for mask in range(1 << len(pairs)):
        yield synth.from_edges(nv, [p for i, p in enumerate(pairs) if mask >> i & 1])


@pytest.mark.parametrize("m", ["CN", "JC", "SC", "LHN", "AA", "RA"])
def test_exhaustive_5_vertices(m):
    for g in all_graphs(5):
        for L in (0, 1, 2, 3, None):
            want = pybf.all_candidates(g, L, m)
            c0 = cands_c(g, L, m)
            assert set(c0) == set(want)
            for p, (h, s) in want.items():
                assert c0[p][0] == h and c0[p][1] == pytest.approx(s, rel=1e-12)
            c1 = cands_o1(g, L, m)
            assert set(c1) == set(c0)
            for p in c0:
                assert c1[p][0] == c0[p][0] and c1[p][1] == pytest.approx(c0[p][1], rel=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("L", [2, 4, 8, None])
def test_random_graphs_three_routes(seed, L):
    g = synth.random_graph(40, 0.15, seed) if seed != 3 else synth.chung_lu(60, 6.0, 2.2, seed)
    for m in MEAS:
        want = pybf.all_candidates(g, L, m)
        c0 = cands_c(g, L, m)
        c1 = cands_o1(g, L, m)
        assert set(want) == set(c0) == set(c1)
        for p, (h, s) in want.items():
            assert c0[p][0] == h == c1[p][0]
            assert c0[p][1] == pytest.approx(s, rel=1e-12)
            assert c1[p][1] == pytest.approx(s, rel=1e-12)


# --------------------------------------------------------------------------
# Library identity: h_L = (A D_L A)_{ac}, weights (A diag(w) A)_{ac}
# --------------------------------------------------------------------------

def adjacency(g):
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(g.offsets))
    return sp.csr_matrix((np.ones(g.nnz), (rows, g.indices)), shape=(n, n))


def scipy_candidates(g, L, diag):
    A = adjacency(g)
    P = (A @ sp.diags(diag) @ A).tocoo()
    a, c, v = P.row, P.col, P.data
    keep = (a < c) & (v != 0)
    a, c, v = a[keep], c[keep], v[keep]
    adj = set(zip(*adjacency(g).nonzero()))
    mask = np.array([(int(x), int(y)) not in adj for x, y in zip(a, c)], dtype=bool)
    return a[mask], c[mask], v[mask]


@pytest.fixture(scope="module")
def config1():
    g = synth.chung_lu_10k(1)
    obs, held = synth.holdout(g, 0.1, 1)
    return obs, held


@pytest.mark.parametrize("L", [256, None])
def test_scipy_identity_config1(config1, L):
    g, _ = config1
    d = np.diff(g.offsets).astype(np.float64)
    lim = np.inf if L is None else L
    a, c, v = scipy_candidates(g, L, (d <= lim).astype(np.float64))
    h = np.rint(v).astype(np.uint64)
    fp = oracle.fingerprint(g, L)
    assert fp[0] == a.shape[0]
    assert fp[1] == int(h.sum())
    assert fp[2] == int(np.bitwise_xor.reduce(np.zeros(1, np.uint64))) + int(
        oracle.mix64(a, c, h).sum(dtype=np.uint64))
    assert fp[3] == oracle.wedges(g, L)


@pytest.mark.parametrize("m", ["AA", "RA"])
def test_scipy_weights_config1(config1, m):
    g, _ = config1
    d = np.diff(g.offsets).astype(np.float64)
    with np.errstate(divide="ignore"):
        w = np.where(d <= 256, (1 / np.log(d)) if m == "AA" else 1 / d, 0.0)
    w[~np.isfinite(w)] = 0.0
    A = adjacency(g)
    P = (A @ sp.diags(w) @ A).tocsr()
    rng = np.random.default_rng(5)
    for a in rng.choice(np.nonzero(d > 0)[0], 40, replace=False):
        r = oracle.source(g, 256, m, int(a), "predict")
        row = P.getrow(int(a)).toarray().ravel()
        np.testing.assert_allclose(r["s"], row[r["c"]], rtol=1e-13)


def test_o0_equals_o1_config1_dlh(config1):
    g, _ = config1
    b = oracle.bruteforce(g, 256, "JC")
    fp = oracle.fingerprint(g, 256)
    assert fp[0] == b["a"].shape[0] and fp[1] == int(b["h"].sum())
    assert fp[2] == int(oracle.mix64(b["a"], b["c"], b["h"]).sum(dtype=np.uint64))


# --------------------------------------------------------------------------
# Wedge identity: sum_C h = W_L - sum_{(u,v) in E} h_L(u, v)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [16, 256, None])
def test_wedge_identity(config1, L):
    g, _ = config1
    A = adjacency(g)
    d = np.diff(g.offsets)
    lim = np.inf if L is None else L
    P = A @ sp.diags((d <= lim).astype(np.float64)) @ A
    edge_term = P.multiply(A).sum() / 2          # h_L over observed edges
    fp = oracle.fingerprint(g, L)
    assert fp[1] == oracle.wedges(g, L) - int(round(edge_term))
    if L is None:
        # IBase: the edge term counts every triangle three times
        tri = int(round((A @ A).multiply(A).sum() / 6))
        assert int(round(edge_term)) == 3 * tri


# --------------------------------------------------------------------------
# Invariants of the measures
# --------------------------------------------------------------------------

def test_measure_identities_and_ranges(config1):
    g, _ = config1
    rng = np.random.default_rng(7)
    for a in rng.choice(np.nonzero(np.diff(g.offsets) > 0)[0], 30, replace=False):
        r = {m: oracle.source(g, 256, m, int(a), "query") for m in MEAS}
        h = r["CN"]["s"]
        assert np.array_equal(h, r["CN"]["h"].astype(float))
        JC, SI, SC, HP, HD, LHN, AA, RA = (r[m]["s"] for m in ("JC", "SI", "SC", "HP", "HD", "LHN", "AA", "RA"))
        np.testing.assert_allclose(JC, SI / (1 - SI), rtol=1e-12)
        np.testing.assert_allclose(LHN, SC ** 2 / h, rtol=1e-12)
        assert np.all(HD <= SC * (1 + 1e-15)) and np.all(SC <= HP * (1 + 1e-15))
        for x in (JC, SC, HP, HD, LHN):
            assert np.all((x > 0) & (x <= 1))
        assert np.all((SI > 0) & (SI <= 0.5))
        assert np.all(RA < AA) and np.all(AA <= h / math.log(2) + 1e-12) and np.all(RA <= h / 2)


def test_symmetry(config1):
    g, _ = config1
    rng = np.random.default_rng(11)
    for m in ("JC", "AA", "LHN"):
        for a in rng.choice(np.nonzero(np.diff(g.offsets) > 0)[0], 10, replace=False):
            ra = oracle.source(g, 256, m, int(a), "query")
            for c, s in list(zip(ra["c"], ra["s"]))[:20]:
                rc = oracle.source(g, 256, m, int(c), "query")
                j = np.searchsorted(rc["c"], a)
                assert rc["c"][j] == a and rc["s"][j] == pytest.approx(s, rel=1e-12)


def test_monotone_in_hub_limit(config1):
    g, _ = config1
    prev = None
    for L in (2, 8, 32, 128, 512, None):
        fp = oracle.fingerprint(g, L)
        if prev is not None:
            assert fp[0] >= prev[0] and fp[1] >= prev[1] and fp[3] >= prev[3]
        prev = fp
    dmax = int(np.diff(g.offsets).max())
    assert oracle.fingerprint(g, dmax) == oracle.fingerprint(g, None)
    assert oracle.fingerprint(g, dmax - 1) != oracle.fingerprint(g, None)
    # per-pair: C_{L1} is a subset of C_{L2} with h_{L1} <= h_{L2}
    small = synth.chung_lu(300, 8.0, 2.2, 4)
    c8, cinf = cands_c(small, 8, "CN"), cands_c(small, None, "CN")
    assert set(c8) <= set(cinf) and all(c8[p][0] <= cinf[p][0] for p in c8)


def test_dlh_equals_ibase_without_hubs():
    """DLH(G, L) equals IBase on G with the hubs deleted, for every pair whose
    endpoints are both non-hubs (counts), and AA/RA weights taken from G."""
    g = synth.chung_lu(400, 10.0, 2.2, 9)
    L = 12
    d = np.diff(g.offsets)
    hubs = set(np.nonzero(d > L)[0].tolist())
    keep_edges = [(u, v) for u, v in g.edges() if u not in hubs and v not in hubs]
    gh = synth.from_edges(g.n, keep_edges)
    dl = cands_c(g, L, "CN")
    ib = cands_c(gh, None, "CN")
    dl_nh = {p: v for p, v in dl.items() if p[0] not in hubs and p[1] not in hubs}
    assert set(dl_nh) == set(ib)
    assert all(dl_nh[p][0] == ib[p][0] for p in ib)


# --------------------------------------------------------------------------
# Top-k: the definition (full sort under the total order) vs Algorithm 1
# --------------------------------------------------------------------------

def sort_reference(cands):
    rows = [(np.float32(s), a, c, s) for (a, c), (h, s) in cands.items()]
    rows.sort(key=lambda r: (-float(r[0]), r[1], r[2]))
    return rows


@pytest.mark.parametrize("m", MEAS)
def test_topk_matches_full_sort(m):
    g = synth.chung_lu(500, 8.0, 2.3, 3)
    cands = cands_c(g, 32, m)
    ref = sort_reference(cands)
    for k in (0, 1, 17, 500, len(ref), len(ref) + 10):
        for th in (0.0, float(ref[len(ref) // 3][0])):
            keep = [r for r in ref if r[0] > np.float32(th)]
            got = oracle.predict(g, 32, m, k, th, threads=3)
            want = keep[:k]
            assert len(got["a"]) == len(want)
            assert [(int(a), int(c)) for a, c in zip(got["a"], got["c"])] == [(r[1], r[2]) for r in want]
            assert np.array_equal(got["s32"], np.array([r[0] for r in want], np.float32))


@pytest.mark.parametrize("m", MEAS)
def test_topk_of_source_subset(m):
    """The subset form (what the CPU baseline times): the top k of the
    candidates owned by the listed sources, i.e. pairs a < c with a listed,
    against the full sort of the brute-force candidates so restricted.  A
    list taken in any order; an empty list gives nothing."""
    g = synth.chung_lu(500, 8.0, 2.3, 4)
    cands = cands_c(g, 32, m)
    rng = np.random.default_rng(7)
    for frac in (0.0, 0.1, 0.5, 1.0):
        src = rng.choice(g.n, int(frac * g.n), replace=False).astype(np.int32)
        listed = set(src.tolist())
        ref = sort_reference({p: v for p, v in cands.items() if p[0] in listed})
        for k in (1, 50, len(ref) + 5):
            got = oracle.predict_sources(g, 32, m, k, src, threads=3)
            want = ref[:k]
            assert len(got["a"]) == len(want)
            assert [(int(a), int(c)) for a, c in zip(got["a"], got["c"])] == [(r[1], r[2]) for r in want]
            assert np.array_equal(got["s32"], np.array([r[0] for r in want], np.float32))
            assert np.allclose(got["s64"], [r[3] for r in want], rtol=1e-12, atol=0)


def test_topk_thread_count_invariant(config1):
    g, held = config1
    k = held.shape[0]
    base = oracle.predict(g, 256, "JC", k, threads=1)
    for t in (2, 7):
        other = oracle.predict(g, 256, "JC", k, threads=t)
        for key in ("a", "c", "s32"):
            assert np.array_equal(base[key], other[key])


@pytest.mark.parametrize("m", ["JC", "AA"])
def test_query_matches_bruteforce(m):
    g = synth.chung_lu(300, 8.0, 2.2, 6)
    src = np.array([0, 5, 17, 40, 299, 5], np.int32)
    for L, kq in ((None, 5), (16, 1000)):
        res = oracle.query(g, L, m, src, kq)
        for s, r in zip(src, res):
            nb = pybf.neighbour_sets(g)
            degs = [len(x) for x in nb]
            lim = math.inf if L is None else L
            rows = []
            for c in range(g.n):
                if c == s or c in nb[s]:
                    continue
                common = {b for b in nb[s] & nb[c] if degs[b] <= lim}
                if common:
                    sc = pybf.measure(m, common, degs[s], degs[c], degs)
                    rows.append((np.float32(sc), c))
            rows.sort(key=lambda x: (-float(x[0]), x[1]))
            rows = rows[:kq]
            assert [int(c) for c in r["c"]] == [c for _, c in rows]
            assert np.array_equal(r["s32"], np.array([x for x, _ in rows], np.float32))
