"""lp_query_static (no device allocation; scratch in the library's fixed
per-device array) against lp_query on the same inputs, through the C ABI:
two calls in a row, the second with a smaller input, on the per-source
tables and on the dense global accumulator; then the limits of the fixed
scratch, after which the graph and the scratch stay usable."""
import numpy as np
import pytest

import synth
from lpcheck import say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2401_11415_amd as m
    m.load()
    return m


def _outputs(torch, ns, kq):
    dev = torch.device("cuda", torch.cuda.current_device())
    return (torch.empty((ns, kq), dtype=torch.int32, device=dev),
            torch.empty((ns, kq), dtype=torch.float32, device=dev),
            torch.zeros(ns, dtype=torch.int32, device=dev))


def _same_rows(ref, got, what):
    rc, rs, rn = ref
    c, s, n = got
    assert np.array_equal(rn, n), what
    for i in range(rn.shape[0]):
        k = int(rn[i])
        assert np.array_equal(rc[i][:k], c[i][:k]), (what, i)
        assert np.array_equal(rs[i][:k], s[i][:k]), (what, i)


def test_query_static_equals_query(lp):
    import torch
    g0 = synth.chung_lu(20000, 12.0, 2.3, 5)
    gr, _ = synth.holdout(g0, 0.1, 5)
    big = synth.sample_sources(gr, 1500, seed=3, top=8)
    # IBase reaches every intermediate: fewer sources keep the path bound
    # (about a million) inside the fixed scratch; the three largest hubs
    # exceed the LDS capacity and take the dense accumulator
    ibase = synth.sample_sources(gr, 400, seed=4, top=3)
    dev = torch.device("cuda", torch.cuda.current_device())
    cases = [("JC", 256, 10, big, 0), ("AA", 32, 7, big, 0), ("RA", None, 5, ibase, 0),
             # every source above 2048 wedges on the dense accumulator
             ("CN", 256, 6, big, 2048)]
    with lp.Graph(gr.offsets, gr.indices) as g:
        # the first call on the device looks the scratch's address up
        lp.query_static(g, big[:3], "CN", 8, 2)
        for (m, L, kq, src0, cap) in cases:
            lp.set_tuning(g, lds_wedge_cap=cap)
            small = src0[:200][::-1].copy()
            for src in (src0, small):
                say(f"[gpu] query_static n={gr.n} {m} L={L} k_q={kq} lds_wedge_cap={cap} "
                    f"sources={src.shape[0]}")
                ref = tuple(to_np(x) for x in lp.query(g, src, m, L, kq))
                src_t = torch.as_tensor(src, device=dev)
                out = _outputs(torch, src.shape[0], kq)
                torch.cuda.synchronize()
                before = torch.cuda.mem_get_info()[0]
                lp.query_static(g, src_t, m, L, kq, out=out)
                torch.cuda.synchronize()
                assert torch.cuda.mem_get_info()[0] == before, "device memory changed during the call"
                got = tuple(to_np(x) for x in out)
                assert int(got[2].sum()) > 0
                _same_rows(ref, got, (m, L, src.shape[0]))
        lp.set_tuning(g)


def test_query_static_limits(lp):
    gr = synth.chung_lu(20000, 12.0, 2.3, 5)
    say("[gpu] query_static limits")
    with lp.Graph(gr.offsets, gr.indices) as g:
        def refused(*args):
            with pytest.raises(lp.LpError) as e:
                lp.query_static(g, *args)
            assert e.value.name == "LP_ERR_INVALID_ARGUMENT", e.value
        refused(np.zeros(5000, np.int32), "JC", 256, 10)     # more sources than the scratch holds
        refused(np.zeros(2000, np.int32), "JC", 256, 1000)   # rows beyond the scratch
        refused(np.array([gr.n], np.int32), "JC", 256, 10)   # source out of range
        hubs = np.argsort(-gr.degrees(), kind="stable")[:4000].astype(np.int32)
        refused(hubs, "CN", None, 1)                          # two-hop path bound beyond the scratch
        # still usable, and equal to lp_query
        src = synth.sample_sources(gr, 50, seed=1, top=2)
        got = tuple(to_np(x) for x in lp.query_static(g, src, "CN", 64, 4))
        ref = tuple(to_np(x) for x in lp.query(g, src, "CN", 64, 4))
        _same_rows(ref, got, "after refusals")


def test_query_static_dense_accumulator_too_large(lp):
    """A source on the dense accumulator needs 12 bytes per vertex; on a
    graph with 3.2 million vertices that is more than the fixed scratch
    holds, and the call says so instead of allocating."""
    gr = synth.chung_lu(3_200_000, 3.0, 2.3, 7)
    deg = gr.degrees()
    # T = wedges + degree of each vertex; pick one that an LDS table holds
    # by default but not under a cap of 64
    nz = deg > 0
    T = np.zeros(gr.n, np.int64)
    T[nz] = np.add.reduceat(deg[gr.indices].astype(np.int64), gr.offsets[:-1][nz]) + deg[nz]
    src = np.nonzero((T > 4096) & (T < 32768))[0][:1].astype(np.int32)
    assert src.shape[0] == 1
    say(f"[gpu] query_static dense accumulator n={gr.n} source T={int(T[src[0]])}")
    with lp.Graph(gr.offsets, gr.indices) as g:
        lp.set_tuning(g, lds_wedge_cap=64)
        with pytest.raises(lp.LpError) as e:
            lp.query_static(g, src, "CN", None, 4)
        assert e.value.name == "LP_ERR_INVALID_ARGUMENT"
        assert "dense accumulator" in str(e.value)
        lp.set_tuning(g)
        # under the default cap the source fits an LDS table
        got = tuple(to_np(x) for x in lp.query_static(g, src, "CN", None, 4))
        ref = tuple(to_np(x) for x in lp.query(g, src, "CN", None, 4))
        assert int(ref[2][0]) > 0
        _same_rows(ref, got, "after the refusal")
