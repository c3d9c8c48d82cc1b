"""Host-side logic of bench.py, without a GPU: the one-GPU guard, the lookup
of the committed HBM traffic summary, and the algorithmic byte counts that
the roofline figures divide by."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no result line


def test_traffic_lookup_requires_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("source_sha256: abc\n"
                 "traffic_bytes_per_launch k<1, 2> = 123\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic("k<1, 2>") == 123.0
    assert bench.measured_traffic("another<3>") is None
    # taken on other kernel sources: not reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "def")
    assert bench.measured_traffic("k<1, 2>") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("k<1, 2>") is None
    # a workload that no summary covers
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc")
    assert bench.measured_traffic("k<1, 2>", "") is None
    assert bench.measured_traffic("k<1, 2>", str(f)) == 123.0


@pytest.mark.parametrize("which", ["jc", "aa", "ra"])
def test_committed_traffic_summary_is_well_formed(which):
    path = {"jc": bench.TRAFFIC_FILE, "aa": bench.TRAFFIC_FILES_CL8M[("AA", 32)],
            "ra": bench.TRAFFIC_FILES_CL8M[("RA", 256)]}[which]
    with open(path) as fh:
        lines = fh.read().splitlines()
    assert sum(l.startswith("source_sha256: ") for l in lines) == 1
    assert any("rocprofv3 --pmc FETCH_SIZE" in l for l in lines)
    rows = [l for l in lines if l.startswith("traffic_bytes_per_launch ")]
    assert rows
    for l in rows:
        name, val = l[len("traffic_bytes_per_launch "):].rsplit("=", 1)
        assert name.strip().startswith("acc_")
        assert float(val) > 0


def test_launch_bytes():
    b = dict(sources=3, first_order=10, arcs=7, wedges=100, candidates=40)
    base = 8 * 3 + 8 * 10 + 4 * 7 + 4 * 100
    assert bench.launch_bytes(b, True) == base + 4 * 40
    assert bench.launch_bytes(b, False) == base


def test_algorithmic_bytes_on_a_path():
    # path 0-1-2-3: degrees 1, 2, 2, 1; n = 4, A = 6
    deg = np.array([1, 2, 2, 1])
    # L = 1: only the two ends may serve as intermediates (A_L = 2)
    assert bench.algorithmic_bytes(deg, 1, wedges=0, candidates=0, k_out=0) == 8 * 4 + 8 * 6 + 4 * 2
    # no hub limit: A_L = A; the two wedges 0-1-2 and 1-2-3, two candidates, two rows out
    full = 8 * 4 + 8 * 6 + 4 * 6 + 4 * 2 + 12 * 2
    assert bench.algorithmic_bytes(deg, None, wedges=2, candidates=2, k_out=2) == full + 4 * 2
    assert bench.algorithmic_bytes(deg, None, 2, 2, 2, normalised=False) == full


def test_observed_graph_cache(tmp_path):
    """The cached observed graph equals a fresh one (same holdout, same k)."""
    import synth
    make = lambda: synth.chung_lu(3000, 8.0, 2.3, 3)  # noqa: E731
    fresh, k = bench.observed_graph(synth, "cl3k", "", make)
    first, k1 = bench.observed_graph(synth, "cl3k", str(tmp_path), make)
    assert (tmp_path / "cl3k_obs.npz").exists()
    again, k2 = bench.observed_graph(synth, "cl3k", str(tmp_path), lambda: None)
    for g in (first, again):
        assert np.array_equal(g.offsets, fresh.offsets) and np.array_equal(g.indices, fresh.indices)
    assert k == k1 == k2 > 0


def test_cpu_model_is_a_name():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
