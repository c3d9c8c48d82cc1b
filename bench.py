"""Benchmark: DLH Jaccard link prediction on one MI355X.

Workload: R-MAT scale 22 (4,194,304 vertices, edge factor 16, a/b/c/d =
0.57/0.19/0.19/0.05, seed 1), symmetrised, self-loops and duplicates removed,
10% of edges held out uniformly at random (seed 1); predict k = |held out|
edges with the Jaccard coefficient, hub limit 256 (DLH).  One step = one
lp_predict call: plan, two-hop accumulation, fused scoring, top-k and result
hand-off, with the graph resident in HBM.

Prints one JSON line (metric, value, roofline, cpu_baseline, ...).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
PAPER_DLH_EDGES_PER_S = 38.1e6  # sk-2005, 2x Xeon Gold 6226R (context only)

# Main-pass accumulation kernel of each scheduling bucket (count tables: CN,
# JC, ..., LHN; weighted tables: AA, RA), as rocprofv3 names them, for graphs
# with fewer than 2^25 - 1 vertices (the batched small-source kernels, packed
# weighted tables).  The
# sampling pass runs the same code as separate instantiations (last template
# argument true).
BUCKET_KERNELS = {
    False: {"tiny": "acc_batch_kernel<256, 48, 3072, 0, 64, false>",
            "small": "acc_batch_kernel<256, 8, 3072, 0, 64, false>",
            "mid1": "acc_batch_kernel<512, 4, 6144, 0, 64, false>",
            "mid2": "acc_lds_kernel<256, 256, 3072, 0, false, 64, false>",
            "mid3": "acc_lds_kernel<512, 512, 6144, 0, false, 64, false>",
            "large": "acc_lds_kernel<1024, 1024, 14336, 0, false, 64, false>",
            "global": "acc_spa_kernel<false, false, false>"},
    # packed weighted tables (graphs below 2^25 - 1 vertices)
    True: {"tiny": "acc_batch_kernel<256, 48, 2432, 2, 64, false>",
           "small": "acc_batch_kernel<256, 8, 2816, 2, 64, false>",
           "mid1": "acc_batch_kernel<512, 4, 5760, 2, 64, false>",
           "mid2": "acc_lds_kernel<256, 256, 3008, 2, false, 64, false>",
           "mid3": "acc_lds_kernel<512, 512, 6016, 2, false, 64, false>",
           "large": "acc_lds_kernel<1024, 1024, 12032, 2, false, 64, false>",
           "global": "acc_spa_kernel<true, false, false>",
           "split": "acc_lds_kernel<1024, 1024, 7680, 1, false, 64, false>"},
}
KERNEL_SOURCES = ["paper_2401_11415_amd/csrc/predict.hip", "paper_2401_11415_amd/csrc/kernels.h",
                  "paper_2401_11415_amd/csrc/lp_common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "acc_kernels_rmat22_dlh_jc_traffic.txt")
# the weighted workloads share kernel names (AA and RA run the same packed
# tables), so each (measure, hub limit) has a summary of its own
TRAFFIC_FILES_CL8M = {
    ("AA", 32): os.path.join(ROOT, "profiles", "acc_kernels_chunglu8m_dlh_aa_l32_traffic.txt"),
    ("RA", 256): os.path.join(ROOT, "profiles", "acc_kernels_chunglu8m_dlh_ra_l256_traffic.txt"),
}
CHUNG_LU_8M = "Chung-Lu 8M vertices, mean degree 40, exponent 2.1, w_max 2e5, seed 1"


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def launch_bytes(b, normalised):
    """Algorithmic bytes of the accumulation launches of one bucket: per source
    its two row offsets (8 B), its row and the degree of every neighbour for
    the hub test (8 B per first-order neighbour), the row start of every
    explored intermediate (4 B per arc), one id per wedge (4 B), and deg[c]
    per distinct candidate for the normalised measures (4 B)."""
    return (8 * b["sources"] + 8 * b["first_order"] + 4 * b["arcs"] + 4 * b["wedges"]
            + (4 * b["candidates"] if normalised else 0))


def measured_traffic(kernel, path=None):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary at `path`, or None when it is missing or was taken on
    other kernel sources (path None: the R-MAT-22 Jaccard summary; "": a
    workload no summary covers)."""
    path = TRAFFIC_FILE if path is None else path
    if not path or not os.path.exists(path):
        return None
    rec, rows = {}, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_sha256:"):
                rec["hash"] = line.split(":", 1)[1].strip()
            elif line.startswith("traffic_bytes_per_launch "):
                name, val = line[len("traffic_bytes_per_launch "):].rsplit("=", 1)
                rows[name.strip()] = float(val)
    if rec.get("hash") != kernel_source_hash():
        return None
    return rows.get(kernel)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(deg, L, wedges, candidates, k_out, normalised=True):
    """Bytes the method must move per prediction (u32 offsets / ids):
    source offsets 2*4n, source rows 4A, first-hop lookups 4A, explored
    intermediate rows 4*A_L, one id per wedge 4*W_L, deg[c] per candidate for
    the normalised measures, 12 bytes per output row."""
    n = deg.shape[0]
    A = int(deg.sum())
    lim = np.inf if L is None else L
    A_L = int(deg[deg <= lim].sum())
    b = 8 * n + 8 * A + 4 * A_L + 4 * wedges + 12 * k_out
    if normalised:
        b += 4 * candidates
    return b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--hub", type=int, default=256)
    ap.add_argument("--measure", default="JC")
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--graph", default="rmat", choices=["rmat", "chung-lu-8m"],
                    help="rmat: R-MAT at --scale; chung-lu-8m: the AA / RA workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the weighted-measure workload (Chung-Lu 8M, AA L=32 and RA L=256)")
    ap.add_argument("--no-digest", action="store_true",
                    help="skip the untimed lp_fingerprint call that counts |C_L| (it launches the "
                         "same kernels as lp_predict; profiles of the timed launches leave it out)")
    ap.add_argument("--secondary-steps", type=int, default=5)
    ap.add_argument("--serve-qps", type=float, default=500.0,
                    help="offered rate of the serving part of the secondary block")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--cache", default="", metavar="DIR",
                    help="keep generated observed graphs in DIR (npz) for later runs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (scales HBM counters)")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload instead: Poisson query stream through lp_server")
    ap.add_argument("--qps", type=float, default=200.0, help="--serve: request arrival rate")
    ap.add_argument("--requests", type=int, default=600, help="--serve: requests in the stream")
    ap.add_argument("--slots", type=int, default=2, help="--serve: concurrent batches")
    ap.add_argument("--host-launches", action="store_true",
                    help="--serve: launch every batch from the host instead of replaying captured graphs")
    ap.add_argument("--sweep", action="store_true",
                    help="hub-limit sweep instead: time and holdout precision / recall / F1 per "
                         "measure and L")
    ap.add_argument("--measures", default="", help="--sweep: comma-separated measures (default all)")
    ap.add_argument("--multi", action="store_true",
                    help="batched workload instead: many uneven graphs in one lp_predict_multi "
                         "call (default and autotuned knobs) vs one lp_predict call per graph")
    ap.add_argument("--graphs", type=int, default=512, help="--multi: number of graphs")
    ap.add_argument("--n-max", type=int, default=1_000_000, help="--multi: largest graph size")
    ap.add_argument("--one-call-only", action="store_true",
                    help="--multi: time only the one-call path with default knobs (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy << 18
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))
        return

    import paper_2401_11415_amd as lp
    import synth

    if args.serve:
        serve(args, lp, synth, torch)
        return
    if args.sweep:
        sweep(args, lp, synth, torch)
        return
    if args.multi:
        multi(args, lp, synth, torch)
        return

    t0 = time.time()
    if args.graph == "rmat":
        workload = f"R-MAT scale {args.scale}, edge factor 16 (0.57/0.19/0.19/0.05), seed 1"
        traffic_file = TRAFFIC_FILE if (args.scale, args.measure.upper(), args.hub) == (22, "JC", 256) else ""
        obs, k = observed_graph(synth, f"rmat{args.scale}", args.cache,
                                lambda: synth.rmat(args.scale, 16.0, 0.57, 0.19, 0.19, seed=1))
    else:
        workload = CHUNG_LU_8M
        traffic_file = TRAFFIC_FILES_CL8M.get((args.measure.upper(), args.hub), "")
        obs, k = observed_graph(synth, "chung_lu_8m", args.cache, lambda: synth.chung_lu_8m(seed=1))
    log(f"graph: n={obs.n} m={obs.m} k={k} ({time.time() - t0:.1f}s)")
    torch.cuda.set_device(0)
    L = args.hub
    r = measure_predict(lp, torch, obs, args.measure.upper(), L, k, args.steps, args.warmup, traffic_file,
                        digest=not args.no_digest)
    ms_per_step = r["ms_per_step"]
    res = {
        "metric": "predicted edges/s (DLH, Jaccard)" if args.measure.upper() == "JC"
                  else f"predicted edges/s (DLH, {args.measure.upper()})",
        "value": r["value"],
        "unit": "edges/s",
        "n_gpus": 1,
        # one graph whose sources would be split across GPUs: total work is fixed
        "scaling": "strong",
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "u32 counts, f64 scores",
        "data": "synthetic",
        "config": {
            "workload": f"{workload}, 10% holdout; DLH {args.measure.upper()}, hub limit {L}, "
                        f"k=|held out|",
            "vertices": obs.n, "observed_edges": obs.m, "k": k, "hub_limit": L,
            "measure": args.measure.upper(),
        },
        "roofline": r["roofline"],
        "kernels": r["kernels"],
        "whole_call": r["whole_call"],
        "context": {"paper_dlh_edges_per_s": PAPER_DLH_EDGES_PER_S,
                    "paper_workload": "sk-2005, 2x Xeon Gold 6226R, 32 threads"},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(obs, L, args.measure, k, args.cpu_seconds)
    del obs
    if args.graph == "rmat" and not args.no_secondary:
        res["secondary"] = secondary(lp, torch, synth, args)
    print(json.dumps(res), flush=True)


def observed_graph(synth, name, cache, make):
    """The observed graph of a workload (its generator's output with 10% of
    the edges held out, seed 1) and k = |held out|; with a cache folder, the
    arrays are stored there on first use and loaded afterwards."""
    path = os.path.join(cache, f"{name}_obs.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        return synth.Graph(z["offsets"], z["indices"]), int(z["k"])
    full = make()
    obs, held = synth.holdout(full, 0.1, seed=1)
    k = int(held.shape[0])
    del full, held
    if path:
        os.makedirs(cache, exist_ok=True)
        np.savez(path, offsets=obs.offsets, indices=obs.indices, k=np.int64(k))
    return obs, k


def measure_predict(lp, torch, obs, measure, L, k, steps, warmup, traffic_file, digest=True):
    """Time `steps` lp_predict calls (after `warmup`) on the resident graph and
    derive the per-kernel rates, the dominant kernel's roofline and the
    whole-call byte model (digest=False: |C_L| is not counted, and the
    all-candidates figures are left out)."""
    stream = torch.cuda.current_stream()
    g = lp.Graph(obs.offsets, obs.indices)
    dev = torch.device("cuda", 0)
    out = (torch.empty(k, dtype=torch.int32, device=dev), torch.empty(k, dtype=torch.int32, device=dev),
           torch.empty(k, dtype=torch.float32, device=dev))
    for i in range(warmup):
        lp.predict(g, measure, L, k, out=out)
        log(f"{measure} L={L} warmup {i}: {lp.last_stats(g)['ms_total']:.3f} ms")
    torch.cuda.synchronize()
    acc_ms, tot_ms = [], []
    per_bucket = {}
    t_start = time.perf_counter()
    for i in range(steps):
        a, c, s = lp.predict(g, measure, L, k, out=out)
        st = lp.last_stats(g)
        acc_ms.append(st["ms_accumulate"])
        tot_ms.append(st["ms_total"])
        for name, b in st["launches"].items():
            acc = per_bucket.setdefault(name, dict.fromkeys(b, 0))
            for f, v in b.items():
                acc[f] += v
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_start) * 1e3
    ms_per_step = wall_ms / steps
    k_out = int(a.shape[0])
    stats = lp.last_stats(g)
    normalised = measure not in ("CN", "AA", "RA")
    weighted = measure in ("AA", "RA")
    # candidates the kernels accumulated (after each source's degree cutoff)
    # and |C_L| itself (the digest call counts every candidate; not timed)
    if stats["retries"] == 0:
        n_acc = sum(b["candidates"] for b in stats["launches"].values()) + \
            sum(b["candidates"] for b in stats["sampled"].values())
    else:
        n_acc = None
    n_cand = lp.fingerprint(g, L)[0] if digest else None
    if n_acc is None:
        n_acc = n_cand if n_cand is not None else stats["wedges"]
    g.close()
    deg = np.diff(obs.offsets)
    B = algorithmic_bytes(deg, L, stats["wedges"], n_acc, k_out, normalised=normalised)
    B_all = None if n_cand is None else algorithmic_bytes(deg, L, stats["wedges"], n_cand, k_out,
                                                          normalised=normalised)
    tot_med = float(np.median(tot_ms))
    kernels = {}
    for name, b in per_bucket.items():
        if b["launches"] == 0:
            continue
        nb = launch_bytes(b, normalised)
        kernels[name] = {
            "kernel": BUCKET_KERNELS[weighted][name], "launches": b["launches"],
            "avg_launch_ms": b["ms"] / b["launches"],
            "algorithmic_bytes_per_launch": nb / b["launches"],
            "wedges_per_launch": b["wedges"] / b["launches"],
            "gbs": nb / (b["ms"] * 1e-3) / 1e9, "share_of_step": b["ms"] / steps / ms_per_step}
    dom = max(kernels, key=lambda n: kernels[n]["avg_launch_ms"] * kernels[n]["launches"])
    dk = kernels[dom]
    achieved = dk["gbs"]
    traffic = measured_traffic(dk["kernel"], traffic_file)
    return {
        "value": k_out / (ms_per_step * 1e-3),
        "ms_per_step": ms_per_step,
        "k_out": k_out,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": dk["kernel"],
            "bucket": dom,
            "algorithmic_bytes_per_launch": dk["algorithmic_bytes_per_launch"],
            "avg_launch_ms": dk["avg_launch_ms"],
            "kernel_source_sha256": kernel_source_hash(),
        },
        "kernels": kernels,
        "whole_call": {"algorithmic_bytes": B, "ms_device_median": tot_med,
                       "ms_accumulate_median": float(np.median(acc_ms)),
                       "frac_hbm": B / (tot_med * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       # the same with every candidate of C_L charged 4 B of deg[c]
                       "algorithmic_bytes_all_candidates": B_all,
                       "frac_hbm_all_candidates": (None if B_all is None else
                                                   B_all / (tot_med * 1e-3) / 1e9 / HBM_PEAK_GBS),
                       "wedges": stats["wedges"], "candidates": n_cand, "candidates_accumulated": n_acc,
                       "appended": stats["appended"], "retries": stats["retries"],
                       "ms_plan": stats["ms_plan"], "ms_select": stats["ms_select"],
                       "wedges_per_s": stats["wedges"] / (ms_per_step * 1e-3)},
    }


def secondary(lp, torch, synth, args):
    """The other workloads, one JSON block each: the weighted measures on the
    social-network stand-in (Chung-Lu 8M), DLH Adamic-Adar at L = 32 and
    resource allocation at L = 256 (the hub limits the paper picks for them),
    k = |held out|; and p50 / p99 latency of the serving loop on R-MAT scale 24
    (DLH AA, L = 32, top-10 per source) at a fixed offered rate."""
    t0 = time.time()
    obs, k = observed_graph(synth, "chung_lu_8m", args.cache, lambda: synth.chung_lu_8m(seed=1))
    log(f"secondary graph: n={obs.n} m={obs.m} k={k} ({time.time() - t0:.1f}s)")
    out = {}
    for measure, L in (("AA", 32), ("RA", 256)):
        r = measure_predict(lp, torch, obs, measure, L, k, args.secondary_steps, 2,
                            TRAFFIC_FILES_CL8M[(measure, L)])
        out[f"{measure}_L{L}"] = {
            "workload": f"{CHUNG_LU_8M}, 10% holdout; DLH {measure}, hub limit {L}, k=|held out|",
            "metric": f"predicted edges/s (DLH, {measure})", "value": r["value"], "unit": "edges/s",
            "ms_per_step": r["ms_per_step"], "steps": args.secondary_steps, "k": k,
            "roofline": r["roofline"], "kernels": r["kernels"], "whole_call": r["whole_call"]}
        log(f"secondary {measure} L={L}: {r['ms_per_step']:.2f} ms, dominant "
            f"{r['roofline']['bucket']} at {r['roofline']['frac'] * 100:.1f}% of HBM peak")
    del obs
    # the serving workload (R-MAT scale 24) at a fixed offered rate
    out["serve_rmat24_AA_L32"] = run_serve(lp, synth, torch, 24, 32, "AA", args.serve_qps,
                                           args.serve_requests, 2, args.cache)
    log(f"secondary serving: p50 {out['serve_rmat24_AA_L32']['p50_ms']:.2f} ms, "
        f"p99 {out['serve_rmat24_AA_L32']['p99_ms']:.2f} ms")
    return out


def sweep(args, lp, synth, torch):
    """Hub-limit sweep (the paper's Section 4.4 experiment on a synthetic
    stand-in): the benchmark graph, every measure (or --measures), L in
    {2, 4, ..., 1024} and IBase; per (measure, L) the device time of
    lp_predict (median of the timed calls after a warm-up), the wedges and
    candidates it handles, the speedup over IBase, and the quality of the k
    predictions against the held-out edges (Section 3.2: precision, recall,
    F1)."""
    full = synth.rmat(args.scale, 16.0, 0.57, 0.19, 0.19, seed=1)
    obs, held = synth.holdout(full, 0.1, seed=1)
    k = int(held.shape[0])
    del full
    hu = np.minimum(held[:, 0], held[:, 1]).astype(np.int64)
    hv = np.maximum(held[:, 0], held[:, 1]).astype(np.int64)
    held_keys = np.sort(hu * obs.n + hv)
    torch.cuda.set_device(0)
    g = lp.Graph(obs.offsets, obs.indices)
    measures = [m.strip().upper() for m in args.measures.split(",")] if args.measures else list(lp.MEASURES)
    limits = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, None]
    table = {}
    for measure in measures:
        rows = []
        for L in limits:
            timed = 3 if (L is not None and L <= 256) else 2
            lp.predict(g, measure, L, k)
            ms, st = [], None
            for _ in range(timed):
                a, c, s = lp.predict(g, measure, L, k)
                st = lp.last_stats(g)
                ms.append(st["ms_total"])
            a = a.cpu().numpy().astype(np.int64)
            c = c.cpu().numpy().astype(np.int64)
            hits = int(np.isin(a * obs.n + c, held_keys, assume_unique=False).sum())
            k_out = int(a.shape[0])
            prec = hits / max(k_out, 1)
            rec = hits / max(k, 1)
            f1 = 2 * prec * rec / (prec + rec) if prec + rec > 0 else 0.0
            row = {"L": L if L is not None else "IBase", "ms": float(np.median(ms)), "wedges": st["wedges"],
                   "k_out": k_out, "hits": hits, "precision": prec, "recall": rec, "f1": f1,
                   "ms_accumulate": st["ms_accumulate"], "ms_select": st["ms_select"],
                   "appended": st["appended"], "retries": st["retries"],
                   "ms_calls": [float(x) for x in ms]}
            rows.append(row)
            log(measure, json.dumps(row))
        ib = rows[-1]["ms"]
        for r in rows:
            r["speedup_vs_ibase"] = ib / r["ms"]
        table[measure] = rows
    g.close()
    print(json.dumps({"sweep": f"R-MAT scale {args.scale}, DLH, k=|held out|={k}", "measures": table}),
          flush=True)


def serve(args, lp, synth, torch):
    measure = "AA" if args.measure.upper() == "JC" else args.measure.upper()
    res = run_serve(lp, synth, torch, args.scale, args.hub, measure, args.qps, args.requests, args.slots,
                    args.cache, host_launches=args.host_launches)
    print(json.dumps(res), flush=True)


def run_serve(lp, synth, torch, scale, L, measure, qps, n_requests, slots, cache="", host_launches=False):
    """Serving workload: a device-resident R-MAT graph (scale `scale`, edge
    factor 16, symmetrised, no holdout); requests arrive as a Poisson stream at
    `qps`, each with a log-uniform number of sources in [1, 4096] drawn with
    probability proportional to degree; each asks for the top 10 per source
    by DLH `measure` (hub limit L).  Latency is submit -> results in the
    caller's buffers, on the host clock.  Batches replay captured HIP graphs
    unless host_launches."""
    import threading
    t0 = time.time()
    path = os.path.join(cache, f"rmat{scale}_full.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        gr = synth.Graph(z["offsets"], z["indices"])
    else:
        gr = synth.rmat(scale, 16.0, 0.57, 0.19, 0.19, seed=1)
        if path:
            os.makedirs(cache, exist_ok=True)
            np.savez(path, offsets=gr.offsets, indices=gr.indices)
    log(f"graph: n={gr.n} m={gr.m} ({time.time() - t0:.1f}s)")
    torch.cuda.set_device(0)
    g = lp.Graph(gr.offsets, gr.indices)
    deg = gr.degrees().astype(np.float64)
    nz = np.nonzero(deg > 0)[0]
    p = deg[nz] / deg[nz].sum()
    rng = np.random.default_rng(2024)
    kq = 10
    sizes = np.exp(rng.uniform(0.0, np.log(4096.0), n_requests)).astype(np.int64)
    cdf = np.cumsum(p)
    reqs = [nz[np.minimum(np.searchsorted(cdf, rng.uniform(0, cdf[-1], int(s))), nz.shape[0] - 1)]
            .astype(np.int32) for s in sizes]
    gaps = rng.exponential(1.0 / qps, n_requests)
    srv = lp.Server(g, slots=slots, host_launches=host_launches)
    for r in reqs[:8]:  # warm-up: buffers grow to their working size
        srv.wait(srv.submit(r, measure, L, kq))
    tickets = [None] * len(reqs)

    def producer():
        t_next = time.perf_counter()
        for i, r in enumerate(reqs):
            t_next += gaps[i]
            d = t_next - time.perf_counter()
            if d > 0:
                time.sleep(d)
            tickets[i] = srv.submit(r, measure, L, kq)

    t_start = time.perf_counter()
    th = threading.Thread(target=producer)
    th.start()
    lat, run, rows, batches, replayed = [], [], 0, {}, 0
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0002)
        out, rec = srv.wait(tickets[i])
        lat.append(rec["total_ms"])
        run.append(rec["run_ms"])
        rows += int(out[2].sum())
        batches[rec["batch"]] = rec["batch_requests"]
        replayed += rec["replayed"] == 1
        if (i + 1) % 100 == 0:
            log(f"served {i + 1}/{len(reqs)}")
    th.join()
    wall = time.perf_counter() - t_start
    srv.close()
    n, m = gr.n, gr.m
    g.close()
    lat = np.array(lat)
    return {"metric": f"query latency p50/p99 and predicted edges/s (served, DLH {measure} top-{kq})",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "value": rows / wall, "unit": "edges/s",
            "batch_run_ms_p50": float(np.percentile(run, 50)),
            "replayed_share": replayed / len(reqs), "host_launches": bool(host_launches),
            "sources_per_s": float(sizes.sum()) / wall, "requests": len(reqs),
            "offered_qps": qps, "achieved_qps": len(reqs) / wall, "slots": slots,
            "batches": len(batches), "mean_requests_per_batch": float(np.mean(list(batches.values()))),
            "data": "synthetic",
            "config": {"workload": f"R-MAT scale {scale}, edge factor 16, seed 1; Poisson "
                                   f"arrivals, 1-4096 sources per request (log-uniform, "
                                   f"degree-biased); DLH {measure} L={L}, top-{kq} per source",
                       "vertices": n, "edges": m}}


def multi(args, lp, synth, torch):
    """Batched workload: --graphs independent Chung-Lu graphs of uneven size
    (vertices log-uniform in [1000, --n-max], mean degree uniform in [8, 32],
    exponent 2.3, graph i seeded 1000 + i, sizes drawn with seed 5), used as
    observed graphs (no holdout); graph i predicts k_i = m_i // 10 edges by
    DLH Jaccard (hub limit --hub).  Times one lp_predict_multi call over the
    disjoint union (default knobs, then the knobs the autotuner picks)
    against one lp_predict call per graph with each graph resident on its own.
    Every timed call returns after its device work; the host clock brackets
    it, so launch and host overheads count on both sides."""
    from paper_2401_11415_amd import tune
    t0 = time.time()
    graphs = synth.chung_lu_batch(
        args.graphs, 1000, args.n_max, seed=5,
        progress=lambda i: (i + 1) % 64 == 0 and log(f"generated {i + 1}/{args.graphs} graphs "
                                                     f"({time.time() - t0:.1f}s)"))
    ks = np.array([gr.m // 10 for gr in graphs], dtype=np.int64)
    union, vstart = synth.disjoint_union(graphs)
    log(f"union: n={union.n} m={union.m} sum k={int(ks.sum())} ({time.time() - t0:.1f}s)")
    torch.cuda.set_device(0)
    L, measure = args.hub, args.measure.upper()
    g = lp.Graph(union.offsets, union.indices)
    n_union, m_union = union.n, union.m
    del union

    def run():
        out = lp.predict_multi(g, vstart, ks, measure, L)
        torch.cuda.synchronize()
        return out

    def timed(steps):
        ts = []
        for _ in range(steps):
            t = time.perf_counter()
            out = run()
            ts.append((time.perf_counter() - t) * 1e3)
        return float(np.median(ts)), float(np.mean(ts)), out

    for i in range(args.warmup):
        run()
        log(f"multi warmup {i}: {lp.last_stats(g)['ms_total']:.3f} ms device")
    med_default, mean_default, out = timed(args.steps)
    stats_default = lp.last_stats(g)
    k_out = sum(int(a.shape[0]) for a, _, _ in out)
    log(f"one call, default knobs: median {med_default:.3f} ms")
    if args.one_call_only:
        g.close()
        print(json.dumps({"metric": "several-graph call only (default knobs)", "ms_per_step": med_default,
                          "value": k_out / (med_default * 1e-3), "unit": "edges/s",
                          "device_ms": stats_default["ms_total"], "graphs": args.graphs}), flush=True)
        return
    tuned = tune.autotune(g, run, repeats=3, log=log)
    for i in range(args.warmup):
        run()
    med_tuned, mean_tuned, out = timed(args.steps)
    stats_tuned = lp.last_stats(g)
    log(f"one call, tuned knobs {tuned['setting']}: median {med_tuned:.3f} ms")
    g.close()

    per_graph_ms = []
    for i, gr in enumerate(graphs):
        gi = lp.Graph(gr.offsets, gr.indices)
        k = int(ks[i])
        dev = torch.device("cuda", 0)
        buf = (torch.empty(max(k, 1), dtype=torch.int32, device=dev),
               torch.empty(max(k, 1), dtype=torch.int32, device=dev),
               torch.empty(max(k, 1), dtype=torch.float32, device=dev))
        for _ in range(max(1, args.warmup)):
            lp.predict(gi, measure, L, k, out=buf)
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            t = time.perf_counter()
            lp.predict(gi, measure, L, k, out=buf)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        per_graph_ms.append(float(np.median(ts)))
        gi.close()
        if (i + 1) % 64 == 0:
            log(f"per-graph calls: {i + 1}/{len(graphs)} graphs, {sum(per_graph_ms):.1f} ms so far")
    loop_ms = float(sum(per_graph_ms))

    def buckets(st):
        return {name: {"sources": b["sources"], "launches": b["launches"], "wedges": b["wedges"],
                       "ms": b["ms"]}
                for name, b in st["launches"].items() if b["launches"]}

    res = {
        "metric": f"predicted edges/s (DLH, {'Jaccard' if measure == 'JC' else measure}), "
                  f"{args.graphs} graphs per call",
        "value": k_out / (med_tuned * 1e-3), "unit": "edges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": med_tuned,
        "higher_is_better": True, "dtype": "u32 counts, f64 scores", "data": "synthetic",
        "ms_one_call_default_knobs": med_default,
        "ms_one_call_per_graph": loop_ms,
        "speedup_vs_one_call_per_graph": loop_ms / med_tuned,
        "speedup_of_tuning": med_default / med_tuned,
        "tuned_knobs": tuned["setting"], "tuning_trials": len(tuned["trials"]),
        "device": {name: {f: st[f] for f in ("ms_total", "ms_plan", "ms_accumulate", "ms_select",
                                             "wedges", "appended", "retries")}
                   for name, st in (("default", stats_default), ("tuned", stats_tuned))},
        "buckets_tuned": buckets(stats_tuned),
        "per_graph_ms": {"min": min(per_graph_ms), "median": float(np.median(per_graph_ms)),
                         "max": max(per_graph_ms)},
        "config": {"workload": f"{args.graphs} Chung-Lu graphs, 1000-{args.n_max} vertices "
                               f"(log-uniform), mean degree 8-32, exponent 2.3, graph i seeded "
                               f"1000 + i; DLH {measure}, hub limit {L}, k_i = m_i / 10",
                   "vertices": n_union, "edges": m_union, "k": int(ks.sum()), "k_out": k_out,
                   "graphs": args.graphs},
    }
    print(json.dumps(res), flush=True)


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(obs, L, measure, k, target_s):
    """The oracle (test infrastructure, untuned) on a uniform sample of sources;
    the full-graph time is extrapolated by the sampled fraction."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(12345)
    nz = np.nonzero(np.diff(obs.offsets) > 0)[0]

    def run(frac):
        src = np.sort(rng.choice(nz, max(1, int(frac * nz.shape[0])), replace=False)).astype(np.int32)
        t = time.perf_counter()
        oracle.predict_sources(obs, L, measure, max(1, int(k * frac)), src, threads=cores)
        return time.perf_counter() - t, src.shape[0]

    t1, _ = run(0.02)
    frac = min(1.0, 0.02 * target_s / max(t1, 1e-3))
    t, ns = run(frac)
    full_s = t / frac
    log(f"cpu oracle: {ns} sources ({frac:.3f}) in {t:.1f}s -> {full_s:.1f}s full")
    return {"value": k / full_s, "unit": "edges/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{ns} uniformly sampled sources ({frac * 100:.1f}% of non-isolated "
                      f"vertices), {t:.1f}s, extrapolated to the full graph ({full_s:.1f}s)"}


if __name__ == "__main__":
    main()
