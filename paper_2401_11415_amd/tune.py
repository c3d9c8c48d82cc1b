"""Autotuner of the scheduler knobs (lp_set_tuning) for one resident graph and
one workload.

The knobs move work between kernels without changing any result: the bucket
bounds decide which kernel a source meets (48, 8 or 2 sources per 256-lane
workgroup for the three batch buckets, one per 256, 512 or 1024 lanes above),
the batch knobs set how many tiny (48 or 32) and small (8 or 4) sources share
a workgroup, the shape knobs pick the kernel of the small and mid1 buckets
(batches, one source per wave, per 128 or per 256 lanes),
the LDS cap decides which sources take the global-memory accumulator, and the
sample budget sizes the pass that sets the top-k threshold.  The tuner runs
the caller's workload under each setting and keeps what is fastest, by
coordinate descent: one knob at a time, the others held at the best setting so
far, a change kept only when it gains more than ``min_gain`` on the median of
``repeats`` runs.
"""
from __future__ import annotations

import time

from . import BUCKET_MAX_DEFAULT, set_tuning

# knob -> candidate values (the first is the default)
DEFAULT_SPACE = {
    "tiny_batch": (48, 32),
    "small_batch": (8, 4),
    "small_shape": (0, "batch", "wave", "workgroup128"),  # 0: the library's default
    "mid1_shape": (0, "batch", "workgroup128", "workgroup256"),
    "bucket_max0": (32, 24, 16),
    "bucket_max1": (256, 192, 128, 64),
    "bucket_max2": (1024, 768, 512),
    "bucket_max3": (2048, 1536),
    "bucket_max4": (4096, 3072),
    "lds_wedge_cap": (65536, 32768, 16384, 131072, 262144),
    "global_slots": (0, 128, 512),
    "sample_budget": (0, 1 << 20, 1 << 22, 1 << 24),  # 0: the library's default rule
}


def default_setting(space=None) -> dict:
    space = space or DEFAULT_SPACE
    return {knob: values[0] for knob, values in space.items()}


def apply(g, setting: dict) -> None:
    """Set g's knobs from a setting dict (keys of DEFAULT_SPACE)."""
    bm = [int(setting.get(f"bucket_max{b}", BUCKET_MAX_DEFAULT[b])) for b in range(5)]
    set_tuning(g, lds_wedge_cap=int(setting.get("lds_wedge_cap", 0)),
               global_slots=int(setting.get("global_slots", 0)),
               sample_budget=int(setting.get("sample_budget", 0)), bucket_max=bm,
               tiny_batch=int(setting.get("tiny_batch", 0)),
               small_batch=int(setting.get("small_batch", 0)),
               small_shape=setting.get("small_shape", 0), mid1_shape=setting.get("mid1_shape", 0))


def _median(xs):
    xs = sorted(xs)
    m = len(xs) // 2
    return xs[m] if len(xs) % 2 else 0.5 * (xs[m - 1] + xs[m])


def autotune(g, run, space=None, repeats: int = 3, min_gain: float = 0.04, sweeps: int = 1,
             clock=time.perf_counter, apply_fn=apply, log=None) -> dict:
    """Tune g's knobs for the workload ``run()`` (which must return only once
    its device work has finished).  Leaves g set to the best setting found and
    returns {"setting", "ms", "default_ms", "trials"}; trials lists every
    (setting, median ms) measured."""
    space = space or DEFAULT_SPACE
    trials = []

    def measure(setting):
        apply_fn(g, setting)
        run()  # first run after a change may grow buffers: not timed
        ts = []
        for _ in range(max(1, repeats)):
            t0 = clock()
            run()
            ts.append((clock() - t0) * 1e3)
        ms = _median(ts)
        trials.append((dict(setting), ms))
        if log:
            log(f"tune {setting} -> {ms:.3f} ms")
        return ms

    best = default_setting(space)
    best_ms = default_ms = measure(best)
    for _ in range(max(1, sweeps)):
        changed = False
        for knob, values in space.items():
            for v in values:
                if v == best[knob]:
                    continue
                cand = dict(best)
                cand[knob] = v
                ms = measure(cand)
                if ms < best_ms * (1.0 - min_gain):
                    best, best_ms, changed = cand, ms, True
        if not changed:
            break
    apply_fn(g, best)
    return {"setting": best, "ms": best_ms, "default_ms": default_ms, "trials": trials}
