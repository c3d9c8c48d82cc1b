"""Host logic of the autotuner (coordinate descent over the scheduler knobs),
driven by a synthetic cost model instead of the device."""
from paper_2401_11415_amd import tune


class FakeDevice:
    """run() advances a fake clock by the cost of the knobs last applied."""

    def __init__(self, cost):
        self.cost = cost
        self.t = 0.0
        self.current = None
        self.applied = []

    def apply(self, g, setting):
        self.current = dict(setting)
        self.applied.append(dict(setting))

    def run(self):
        self.t += self.cost(self.current)

    def clock(self):
        return self.t


def test_picks_best_per_knob_and_ignores_noise():
    def cost(s):
        c = 0.010
        if s["bucket_max0"] == 16:
            c -= 0.003
        if s["lds_wedge_cap"] == 32768:
            c -= 0.0001  # 1.4 %: below the default min_gain
        if s["sample_budget"] == 1 << 20:
            c += 0.005
        return c

    dev = FakeDevice(cost)
    res = tune.autotune("g", dev.run, apply_fn=dev.apply, clock=dev.clock)
    assert abs(res["default_ms"] - 10.0) < 1e-9
    assert abs(res["ms"] - 7.0) < 1e-9
    best = res["setting"]
    assert best["bucket_max0"] == 16
    assert best["lds_wedge_cap"] == tune.DEFAULT_SPACE["lds_wedge_cap"][0]
    assert best["sample_budget"] == tune.DEFAULT_SPACE["sample_budget"][0]
    assert dev.applied[-1] == best
    n_trials = 1 + sum(len(v) - 1 for v in tune.DEFAULT_SPACE.values())
    assert len(res["trials"]) == n_trials


def test_second_sweep_finds_coupled_gain():
    # bucket_max0 = 16 only pays once global_slots = 512, a knob tried later
    def cost(s):
        c = 0.010
        if s["global_slots"] == 512:
            c -= 0.001
            if s["bucket_max0"] == 16:
                c -= 0.004
        return c

    one = FakeDevice(cost)
    r1 = tune.autotune("g", one.run, apply_fn=one.apply, clock=one.clock, sweeps=1)
    assert r1["setting"]["global_slots"] == 512 and r1["setting"]["bucket_max0"] == 32
    two = FakeDevice(cost)
    r2 = tune.autotune("g", two.run, apply_fn=two.apply, clock=two.clock, sweeps=2)
    assert r2["setting"]["bucket_max0"] == 16 and abs(r2["ms"] - 5.0) < 1e-9


def test_apply_maps_setting_to_set_tuning(monkeypatch):
    seen = {}

    def fake_set_tuning(g, **kw):
        seen.update(kw)

    monkeypatch.setattr(tune, "set_tuning", fake_set_tuning)
    tune.apply("g", {"bucket_max0": 16, "bucket_max3": 1536, "lds_wedge_cap": 4096,
                     "global_slots": 128, "sample_budget": 1 << 20, "mid1_shape": "workgroup128"})
    assert seen == {"lds_wedge_cap": 4096, "global_slots": 128, "sample_budget": 1 << 20,
                    "bucket_max": [16, 256, 1024, 1536, 4096], "tiny_batch": 0, "small_batch": 0,
                    "small_shape": 0, "mid1_shape": "workgroup128"}
