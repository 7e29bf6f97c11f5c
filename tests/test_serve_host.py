"""Host logic of the request loop and the design-map driver, on the CPU.

The engine is replaced by a stand-in that finishes a request after its step
count has been run; the loop's bookkeeping (arrival replay, polling,
latency percentiles, throughput) is what is checked here.  The engine itself
is exercised on the GPU in test_gpu_engine.py.
"""
import types

import paper_2509_22308_amd.serve as S
import workloads as W


class FakeEngine:
    def __init__(self, budget, slots):
        self.budget, self.slots = budget, slots
        self.reqs = {}
        self.next = 1
        self.finished = 0

    def submit(self, prob):
        t = self.next
        self.next += 1
        self.reqs[t] = {"left": int(prob.steps), "status": "running", "fx": float(prob.radius)}
        return t

    def run(self, steps):
        live = [r for r in self.reqs.values() if r["status"] == "running"]
        for r in live[: self.slots]:
            r["left"] -= steps
            if r["left"] <= 0:
                r["status"] = "done"
                self.finished += 1
        return sum(1 for r in self.reqs.values() if r["status"] == "running")

    def stats(self):
        running = sum(1 for r in self.reqs.values() if r["status"] == "running")
        return {"queued": 0, "resident": running, "finished": self.finished, "bytes_in_use": 0}

    def poll(self, t):
        r = self.reqs[t]
        return r["status"], types.SimpleNamespace(fx=r["fx"], fy=0.0, tz=0.0, total_ms=0.0, loop_ms=0.0,
                                                  as_dict=lambda: {"fx": r["fx"], "fy": 0.0, "tz": 0.0})

    def set_policy(self, policy="fifo", max_slots=0):
        self.policy = policy
        if max_slots:
            self.slots = max_slots

    def four_step_choice(self, precision="fp32"):
        return {"variant": "four-step H16 X4", "ms_per_launch": {}, "tunings": 0}

    def close(self):
        pass


def test_serve_replays_arrivals_and_reports_percentiles(monkeypatch):
    monkeypatch.setattr(S, "Engine", FakeEngine)
    reqs = W.config5_requests(n_req=12, a_min=16, a_max=20)
    out = S.serve(reqs, "fp32", budget_bytes=1 << 30, steps_per_call=4000, time_scale=0.05)
    assert out["requests"] == 12 and out["completed"] == 12
    assert [d["index"] for d in out["done"]] == list(range(12))
    assert all(d["latency_s"] >= 0 for d in out["done"])
    assert out["p50_s"] <= out["p99_s"]
    # results come back attached to the right request (the fake echoes the radius)
    for d in out["done"]:
        assert d["fx"] == reqs[d["index"]][1]["radius"]


def test_design_map_driver_collects_every_result(monkeypatch):
    monkeypatch.setattr(S, "Engine", FakeEngine)
    probs = W.config4_sweep()[:7]
    out = S.run_design_map(probs, "bf16", budget_bytes=1 << 30, steps_per_call=100000)
    assert len(out["results"]) == 7 and all(r["status"] == "done" for r in out["results"])
    assert out["solves_per_hour"] > 0


def test_config_generators_are_seeded_and_in_range():
    a = W.config4_sweep()
    b = W.config4_sweep()
    assert len(a) == 576 and a == b
    assert all(32 <= p["radius"] <= 128 and p["nx"] == 8 * p["radius"] for p in a)
    ratios = sorted({round(p["eps2"] / p["eps1"], 9) for p in a})
    assert len(ratios) == 16 and abs(ratios[0] - 1.1) < 1e-9 and abs(ratios[-1] - 10.0) < 1e-9
    r = W.config5_requests()
    assert len(r) == 256 and all(r[k][0] < r[k + 1][0] for k in range(255))
    assert all(1.5 <= p["eps1"] <= 10 and 0 <= p["phi0"] < 3.1416 for _, p in r)
    mean_gap = r[-1][0] / 256
    assert 0.03 < mean_gap < 0.07  # mean 1/20 s
