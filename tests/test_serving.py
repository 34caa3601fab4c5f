"""Continuous-batching server: scheduler behaviour on the CPU with a simulated
clock and executor; on the GPU, every request's outputs are bit-identical
whether it is served alone or inside a mixed stream of batches."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2402_03060_amd.serve import ModelSpec, Request, Scheduler, poisson_requests, serve


class SimClock:
    """Time advances only when the fake executor works or the loop polls."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5
        return self.t


class FakeExecutor:
    """A batch of model m takes base[m] + per_item[m] * batch seconds of
    simulated time; batches of different models overlap."""

    def __init__(self, clock, base, per_item):
        self.clock, self.base, self.per_item = clock, base, per_item
        self.log = []        # (model, [rid...], start)

    def launch(self, m, reqs):
        start = self.clock.t
        self.log.append((m, [r.rid for r in reqs], start))
        return start + self.base[m] + self.per_item[m] * len(reqs)

    def done(self, end):
        return self.clock.t >= end

    def collect(self, handle, reqs):
        for r in reqs:
            r.result = ("done", r.rid)


MODELS = {"a": ModelSpec("a", 4, 100), "b": ModelSpec("b", 2, 300), "c": ModelSpec("c", 1, 1000)}


def _run(reqs, budget, models=MODELS):
    clock = SimClock()
    ex = FakeExecutor(clock, {"a": 1e-3, "b": 2e-3, "c": 5e-3}, {"a": 1e-4, "b": 2e-4, "c": 1e-3})
    sch = Scheduler(models, budget)
    seen = []
    orig = sch.admit

    def admit(now):
        orig(now)
        seen.append(sch.in_flight_bytes)
    sch.admit = admit
    st = serve(sch, ex, reqs, clock=clock)
    return st, ex, seen, sch


def _reqs(n=200, rate=2000.0, seed=4):
    return poisson_requests({"a": 0.5, "b": 0.3, "c": 0.2}, rate, n, seed, {"a": [0] * 3, "b": [0], "c": [0] * 2})


def test_all_requests_complete_once():
    reqs = _reqs()
    st, ex, _, sch = _run(reqs, 10 ** 9)
    assert st.completed == len(reqs)
    served = sorted(rid for _, rids, _ in ex.log for rid in rids)
    assert served == list(range(len(reqs)))
    assert all(r.result == ("done", r.rid) for r in reqs)
    assert sch.in_flight_bytes == 0 and sch.idle()


def test_budget_never_exceeded_and_queue_used():
    reqs = _reqs(rate=20000.0)
    budget = 2500
    st, ex, seen, _ = _run(reqs, budget)
    assert max(seen) <= budget
    assert st.max_in_flight_bytes <= budget
    assert st.max_host_queue > 0            # the budget held requests back on the host
    assert st.completed == len(reqs)


def test_batches_fifo_per_model_and_bounded():
    reqs = _reqs(rate=20000.0)
    st, ex, _, _ = _run(reqs, 10 ** 9)
    by_model = {}
    for m, rids, _ in ex.log:
        assert 1 <= len(rids) <= MODELS[m].max_batch
        by_model.setdefault(m, []).extend(rids)
    model_of = {r.rid: r.model for r in reqs}
    for m, rids in by_model.items():
        assert all(model_of[i] == m for i in rids)
        assert rids == sorted(rids)          # first come, first served within a model
    # under load the server forms full batches (continuous batching)
    assert max(len(r) for m, r, _ in ex.log if m == "a") == MODELS["a"].max_batch


def test_one_batch_per_model_in_flight_and_models_overlap():
    reqs = _reqs(rate=20000.0)
    clock = SimClock()
    ex = FakeExecutor(clock, {"a": 1e-3, "b": 2e-3, "c": 5e-3}, {"a": 1e-4, "b": 2e-4, "c": 1e-3})
    sch = Scheduler(MODELS, 10 ** 9)
    spans = []
    orig_launch = ex.launch

    def launch(m, rs):
        end = orig_launch(m, rs)
        spans.append((m, clock.t, end))
        return end
    ex.launch = launch
    serve(sch, ex, reqs, clock=clock)
    for m in MODELS:
        s = sorted((a, b) for k, a, b in spans if k == m)
        assert all(s[i][1] <= s[i + 1][0] for i in range(len(s) - 1))
    overlap = any(a1 < b2 and a2 < b1 for (m1, a1, b1) in spans for (m2, a2, b2) in spans if m1 != m2)
    assert overlap


def test_latency_accounting():
    reqs = [Request(0, "a", 0.0, 0), Request(1, "a", 0.0, 0), Request(2, "c", 0.0005, 0)]
    st, ex, _, _ = _run(reqs, 10 ** 9)
    assert st.completed == 3
    for r in reqs:
        assert r.arrival <= r.admitted <= r.started <= r.finished
    lat = sorted(v for vs in st.latencies.values() for v in vs)
    s = st.summary()
    assert s["p50_ms"] == pytest.approx(1e3 * float(np.percentile(lat, 50)), abs=1e-3)
    assert set(s["per_model"]) == {"a", "c"}


def test_request_above_budget_is_an_error():
    with pytest.raises(RuntimeError, match="above the budget"):
        _run([Request(0, "c", 0.0, 0)], 999)


def test_poisson_mix_is_seeded():
    a = _reqs(n=4000, seed=4)
    b = _reqs(n=4000, seed=4)
    assert [(r.model, r.arrival) for r in a] == [(r.model, r.arrival) for r in b]
    frac = {m: sum(r.model == m for r in a) / len(a) for m in "abc"}
    assert abs(frac["a"] - 0.5) < 0.03 and abs(frac["b"] - 0.3) < 0.03 and abs(frac["c"] - 0.2) < 0.03
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 2000.0) < 0.1 / 2000.0


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [False, True])
def test_served_outputs_equal_alone(variant):
    """Three models (ring sizes 2^11, 2^12, 2^12 here) served together from a
    Poisson stream with varying batch sizes: each request's output
    ciphertexts equal those of evaluating its ciphertext alone (default plan,
    and deferred ModDown with the doubling FC sum, which the server runs)."""
    import torch
    import workloads as W
    import paper_2402_03060_amd as P
    from paper_2402_03060_amd.serve import GpuExecutor, prepare_model

    shrink = {"conv1": 11, "lenet1": 12, "cnn1d": 12}
    batches = {"conv1": 4, "lenet1": 3, "cnn1d": 2}
    models = {}
    orig = W.config
    try:
        def small(name):
            c = orig(name)
            c["log_n"] = shrink[name]
            if name == "cnn1d":
                c["samples_per_ct"] = 2
            return c
        W.config = small
        for name in shrink:
            models[name] = prepare_model(P, W, name, batches[name], pool_size=5, seed=40, lazy=variant,
                                         fc_doubling=variant)
    finally:
        W.config = orig
    ex = GpuExecutor(models, keep_results=True)
    specs = {m: d["spec"] for m, d in models.items()}
    reqs = poisson_requests({"conv1": 0.5, "lenet1": 0.3, "cnn1d": 0.2}, 3000.0, 60, 4,
                            {m: list(range(5)) for m in models})
    st = serve(Scheduler(specs, 10 ** 10), ex, reqs)
    torch.cuda.synchronize()
    assert st.completed == len(reqs)
    alone = {}
    for m, d in models.items():
        d["net"].set_mode(P.EVAL_HOISTED)
        for i in range(5):
            ct = P.Ciphertext(d["pool"].data[i:i + 1].clone(), d["pool"].scale)
            alone[(m, i)] = [o.data[0].cpu() for o in d["net"].eval(ct)]
    for r in reqs:
        exp = alone[(r.model, r.payload)]
        assert len(r.result) == len(exp)
        for a, b in zip(r.result, exp):
            assert torch.equal(a.cpu(), b), (r.rid, r.model)
    for m, d in models.items():
        assert d["pool"].data.shape[0] == 5
    assert st.batches < len(reqs)          # some batches held several requests
