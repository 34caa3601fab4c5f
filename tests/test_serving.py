"""Continuous-batching server: scheduler behaviour on the CPU with a simulated
clock and executor (admission by HBM footprint, slots, rounds of layer stages,
joining at layer boundaries); on the GPU, every request's outputs are
bit-identical whether it is served alone or inside a mixed stream, also when
the HBM budget holds requests back."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2402_03060_amd.serve import ModelSpec, Request, Scheduler, poisson_requests, serve


class SimClock:
    """Time advances only when the loop reads it (and the fake executor works)."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-5
        return self.t


class FakeExecutor:
    """A layer stage of a group of n requests of model m takes base[m] +
    per_item[m] * n seconds of simulated time; a round runs its stages one
    after another, and rounds of different models overlap."""

    def __init__(self, clock, base, per_item):
        self.clock, self.base, self.per_item = clock, base, per_item
        self.rounds = []       # (model, start, end, [(group id, first rid, stage, size)])
        self.stage_log = {}    # rid -> stages run, in order
        self.slots_live = {}   # model -> {slot: rid} while in flight

    def run_round(self, m, new, steps):
        start = self.clock.t
        dur = sum(self.base[m] + self.per_item[m] * g.size for g, _ in steps)
        live = self.slots_live.setdefault(m, {})
        if new is not None:
            for i, r in enumerate(new.reqs):
                assert new.slot + i not in live, "slot in use by another request"
                live[new.slot + i] = r.rid
        for g, k in steps:
            for r in g.reqs:
                self.stage_log.setdefault(r.rid, []).append(k)
        self.rounds.append((m, start, start + dur, [(id(g), g.reqs[0].rid, k, g.size) for g, k in steps]))
        return start + dur

    def done(self, end):
        return self.clock.t >= end

    def collect(self, m, g):
        for i, r in enumerate(g.reqs):
            r.result = ("done", r.rid)
            assert self.slots_live[m].pop(g.slot + i) == r.rid


MODELS = {"a": ModelSpec("a", 8, 100, 4, 4), "b": ModelSpec("b", 4, 300, 3, 2), "c": ModelSpec("c", 2, 1000, 5, 1)}
BASE = {"a": 1e-4, "b": 2e-4, "c": 5e-4}
PER = {"a": 1e-5, "b": 2e-5, "c": 1e-4}


def _run(reqs, budget, models=MODELS):
    clock = SimClock()
    ex = FakeExecutor(clock, BASE, PER)
    sch = Scheduler(models, budget)
    seen = []
    orig = sch.admit

    def admit(now):
        orig(now)
        seen.append(sch.in_flight_bytes)
    sch.admit = admit
    st = serve(sch, ex, reqs, clock=clock)
    return st, ex, seen, sch


def _reqs(n=300, rate=20000.0, seed=4):
    return poisson_requests({"a": 0.5, "b": 0.3, "c": 0.2}, rate, n, seed, {"a": [0] * 3, "b": [0], "c": [0] * 2})


def test_all_requests_complete_once_through_every_layer():
    reqs = _reqs()
    st, ex, _, sch = _run(reqs, 10 ** 9)
    assert st.completed == len(reqs)
    assert all(r.result == ("done", r.rid) for r in reqs)
    for r in reqs:
        assert ex.stage_log[r.rid] == list(range(MODELS[r.model].n_stages)), r.rid
    assert sch.in_flight_bytes == 0 and sch.idle()
    assert all(sorted(sch.free[m]) == list(range(s.slots // s.group_max)) for m, s in MODELS.items())


def test_budget_never_exceeded_and_queue_used():
    reqs = _reqs(rate=50000.0)
    budget = 2500
    st, ex, seen, _ = _run(reqs, budget)
    assert max(seen) <= budget
    assert st.max_in_flight_bytes <= budget
    assert st.max_host_queue > 0            # the budget held requests back on the host
    assert st.completed == len(reqs)


def test_joining_at_layer_boundaries():
    """A request arriving while a group of its model is in flight starts at
    the next round, while that group is still running later layers, and the
    two groups' rounds interleave."""
    clock = SimClock()
    ex = FakeExecutor(clock, BASE, PER)
    reqs = [Request(0, "a", 0.0, 0), Request(1, "a", 1.5e-4, 0)]   # the second arrives during round one
    st = serve(Scheduler(MODELS, 10 ** 9), ex, reqs, clock=clock)
    assert st.completed == 2 and st.joins == 1
    assert reqs[1].started < reqs[0].finished          # did not wait for the first to finish
    rounds_a = [r for r in ex.rounds if r[0] == "a"]
    # some round advanced the first request (stage >= 1) and started the second (stage 0)
    assert any({(rid, k) for _, rid, k, _ in steps} >= {(0, k0), (1, 0)} for _, _, _, steps in rounds_a
               for k0 in range(1, 4))
    # the second needed n_stages rounds, not the first request's remaining rounds + its own
    assert reqs[1].finished - reqs[1].started < 1.5 * (reqs[0].finished - reqs[0].started)


def test_groups_fifo_bounded_and_slots_disjoint():
    reqs = _reqs(rate=50000.0)
    st, ex, _, _ = _run(reqs, 10 ** 9)
    starts = {}
    for m, _, _, steps in ex.rounds:
        for _, rid0, k, size in steps:
            if k == 0:
                assert 1 <= size <= MODELS[m].group_max
                starts.setdefault(m, []).append(rid0)
    model_of = {r.rid: r.model for r in reqs}
    for m, rids in starts.items():
        assert all(model_of[i] == m for i in rids)
        assert rids == sorted(rids)          # first come, first started within a model
    # under load the server starts full groups and keeps several in flight
    assert max(size for m, _, _, steps in ex.rounds if m == "a" for _, _, k, size in steps) == MODELS["a"].group_max
    assert max(len(steps) for m, _, _, steps in ex.rounds if m == "a") >= 2
    assert st.joins > 0


def test_one_round_per_model_in_flight_and_models_overlap():
    reqs = _reqs(rate=50000.0)
    st, ex, _, _ = _run(reqs, 10 ** 9)
    for m in MODELS:
        s = sorted((a, b) for k, a, b, _ in ex.rounds if k == m)
        assert all(s[i][1] <= s[i + 1][0] for i in range(len(s) - 1))
    spans = [(m, a, b) for m, a, b, _ in ex.rounds]
    assert any(a1 < b2 and a2 < b1 for (m1, a1, b1) in spans for (m2, a2, b2) in spans if m1 != m2)


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
    a = _reqs(n=4000, rate=2000.0, seed=4)
    b = _reqs(n=4000, rate=2000.0, seed=4)
    assert [(r.model, r.arrival) for r in a] == [(r.model, r.arrival) for r in b]
    frac = {m: sum(r.model == m for r in a) / len(a) for m in "abc"}
    assert abs(frac["a"] - 0.5) < 0.03 and abs(frac["b"] - 0.3) < 0.03 and abs(frac["c"] - 0.2) < 0.03
    gaps = np.diff([0.0] + [r.arrival for r in a])
    assert abs(gaps.mean() - 1 / 2000.0) < 0.1 / 2000.0


def _gpu_models(variant, slots=None):
    import workloads as W
    import paper_2402_03060_amd as P
    from paper_2402_03060_amd.serve import prepare_model
    shrink = {"conv1": 11, "lenet1": 12, "cnn1d": 12}
    slots = slots or {"conv1": (6, 3), "lenet1": (4, 2), "cnn1d": (4, 2)}
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
            models[name] = prepare_model(P, W, name, slots[name][0], pool_size=5, seed=40, group_max=slots[name][1],
                                         lazy=variant, fc_doubling=variant)
    finally:
        W.config = orig
    return models


def _alone(models):
    import paper_2402_03060_amd as P
    alone = {}
    for m, d in models.items():
        for i in range(5):
            ct = P.Ciphertext(d["pool"].data[i:i + 1].clone(), d["pool"].scale)
            alone[(m, i)] = [o.data[0].cpu() for o in d["net"].eval(ct)]
    return alone


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [False, True])
def test_served_outputs_equal_alone(variant):
    """Three models (ring sizes 2^11, 2^12, 2^12 here) served together from a
    Poisson stream, groups joining at layer boundaries in several slot ranges:
    each request's output ciphertexts equal those of evaluating its
    ciphertext alone (default plan, and deferred ModDown with the doubling FC
    sum, which the server runs)."""
    import torch
    from paper_2402_03060_amd.serve import GpuExecutor
    models = _gpu_models(variant)
    ex = GpuExecutor(models, keep_results=True)
    specs = {m: d["spec"] for m, d in models.items()}
    ex.warmup(specs)
    reqs = poisson_requests({"conv1": 0.5, "lenet1": 0.3, "cnn1d": 0.2}, 3000.0, 60, 4,
                            {m: list(range(5)) for m in models})
    st = serve(Scheduler(specs, 10 ** 12), ex, reqs)
    torch.cuda.synchronize()
    assert st.completed == len(reqs)
    alone = _alone(models)
    for r in reqs:
        exp = alone[(r.model, r.payload)]
        assert len(r.result) == len(exp)
        for a, b in zip(r.result, exp):
            assert torch.equal(a.cpu(), b), (r.rid, r.model)
    assert st.batches < len(reqs)          # some groups held several requests
    assert st.joins > 0                    # some groups started while others were in flight


@pytest.mark.gpu
def test_binding_hbm_budget_queues_and_matches_alone():
    """A budget of two requests' bytes: requests wait on the host, none
    fails, and every result equals the request evaluated alone."""
    import torch
    from paper_2402_03060_amd.serve import GpuExecutor
    models = _gpu_models(True)
    ex = GpuExecutor(models, keep_results=True)
    specs = {m: d["spec"] for m, d in models.items()}
    budget = 2 * max(s.slot_bytes for s in specs.values())
    reqs = poisson_requests({"conv1": 0.5, "lenet1": 0.3, "cnn1d": 0.2}, 20000.0, 40, 5,
                            {m: list(range(5)) for m in models})
    st = serve(Scheduler(specs, budget), ex, reqs)
    torch.cuda.synchronize()
    assert st.completed == len(reqs)
    assert st.max_in_flight_bytes <= budget and st.max_host_queue > 0
    alone = _alone(models)
    for r in reqs:
        for a, b in zip(r.result, alone[(r.model, r.payload)]):
            assert torch.equal(a.cpu(), b), (r.rid, r.model)


def test_full_model_does_not_block_others():
    """Model c (2 slots, slow) receives a burst; requests of model a that
    arrive behind it are admitted and finish while c's queue drains."""
    reqs = [Request(i, "c", 0.0, 0) for i in range(8)] + [Request(8 + i, "a", 1e-4, 0) for i in range(4)]
    st, ex, _, sch = _run(reqs, 10 ** 9)
    assert st.completed == len(reqs)
    last_c = max(r.finished for r in reqs if r.model == "c")
    assert all(r.finished < last_c for r in reqs if r.model == "a")
    # c never has more admitted-but-waiting requests than free slots
    assert st.max_host_queue > 0


def test_budget_is_first_come_first_served():
    """With a budget of one c request, a c request at the head is not
    overtaken by later a requests that would fit."""
    reqs = [Request(0, "c", 0.0, 0), Request(1, "c", 1e-6, 0), Request(2, "a", 2e-6, 0)]
    st, _, _, _ = _run(reqs, 1000)
    assert st.completed == 3
    assert reqs[2].admitted >= reqs[1].admitted


def test_partial_group_waits_only_while_others_are_backlogged():
    """Model a alone: a single request starts at once.  With model c's
    requests queued (a full group of c waiting), a's partial group waits up
    to max_wait_s to fill."""
    import dataclasses
    models = dict(MODELS)
    models["a"] = dataclasses.replace(MODELS["a"], max_wait_s=5e-4)
    st, _, _, _ = _run([Request(0, "a", 0.0, 0)], 10 ** 9, models)
    assert st.group_sizes["a"] == [1]
    reqs = [Request(i, "c", 0.0, 0) for i in range(6)] + [Request(6 + i, "a", 1e-4 * (i + 1), 0) for i in range(3)]
    st, _, _, _ = _run(reqs, 10 ** 9, models)
    assert st.completed == len(reqs)
    assert st.group_sizes["a"][0] >= 2          # waited for company
    for r in reqs:
        if r.model == "a":
            assert r.started - r.arrival <= 5e-4 + 1e-4


def test_partial_group_does_not_wait_for_a_short_queue():
    """Another model with less than a full group waiting is not backlogged:
    a's single request starts at once."""
    import dataclasses
    models = dict(MODELS)
    models["a"] = dataclasses.replace(MODELS["a"], max_wait_s=5e-3)
    reqs = [Request(0, "b", 0.0, 0), Request(1, "a", 0.0, 0)]      # b: group of 2, one waiting
    st, _, _, _ = _run(reqs, 10 ** 9, models)
    assert st.completed == 2
    assert reqs[1].started - reqs[1].arrival < 1e-3
