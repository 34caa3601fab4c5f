"""Continuous-batching server for encrypted inference on one GPU.

Clients send one ciphertext per request to one of several models, each with
its own ring size (the multi-model service of the paper's Fig. 1).  The server
keeps every model's evaluation keys and encoded plaintexts resident in HBM.

Batching is continuous at layer boundaries.  A model's net has a fixed number
of batch slots in blocks of its group size; a request occupies one slot from
the start of its first layer to the end of its last.  The model runs in
rounds on its own stream: a round starts a group of newly admitted requests
in a free block (their first layer) and advances every group already in
flight by one layer (unihenn_eval_stage on the group's slots, one captured
graph per layer, block and group size).  A request that arrives while
others are on the GPU therefore joins at the next layer boundary instead of
waiting for a whole batch, and the rounds of different models overlap on the
device.

Admission is by HBM footprint: a request holds its slot's share of the net's
registers and workspace plus its input and output ciphertexts
(unihenn_net_memory); requests wait in per-model host queues while the bytes
held by admitted requests would exceed the budget.  Requests are admitted
oldest first across the models that have free slots for them, so a model
whose slots are full does not hold back the others, while no request
overtakes an older one on the budget.

The scheduling logic (admission, slots, rounds, latency accounting) is
independent of the executor: `GpuExecutor` drives the C ABI, and tests drive
it with a fake executor on a simulated clock.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    model: str
    arrival: float            # seconds since the start of the run
    payload: object = None    # executor-specific input (e.g. an index into a ciphertext pool)
    admitted: float = -1.0
    started: float = -1.0
    finished: float = -1.0
    result: object = None


@dataclass
class ModelSpec:
    name: str
    slots: int                # batch slots of the model's net: requests in flight at once
    slot_bytes: int           # HBM one admitted request holds (its slot, input and outputs)
    n_stages: int = 1         # layers; a request is done after that many rounds
    group_max: int = 0        # most requests one round starts (0: all free slots)
    max_wait_s: float = 0.0   # while another model is backlogged, a partial group waits up to this


@dataclass
class Group:
    model: str
    slot: int                 # first batch slot
    reqs: list
    stage: int = 0            # next layer to run

    @property
    def size(self) -> int:
        return len(self.reqs)


@dataclass
class RunStats:
    latencies: dict = field(default_factory=dict)   # model -> list of seconds
    completed: int = 0
    duration: float = 0.0
    batches: int = 0          # groups started
    rounds: int = 0
    joins: int = 0            # groups started while another group of their model was in flight
    max_in_flight_bytes: int = 0
    max_host_queue: int = 0
    backlog_at_last_arrival: int = 0   # requests arrived but not finished when the last one arrived
    group_sizes: dict = field(default_factory=dict)   # model -> sizes of the groups started

    def summary(self) -> dict:
        allv = np.array([v for vs in self.latencies.values() for v in vs]) if self.completed else np.zeros(1)
        out = {"completed": self.completed, "seconds": round(self.duration, 3),
               "throughput_per_s": round(self.completed / max(self.duration, 1e-9), 2),
               "p50_ms": round(1e3 * float(np.percentile(allv, 50)), 3),
               "p99_ms": round(1e3 * float(np.percentile(allv, 99)), 3),
               "groups": self.batches, "rounds": self.rounds, "joins": self.joins,
               "max_host_queue": self.max_host_queue, "max_in_flight_bytes": self.max_in_flight_bytes,
               "backlog_at_last_arrival": self.backlog_at_last_arrival,
               "per_model": {}}
        for m, vs in self.latencies.items():
            a = np.array(vs)
            out["per_model"][m] = {"n": len(vs), "p50_ms": round(1e3 * float(np.percentile(a, 50)), 3),
                                   "p99_ms": round(1e3 * float(np.percentile(a, 99)), 3),
                                   "mean_group": round(float(np.mean(self.group_sizes.get(m, [0]))), 2)}
        return out


class Scheduler:
    """Admission by HBM footprint and per-model rounds of layer stages."""

    def __init__(self, models: dict, hbm_budget_bytes: int):
        self.models = models
        self.budget = int(hbm_budget_bytes)
        self.in_flight_bytes = 0
        self.host = {m: collections.deque() for m in models}                # not yet admitted, per model
        self.ready = {m: collections.deque() for m in models}               # admitted, not yet started
        self.groups = {m: [] for m in models}                               # in flight
        # slots come in aligned blocks of group_max (a group takes one block),
        # so each (layer, block, size) is one captured graph
        self.free = {m: list(range(s.slots // self._block(m))) for m, s in models.items()}
        self.busy = {m: None for m in models}                               # the executor's round handle

    def _block(self, m: str) -> int:
        s = self.models[m]
        return s.group_max if 0 < s.group_max <= s.slots else s.slots

    def arrive(self, req: Request):
        self.host[req.model].append(req)

    def queued(self) -> int:
        """Requests waiting on the host (not yet admitted)."""
        return sum(len(q) for q in self.host.values())

    def _room(self, m: str) -> bool:
        # admitted requests never outnumber the slots they can start in
        return len(self.ready[m]) < len(self.free[m]) * self._block(m)

    def admit(self, now: float):
        """Admit waiting requests oldest first across the models that have
        free slots for them, while the bytes they hold fit the budget.  A
        model whose slots are full does not hold back the others; a request
        that does not fit the budget does (no overtaking on the budget)."""
        while True:
            heads = [(q[0].arrival, q[0].rid, m) for m, q in self.host.items() if q and self._room(m)]
            if not heads:
                return
            m = min(heads)[2]
            req = self.host[m][0]
            fb = self.models[m].slot_bytes
            if self.in_flight_bytes + fb > self.budget:
                if self.in_flight_bytes == 0 and fb > self.budget:
                    raise RuntimeError(f"one {m} request needs {fb} bytes, above the budget {self.budget}")
                return
            self.host[m].popleft()
            self.in_flight_bytes += fb
            req.admitted = now
            self.ready[m].append(req)

    def _take_slots(self, m: str, want: int):
        """The first slot and count (at most want, at most a block) of the
        lowest free block; (0, 0) when every block is in use."""
        if not self.free[m]:
            return 0, 0
        blk = min(self.free[m])
        self.free[m].remove(blk)
        g = self._block(m)
        return blk * g, min(want, g)

    def _release_slots(self, m: str, a: int, k: int):
        self.free[m].append(a // self._block(m))

    def _backlogged(self, m: str) -> bool:
        """Model m has at least a full group of requests waiting."""
        return len(self.host[m]) + len(self.ready[m]) >= self._block(m)

    def _start_now(self, m: str, now: float) -> bool:
        """Start a group of m's admitted requests now: when it would be full,
        when its oldest request has waited max_wait_s, or when no other model
        is backlogged (nothing to give the GPU time to).  Fuller groups cost
        less GPU time per request, which goes to the backlogged models."""
        spec = self.models[m]
        if len(self.ready[m]) >= self._block(m) or now - self.ready[m][0].arrival >= spec.max_wait_s:
            return True
        return not any(self._backlogged(x) for x in self.models if x != m)

    def plan_round(self, m: str, now: float):
        """The next round of model m: a new group of its admitted requests
        (first come, first served, in one free slot range), then one layer of
        every group in flight, oldest first.  Returns (new group or None,
        [(group, stage)])."""
        spec = self.models[m]
        new = None
        if self.ready[m] and self._start_now(m, now):
            slot, k = self._take_slots(m, len(self.ready[m]))
            if k:
                new = Group(m, slot, [self.ready[m].popleft() for _ in range(k)])
                for r in new.reqs:
                    r.started = now
                self.groups[m].append(new)
        steps = [(g, g.stage) for g in self.groups[m]]
        for g in self.groups[m]:
            g.stage += 1
        return new, steps

    def finish_round(self, m: str, now: float) -> list:
        """Groups of model m whose last layer ran in the round that ended:
        their slots and bytes are released.  Returns those groups."""
        spec = self.models[m]
        done = [g for g in self.groups[m] if g.stage >= spec.n_stages]
        self.groups[m] = [g for g in self.groups[m] if g.stage < spec.n_stages]
        for g in done:
            self._release_slots(m, g.slot, g.size)
            for r in g.reqs:
                r.finished = now
                self.in_flight_bytes -= spec.slot_bytes
        return done

    def idle(self) -> bool:
        return not self.queued() and all(not q for q in self.ready.values()) and \
            all(not g for g in self.groups.values()) and all(v is None for v in self.busy.values())


def serve(scheduler: Scheduler, executor, requests: list, clock=time.perf_counter, poll_s: float = 0.0) -> RunStats:
    """Run `requests` (sorted by arrival time, seconds from start) through the
    scheduler and executor in real time; returns per-request latencies."""
    stats = RunStats()
    t0 = clock()
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    while pending or not scheduler.idle():
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            scheduler.arrive(pending.popleft())
            if not pending:
                stats.backlog_at_last_arrival = len(requests) - stats.completed
        stats.max_host_queue = max(stats.max_host_queue, scheduler.queued())
        for m in scheduler.models:
            h = scheduler.busy[m]
            if h is not None:
                if not executor.done(h):
                    continue
                scheduler.busy[m] = None
                for g in scheduler.finish_round(m, clock() - t0):
                    executor.collect(m, g)
                    for r in g.reqs:
                        stats.latencies.setdefault(m, []).append(r.finished - r.arrival)
                        stats.completed += 1
        scheduler.admit(clock() - t0)
        stats.max_in_flight_bytes = max(stats.max_in_flight_bytes, scheduler.in_flight_bytes)
        for m in scheduler.models:
            if scheduler.busy[m] is not None:
                continue
            in_flight = len(scheduler.groups[m])
            new, steps = scheduler.plan_round(m, clock() - t0)
            if not steps:
                continue
            if new is not None:
                stats.batches += 1
                stats.joins += in_flight > 0
                stats.group_sizes.setdefault(m, []).append(new.size)
            stats.rounds += 1
            scheduler.busy[m] = executor.run_round(m, new, steps)
        if poll_s:
            time.sleep(poll_s)
    stats.duration = clock() - t0
    return stats


def poisson_requests(mix: dict, rate_per_s: float, n: int, seed: int, payloads: dict) -> list:
    """n requests with exponential inter-arrival gaps; model drawn from `mix`
    (name -> probability); payload i of a model cycles through payloads[model]."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
    names = list(mix)
    probs = np.array([mix[m] for m in names], dtype=np.float64)
    choice = rng.choice(len(names), size=n, p=probs / probs.sum())
    count = collections.Counter()
    out = []
    for i in range(n):
        m = names[choice[i]]
        out.append(Request(i, m, float(t[i]), payload=count[m] % len(payloads[m])))
        count[m] += 1
    return out


class GpuExecutor:
    """Runs rounds through the C ABI: per model one net (its batch slots),
    stream, input staging buffer and output buffers, all slot-indexed.  A
    round copies a new group's ciphertexts into their staging slots, runs one
    layer stage per group in flight (unihenn_eval_stage) and records an event
    on the model's stream."""

    def __init__(self, models: dict, keep_results: bool = False):
        import torch
        self.torch = torch
        self.m = models          # name -> dict(net, ctx, pool (ciphertext batch tensor), ...)
        self.keep_results = keep_results
        self.batch_time = {}     # name -> seconds for a full group through every layer (warmup)
        for name, d in models.items():
            ctx, net = d["ctx"], d["net"]
            pool = d["pool"]      # Ciphertext [P][2][nl][N]
            d["stream"] = torch.cuda.Stream()
            d["staging"] = ctx.empty_ct(net.max_batch, pool.n_limbs, pool.scale)
            d["outs"] = net.alloc_outputs(net.max_batch)
            d["n_stages"] = net.stages()

    def run_round(self, model: str, new, steps):
        import paper_2402_03060_amd as P
        torch = self.torch
        d = self.m[model]
        st = d["stream"]
        ns = d["n_stages"]
        with torch.cuda.stream(st):
            if new is not None:
                # row copies on the model's stream into buffers that live as
                # long as the executor (no temporary device tensors)
                for i, r in enumerate(new.reqs):
                    d["staging"].data[new.slot + i].copy_(d["pool"].data[r.payload])
            for g, k in steps:
                a, n = g.slot, g.size
                ct = P.Ciphertext(d["staging"].data[a:a + n], d["pool"].scale) if k == 0 else None
                outs = [P.Ciphertext(o.data[a:a + n], 0.0) for o in d["outs"]] if k == ns - 1 else None
                d["net"].eval_stage(k, a, n, ct=ct, outs=outs, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def warmup(self, specs: dict):
        """Every group a scheduler over `specs` can form (each block, each
        size) through every layer, so that the graphs are captured before
        requests are timed."""
        for m, d in self.m.items():
            spec = specs[m]
            blk = spec.group_max if 0 < spec.group_max <= spec.slots else spec.slots
            for a in range(0, spec.slots - blk + 1, blk):
                for b in range(1, blk + 1):
                    g = Group(m, a, [Request(-1, m, 0.0, payload=i % d["pool"].batch) for i in range(b)])
                    for k in range(d["n_stages"]):
                        self.run_round(m, g if k == 0 else None, [(g, k)]).synchronize()
            # batch time: a full group through every layer (replays), median of 3
            g = Group(m, 0, [Request(-1, m, 0.0, payload=i % d["pool"].batch) for i in range(blk)])
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                for k in range(d["n_stages"]):
                    self.run_round(m, g if k == 0 else None, [(g, k)]).synchronize()
                ts.append(time.perf_counter() - t0)
            self.batch_time[m] = sorted(ts)[1]

    def done(self, handle) -> bool:
        return handle.query()

    def collect(self, model: str, group):
        if not self.keep_results:
            return
        d = self.m[model]
        with self.torch.cuda.stream(d["stream"]):
            for i, r in enumerate(group.reqs):
                r.result = [o.data[group.slot + i].clone() for o in d["outs"]]
        d["stream"].synchronize()


def prepare_model(P, W, name: str, slots: int, pool_size: int, seed: int = 5, group_max: int = 0,
                  lazy: bool = False, fc_doubling: bool = False, tuning_cache: str | None = None) -> dict:
    """Context, net with `slots` batch slots (hoisted, graph replay of each
    layer stage; lazy / fc_doubling select the plan variants), product-client
    keys and a pool of encrypted synthetic
    inputs for one workload, and its ModelSpec (bytes per request from the
    net's per-slot memory plus the input and output ciphertexts).  With
    tuning_cache, launch parameters tuned on whole evaluations of a full
    group (looked up in or recorded to that file) apply to the stages too."""
    import torch
    cfg = W.config(name)
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    params = W.gen_params(cfg["layers"])
    S, stride = cfg["samples_per_ct"], cfg["sample_stride"]
    net = P.Net(ctx, cfg["input"], cfg["layers"], params, samples=S, stride=stride, max_batch=slots,
                lazy=lazy, fc_doubling=fc_doubling)
    sk = P.keygen_secret(ctx, seed)
    keys = {r: P.gen_switch_key(ctx, sk, seed + 1, steps=r) for r in net.rotations()}
    rlk = P.gen_switch_key(ctx, sk, seed + 2, relin=True)
    net.bind_keys(keys, rlk)
    net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
    if tuning_cache:
        net.autotune(group_max if group_max > 0 else slots, cache_path=tuning_cache)
    xs = W.gen_inputs(cfg["input"], S * pool_size)
    st = stride if S > 1 else ctx.slots
    pts = []
    for b in range(pool_size):
        v = np.zeros(ctx.slots)
        for j in range(S):
            flat = xs[b * S + j].reshape(-1)
            v[j * st: j * st + flat.size] = flat
        pts.append(ctx.encode(v, ctx.scale, net.in_limbs, mont=False))
    pool = P.encrypt_sk(ctx, sk, torch.stack(pts), seed + 3, ctx.scale)
    torch.cuda.synchronize()
    _, per_slot = net.memory()
    ct_bytes = 2 * net.in_limbs * ctx.n * 8
    out_bytes = net.n_out * 2 * ctx.n * 8
    spec = ModelSpec(name, slots, per_slot + ct_bytes + out_bytes, net.stages(), group_max)
    return {"ctx": ctx, "net": net, "sk": sk, "keys": keys, "rlk": rlk, "pool": pool, "xs": xs, "cfg": cfg,
            "params": params, "spec": spec}


# ---------------------------------------------------------------- measurement
# model -> (batch slots, most requests one round starts)
SERVE_MODELS = {"conv1": (32, 16), "cnn1d": (16, 8), "cifar_cnn": (8, 4)}
SERVE_MIX = {"conv1": 0.5, "cnn1d": 0.3, "cifar_cnn": 0.2}


def serving_benchmark(P, W, n_requests: int, tuning_cache: str | None = None, hbm_budget: int | None = None,
                      levels=(0.5, 0.8, 0.9, 1.0), log=print, lazy: bool = True, fc_doubling: bool = True,
                      wait_batches: float = 3.0, slots: dict | None = None) -> dict:
    """Three models of different ring sizes behind the server: saturation
    throughput (a burst of requests queued at t = 0), then Poisson arrivals
    (seed 4, mix 50/30/20) at the given fractions of it.  The admission budget
    defaults to the bytes of every model's slots (the memory reserved for
    requests).  The models run the deferred-ModDown plan with the doubling FC
    sum unless lazy / fc_doubling say otherwise.  While another model has a
    full group waiting, a partial group waits up to wait_batches of its
    model's batch time (a full group through every layer), and at least half
    the longest model's batch time, to fill."""
    import torch
    plan = " + ".join([n for n, on in (("deferred ModDown", lazy), ("doubling FC sum", fc_doubling)) if on]) \
        or "default"
    slots = dict(SERVE_MODELS, **(slots or {}))
    log("setup serving models " + ", ".join(f"{m} ({s} slots, groups of {g})" for m, (s, g) in slots.items()) +
        f" ({plan} plan)")
    models = {m: prepare_model(P, W, m, s, pool_size=16, group_max=g, lazy=lazy, fc_doubling=fc_doubling,
                               tuning_cache=tuning_cache) for m, (s, g) in slots.items()}
    ex = GpuExecutor(models)
    specs = {m: d["spec"] for m, d in models.items()}
    ex.warmup(specs)
    # a model with short batches may wait at least half the longest batch
    # time: its latency stays far below the slow models' while its fuller
    # groups free GPU time for them
    floor_s = 0.5 * max(ex.batch_time.values())
    for m, spec in specs.items():
        spec.max_wait_s = max(wait_batches * ex.batch_time[m], floor_s)
    log("warmed up: a graph per layer, block and group size captured; batch times " +
        ", ".join(f"{m} {1e3 * t:.2f} ms" for m, t in ex.batch_time.items()))
    if hbm_budget is None:
        hbm_budget = sum(s.slots * s.slot_bytes for s in specs.values())
    payloads = {m: list(range(16)) for m in models}
    out = {"models": {m: {"log_n": d["cfg"]["log_n"], "slots": d["spec"].slots, "group_max": d["spec"].group_max,
                          "layers": d["spec"].n_stages, "ciphertexts_per_request": 1,
                          "samples_per_ct": d["cfg"]["samples_per_ct"], "request_bytes": d["spec"].slot_bytes}
                      for m, d in models.items()},
           "plan": plan, "batching": "continuous at layer boundaries", "mix": SERVE_MIX,
           "arrival_seed": W.SEED_ARRIVALS, "hbm_budget_bytes": hbm_budget, "requests_per_level": n_requests,
           "batch_time_ms": {m: round(1e3 * t, 3) for m, t in ex.batch_time.items()},
           "max_wait_batches": wait_batches,
           "max_wait_ms": {m: round(1e3 * sp.max_wait_s, 3) for m, sp in specs.items()}}
    burst = poisson_requests(SERVE_MIX, 1e9, min(n_requests, 3000), W.SEED_ARRIVALS, payloads)
    st = serve(Scheduler(specs, hbm_budget), ex, burst)
    torch.cuda.synchronize()
    sat = st.completed / st.duration
    out["saturation_requests_per_s"] = round(sat, 2)
    log(f"serving saturation {sat:.1f} req/s")
    res = {}
    for frac in levels:
        reqs = poisson_requests(SERVE_MIX, frac * sat, n_requests, W.SEED_ARRIVALS, payloads)
        st = serve(Scheduler(specs, hbm_budget), ex, reqs)
        torch.cuda.synchronize()
        summ = st.summary()
        summ["offered_requests_per_s"] = round(frac * sat, 2)
        res[str(frac)] = summ
        log(f"serving at {frac:.1f}x: {summ['throughput_per_s']} req/s, p50 {summ['p50_ms']} ms, "
            f"p99 {summ['p99_ms']} ms, {summ['joins']} joins")
    out["load_levels"] = res
    del ex, models
    torch.cuda.empty_cache()
    return out


def main():
    import argparse
    import json
    import os
    import sys
    ap = argparse.ArgumentParser(description="serving measurement: saturation, then Poisson load levels")
    ap.add_argument("--requests", type=int, default=10000, help="requests per load level")
    ap.add_argument("--levels", default="0.5,0.8,0.9,1.0")
    ap.add_argument("--wait-batches", type=float, default=3.0,
                    help="longest wait of a partial group, in batch times, while another model is backlogged")
    ap.add_argument("--slots", default="", help="per model slots:group, e.g. cifar_cnn=16:8,conv1=32:16")
    ap.add_argument("--default-plan", action="store_true",
                    help="the default plan instead of deferred ModDown + doubling FC sum")
    ap.add_argument("--tuning-cache", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                           "tuning_cache.json"))
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_2402_03060_amd as P
    import workloads as W
    out = serving_benchmark(P, W, a.requests, tuning_cache=a.tuning_cache,
                            levels=tuple(float(x) for x in a.levels.split(",")),
                            lazy=not a.default_plan, fc_doubling=not a.default_plan, wait_batches=a.wait_batches,
                            slots={k: tuple(int(x) for x in v.split(":")) for k, v in
                                   (kv.split("=") for kv in a.slots.split(",") if kv)},
                            log=lambda m: print("[serve] " + m, file=sys.stderr, flush=True))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
