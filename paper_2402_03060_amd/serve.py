"""Continuous-batching server for encrypted inference on one GPU.

Clients send one ciphertext per request to one of several models, each with
its own ring size (the multi-model service of the paper's Fig. 1).  The server
keeps every model's evaluation keys and encoded plaintexts resident in HBM.
It admits requests into device memory while their ciphertext footprint fits
an HBM budget; requests past the budget wait in a host-side queue.  As soon
as a model's previous batch finishes, it forms the next batch from that
model's admitted requests (up to the model's batch size).  Batches of
different models run concurrently on their own streams, so requests that
arrive while others are on the GPU join the next free batch and their work
overlaps on the device.

The scheduling logic (admission, per-model FIFO batching, latency
accounting) is independent of the executor: `GpuExecutor` drives the C ABI,
and tests can drive it with a fake executor on the CPU.
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
    max_batch: int
    footprint_bytes: int      # HBM bytes one admitted request holds (input ciphertext + outputs)


@dataclass
class RunStats:
    latencies: dict = field(default_factory=dict)   # model -> list of seconds
    completed: int = 0
    duration: float = 0.0
    batches: int = 0
    max_in_flight_bytes: int = 0
    max_host_queue: int = 0

    def summary(self) -> dict:
        allv = np.array([v for vs in self.latencies.values() for v in vs]) if self.completed else np.zeros(1)
        out = {"completed": self.completed, "seconds": round(self.duration, 3),
               "throughput_per_s": round(self.completed / max(self.duration, 1e-9), 2),
               "p50_ms": round(1e3 * float(np.percentile(allv, 50)), 3),
               "p99_ms": round(1e3 * float(np.percentile(allv, 99)), 3),
               "batches": self.batches, "max_host_queue": self.max_host_queue,
               "per_model": {}}
        for m, vs in self.latencies.items():
            a = np.array(vs)
            out["per_model"][m] = {"n": len(vs), "p50_ms": round(1e3 * float(np.percentile(a, 50)), 3),
                                   "p99_ms": round(1e3 * float(np.percentile(a, 99)), 3)}
        return out


class Scheduler:
    """Admission by HBM budget and per-model continuous batching."""

    def __init__(self, models: dict, hbm_budget_bytes: int):
        self.models = models
        self.budget = int(hbm_budget_bytes)
        self.in_flight_bytes = 0
        self.host_queue: collections.deque = collections.deque()            # not yet admitted
        self.ready = {m: collections.deque() for m in models}               # admitted, waiting for a batch
        self.running = {m: None for m in models}                            # (handle, [requests])

    def arrive(self, req: Request):
        self.host_queue.append(req)

    def admit(self, now: float):
        """Move requests from the host queue into device queues, oldest
        first, while their footprint fits the budget."""
        while self.host_queue:
            req = self.host_queue[0]
            fb = self.models[req.model].footprint_bytes
            if self.in_flight_bytes + fb > self.budget:
                if self.in_flight_bytes == 0 and fb > self.budget:
                    raise RuntimeError(f"one {req.model} request needs {fb} bytes, above the budget {self.budget}")
                break
            self.host_queue.popleft()
            self.in_flight_bytes += fb
            req.admitted = now
            self.ready[req.model].append(req)

    def next_batches(self):
        """For every idle model with admitted requests: the next batch (FIFO)."""
        out = []
        for m, q in self.ready.items():
            if self.running[m] is None and q:
                n = min(len(q), self.models[m].max_batch)
                out.append((m, [q.popleft() for _ in range(n)]))
        return out

    def finish(self, model: str, now: float):
        _, reqs = self.running[model]
        self.running[model] = None
        for r in reqs:
            r.finished = now
            self.in_flight_bytes -= self.models[model].footprint_bytes
        return reqs

    def idle(self) -> bool:
        return not self.host_queue and all(not q for q in self.ready.values()) and \
            all(v is None for v in self.running.values())


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
        stats.max_host_queue = max(stats.max_host_queue, len(scheduler.host_queue))
        scheduler.admit(now)
        stats.max_in_flight_bytes = max(stats.max_in_flight_bytes, scheduler.in_flight_bytes)
        for m, reqs in scheduler.next_batches():
            for r in reqs:
                r.started = now
            scheduler.running[m] = (executor.launch(m, reqs), reqs)
            stats.batches += 1
        for m, run in list(scheduler.running.items()):
            if run is not None and executor.done(run[0]):
                executor.collect(run[0], run[1])
                for r in scheduler.finish(m, clock() - t0):
                    stats.latencies.setdefault(m, []).append(r.finished - r.arrival)
                    stats.completed += 1
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
    """Runs batches through the C ABI: one net, stream, staging buffer and
    output buffers per model; each batch is gathered into the staging
    buffer, evaluated (a replayed HIP graph per batch size) and marked with
    an event on the model's stream."""

    def __init__(self, models: dict, keep_results: bool = False):
        import torch
        self.torch = torch
        self.m = models          # name -> dict(net, ctx, pool (ciphertext batch tensor), stream, ...)
        self.keep_results = keep_results
        for name, d in models.items():
            ctx, net = d["ctx"], d["net"]
            pool = d["pool"]      # Ciphertext [P][2][nl][N]
            d["stream"] = torch.cuda.Stream()
            d["staging"] = ctx.empty_ct(net.max_batch, pool.n_limbs, pool.scale)
            d["outs"] = net.alloc_outputs(net.max_batch)

    def launch(self, model: str, reqs: list):
        import paper_2402_03060_amd as P
        torch = self.torch
        d = self.m[model]
        b = len(reqs)
        st = d["stream"]
        with torch.cuda.stream(st):
            # Row copies on the model's stream into a buffer that lives as
            # long as the executor.  No temporary device tensor is made here:
            # one allocated on another stream and dropped before this stream
            # has read it could be handed to a new allocation and overwritten.
            for i, r in enumerate(reqs):
                d["staging"].data[i].copy_(d["pool"].data[r.payload])
            inp = P.Ciphertext(d["staging"].data[:b], d["pool"].scale)
            outs = [P.Ciphertext(o.data[:b], 0.0) for o in d["outs"]]
            d["net"].eval(inp, outs, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (model, b, ev, outs)

    def warmup(self):
        """Evaluate every batch size of every model once, so that the graphs
        are captured before requests are timed."""
        for m, d in self.m.items():
            for b in range(1, d["net"].max_batch + 1):
                reqs = [Request(-1, m, 0.0, payload=i % d["pool"].batch) for i in range(b)]
                d["stream"].synchronize()
                self.launch(m, reqs)[2].synchronize()

    def done(self, handle) -> bool:
        return handle[2].query()

    def collect(self, handle, reqs):
        if not self.keep_results:
            return
        _, b, ev, outs = handle
        ev.synchronize()
        for i, r in enumerate(reqs):
            r.result = [o.data[i].clone() for o in outs]


def prepare_model(P, W, name: str, max_batch: int, pool_size: int, seed: int = 5,
                  tuning_cache: str | None = None, lazy: bool = False, fc_doubling: bool = False) -> dict:
    """Context, net (hoisted, graph replay; lazy / fc_doubling select the plan
    variants), product-client keys and a pool of encrypted synthetic inputs
    for one workload; with tuning_cache, launch parameters tuned for full
    batches (looked up in or recorded to that file)."""
    import torch
    cfg = W.config(name)
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    params = W.gen_params(cfg["layers"])
    S, stride = cfg["samples_per_ct"], cfg["sample_stride"]
    net = P.Net(ctx, cfg["input"], cfg["layers"], params, samples=S, stride=stride, max_batch=max_batch,
                lazy=lazy, fc_doubling=fc_doubling)
    sk = P.keygen_secret(ctx, seed)
    keys = {r: P.gen_switch_key(ctx, sk, seed + 1, steps=r) for r in net.rotations()}
    rlk = P.gen_switch_key(ctx, sk, seed + 2, relin=True)
    net.bind_keys(keys, rlk)
    net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
    if tuning_cache:
        net.autotune(max_batch, cache_path=tuning_cache)
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
    ct_bytes = 2 * net.in_limbs * ctx.n * 8
    out_bytes = net.n_out * 2 * ctx.n * 8
    return {"ctx": ctx, "net": net, "sk": sk, "keys": keys, "rlk": rlk, "pool": pool, "xs": xs, "cfg": cfg,
            "params": params, "spec": ModelSpec(name, max_batch, ct_bytes + out_bytes)}


# ---------------------------------------------------------------- measurement
SERVE_MODELS = {"conv1": 16, "cnn1d": 8, "cifar_cnn": 4}     # model -> largest batch (ciphertexts)
SERVE_MIX = {"conv1": 0.5, "cnn1d": 0.3, "cifar_cnn": 0.2}


def serving_benchmark(P, W, n_requests: int, tuning_cache: str | None = None, hbm_budget: int | None = None,
                      levels=(0.5, 0.8, 1.0), log=print, lazy: bool = True, fc_doubling: bool = True) -> dict:
    """Three models of different ring sizes behind the server: saturation
    throughput (all requests queued at t = 0), then Poisson arrivals (seed 4,
    mix 50/30/20) at the given fractions of it.  The admission budget
    defaults to 90% of the HBM left free once the models are resident.  The
    models run the deferred-ModDown plan with the doubling FC sum unless
    lazy / fc_doubling say otherwise."""
    import torch
    plan = " + ".join([n for n, on in (("deferred ModDown", lazy), ("doubling FC sum", fc_doubling)) if on]) \
        or "default"
    log("setup serving models " + ", ".join(SERVE_MODELS) + f" ({plan} plan)")
    models = {m: prepare_model(P, W, m, b, pool_size=16, tuning_cache=tuning_cache, lazy=lazy, fc_doubling=fc_doubling)
              for m, b in SERVE_MODELS.items()}
    ex = GpuExecutor(models)
    ex.warmup()
    if hbm_budget is None:
        free, _ = torch.cuda.mem_get_info()
        hbm_budget = int(0.9 * free)
    specs = {m: d["spec"] for m, d in models.items()}
    payloads = {m: list(range(16)) for m in models}
    out = {"models": {m: {"log_n": d["cfg"]["log_n"], "max_batch": SERVE_MODELS[m], "ciphertexts_per_request": 1,
                          "samples_per_ct": d["cfg"]["samples_per_ct"], "request_bytes": d["spec"].footprint_bytes}
                      for m, d in models.items()},
           "plan": plan, "mix": SERVE_MIX, "arrival_seed": W.SEED_ARRIVALS, "hbm_budget_bytes": hbm_budget,
           "requests_per_level": n_requests}
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
            f"p99 {summ['p99_ms']} ms")
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
    ap.add_argument("--levels", default="0.5,0.8,1.0")
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
                            lazy=not a.default_plan, fc_doubling=not a.default_plan,
                            log=lambda m: print("[serve] " + m, file=sys.stderr, flush=True))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
