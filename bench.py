"""Benchmark: encrypted LeNet-1-shape inference on one MI355X.

Headline (`value`): plain LeNet-1 (Table M2 shape) encrypted inferences per
second at N = 2^14 with the 60 + 7 x 40-bit chain and a 60-bit special
prime, scale 2^40, one image per ciphertext, one key switch per rotation,
evaluated layer by layer (the paper's method as written).  A step is one
whole encrypted inference; its input ciphertext and the evaluation keys are
resident in HBM before the timer starts.

The last stdout line is one compact JSON object (see `headline`):
  batched   - the batched evaluator (ten 28 x 28 images per ciphertext at
              stride 784, 128 ciphertexts per launch, hoisted rotations, one
              HIP graph): images/s, launch-time distribution and its multiple
              of the plain rate; the same for the 1D CNN (8 sequences x 64);
  rotations - rotations/s of one rotation at the same size, and a sweep over
              ring sizes (single, 24 hoisted, 128 ciphertexts per launch);
  serving   - the three-model server under Poisson load: p50/p99 latency;
  roofline  - the dominant kernel, timed with HIP events on its launch stream
              over a replay of the timed steps, on its algorithmic bytes;
  cpu_baseline - the CPU oracle (scalar C, one thread per process) on the
              host's cores.
The full result (kernel-family tables, tuning, plan variants) goes to the
file named by --detail, whose path is printed on stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def _pack(net_input: dict, xs: np.ndarray, n_slots: int, stride: int) -> np.ndarray:
    """Client-side packing: sample b's channel c, row y at slot
    b * stride + lead + (c H + y) pitch (row-major (C, H, W) without padding
    space)."""
    H, Wd = net_input["h"], net_input["w"]
    pitch, lead = net_input.get("pitch", Wd), net_input.get("lead", 0)
    v = np.zeros(n_slots)
    for b, x in enumerate(xs):
        a = np.asarray(x, dtype=np.float64).reshape(-1, H, Wd)
        for c in range(a.shape[0]):
            for y in range(H):
                base = b * stride + lead + (c * H + y) * pitch
                v[base: base + Wd] = a[c, y]
    return v


TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2402_03060_amd", "tuning_cache.json")


def setup(P, W, name: str, batch: int, seed: int = 5, tune: bool = True, mode: int = 0, log_n: int | None = None,
          lazy: bool = False, fc_doubling: bool = False, channel_cts: bool = False):
    import torch
    cfg = W.config(name)
    if log_n is not None:
        cfg["log_n"] = log_n
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    params = W.gen_params(cfg["layers"])
    S, stride = cfg["samples_per_ct"], cfg["sample_stride"]
    net = P.Net(ctx, cfg["input"], cfg["layers"], params, samples=S, stride=stride, max_batch=batch, lazy=lazy,
                fc_doubling=fc_doubling, channel_cts=channel_cts)
    sk = P.keygen_secret(ctx, seed)
    keys = {r: P.gen_switch_key(ctx, sk, seed + 1, steps=r) for r in net.rotations()}
    rlk = P.gen_switch_key(ctx, sk, seed + 2, relin=True)
    net.bind_keys(keys, rlk)
    xs = W.gen_inputs(cfg["input"], S * batch)
    st = stride if S > 1 else ctx.slots
    if channel_cts:
        # one ciphertext batch per channel: channel c's planes of the samples
        ct = []
        for c in range(cfg["input"]["c"]):
            pts = [ctx.encode(_pack(cfg["input"], xs[b * S:(b + 1) * S, c], ctx.slots, st), ctx.scale,
                              net.in_limbs, mont=False) for b in range(batch)]
            ct.append(P.encrypt_sk(ctx, sk, torch.stack(pts), seed + 3 + c, ctx.scale))
    else:
        pts = [ctx.encode(_pack(cfg["input"], xs[b * S:(b + 1) * S], ctx.slots, st), ctx.scale, net.in_limbs,
                          mont=False) for b in range(batch)]
        ct = P.encrypt_sk(ctx, sk, torch.stack(pts), seed + 3, ctx.scale)
    torch.cuda.synchronize()
    net.set_mode(mode)
    tuning = net.autotune(batch, cache_path=TUNING_CACHE) if tune else net.tuning()
    return {"cfg": cfg, "ctx": ctx, "net": net, "sk": sk, "keys": keys, "rlk": rlk, "ct": ct, "xs": xs,
            "params": params, "outs": net.alloc_outputs(batch), "tuning": tuning}


def max_error(P, W, st) -> float:
    """Decrypt every sample's outputs and compare with a direct FP64 CNN."""
    cfg, ctx, net = st["cfg"], st["ctx"], st["net"]
    S = cfg["samples_per_ct"]
    B = (st["ct"][0] if isinstance(st["ct"], list) else st["ct"]).batch
    pos = net.output_slots()                     # [S][values]: (ciphertext << 32) | slot
    ids = pos >> np.uint64(32)
    slots = (pos & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    got = np.zeros((B,) + pos.shape)
    for k in np.unique(ids):
        sel = ids == k
        vals = P.decrypt_slots(ctx, st["sk"], st["outs"][int(k)], slots[sel])
        for b in range(B):
            got[b][sel] = vals[b]
    err = 0.0
    for b in range(B):
        for s in range(S):
            ref = _fp64_cnn(st["xs"][b * S + s], cfg["layers"], st["params"])
            err = max(err, float(np.abs(got[b, s] - ref).max()))
    return err


def _fp64_cnn(x, layers, params):
    """Direct FP64 forward pass (valid convolutions, mean pooling)."""
    a = np.asarray(x, dtype=np.float64)
    for L, p in zip(layers, params):
        k = L["kind"]
        if k == "conv":
            w, b = p
            kh, kw = w.shape[2], w.shape[3]
            sh = 1 if L.get("dims") == 1 else L["s"]
            sw = L["s"]
            pw = L.get("pad", 0)
            a = np.pad(a, ((0, 0), (0 if L.get("dims") == 1 else pw,) * 2, (pw, pw)))
            C, H, Wd = a.shape
            Ho, Wo = (H - kh) // sh + 1, (Wd - kw) // sw + 1
            out = np.zeros((w.shape[0], Ho, Wo))
            for y in range(Ho):
                for xx in range(Wo):
                    patch = a[:, sh * y:sh * y + kh, sw * xx:sw * xx + kw]
                    out[:, y, xx] = np.tensordot(w, patch, axes=3) + b
            a = out
        elif k == "square":
            a = a * a
        elif k == "relu_approx":
            ca, cb, cc = L.get("coeffs", (0.375373, 0.5, 0.117071))
            a = ca + cb * a + cc * a * a
        elif k == "avgpool":
            c = L["c"]
            C, H, Wd = a.shape
            a = a[:, :H // c * c, :Wd // c * c].reshape(C, H // c, c, Wd // c, c).mean(axis=(2, 4))
        elif k == "flatten":
            a = a.reshape(-1)
        elif k == "fc":
            w, b = p
            a = w @ a.reshape(-1) + b
    return a.reshape(-1)


def timed(fn, steps: int, warmup: int) -> float:
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def family_stats(P, fn, steps: int) -> dict:
    import torch
    torch.cuda.synchronize()
    P.stats_enable(True)
    P.stats_reset()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    s = P.stats()
    P.stats_enable(False)
    return s


# Peak 64-bit modular butterflies per second, from the chip's unit counts:
# the fp32 vector peak (157.3 TFLOP/s = 256 CUs x 2.4 GHz x 128 lanes x 2)
# gives 128 full-rate VALU lane-operations per clock per CU, 7.86e13/s.
# v_mul_lo_u32 / v_mul_hi_u32 issue at 1/4 of that and v_mad_u64_u32 at 1/2
# (integer rate microbenchmark).  One butterfly on 64-bit words is one Shoup
# product (6 v_mad_u64_u32 + 4 v_mul_lo_u32) plus about ten full-rate adds,
# subtracts, compares and selects: 6*2 + 4*4 + 10 = 38 slots.
VALU_LANE_OPS_PER_S = 256 * 128 * 2.4e9
BUTTERFLY_SLOTS = 6 * 2 + 4 * 4 + 10
BUTTERFLY_PEAK = VALU_LANE_OPS_PER_S / BUTTERFLY_SLOTS
PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")


def measured_traffic(family: str, workload: str = "lenet1_plain"):
    """HBM bytes per launch of a kernel family from the committed rocprofv3
    PMC summary, or None when there is none or any kernel source has changed
    since the counters were taken."""
    from paper_2402_03060_amd.profiling import source_digest
    path = os.path.join(PROFILES, f"{family}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2402_03060_amd", "csrc")
    if source_digest(csrc) != kv.get("source_sha256"):
        return None
    return {"bytes_per_launch": float(kv["measured_bytes_per_launch"]),
            "read_bytes_per_launch": float(kv["measured_read_bytes_per_launch"]),
            "write_bytes_per_launch": float(kv["measured_write_bytes_per_launch"]),
            "measured_over_algorithmic": float(kv["measured_over_algorithmic"]),
            "fetch_scale": float(kv["fetch_scale"]), "write_scale": float(kv["write_scale"]),
            "source": os.path.basename(path)}


def roofline_entry(stats: dict, family: str | None = None) -> dict:
    """The roofline of one kernel family (default: the one with the most
    time): achieved = its algorithmic bytes per launch / its average launch
    duration (HIP events on the launch stream), against the 8 TB/s HBM peak;
    for families with an operation count also the butterfly-equivalent rate
    against the derived integer-ALU peak."""
    fam = family if family is not None else max(stats, key=lambda k: stats[k][1])
    n, ms, by, ops = stats[fam]
    n = max(n, 1)
    avg_s = ms / 1e3 / n
    achieved = by / n / avg_s / 1e9
    out = {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "launches": n,
           "avg_us": round(avg_s * 1e6, 3), "bytes_per_launch": round(by / n)}
    if ops > 0:
        out["alu_frac"] = round(ops / n / avg_s / BUTTERFLY_PEAK, 4)
    return out


def family_table(stats: dict, steps: int) -> dict:
    """Per kernel family: launches and time per step, achieved HBM rate on
    its algorithmic bytes and its fraction of 8 TB/s; for NTT passes also the
    butterfly rate against the derived integer-ALU peak."""
    out = {}
    for fam, (n, ms, by, ops) in sorted(stats.items(), key=lambda kv: -kv[1][1]):
        if not n or ms <= 0:
            continue
        sec = ms / 1e3
        e = {"launches_per_step": round(n / steps, 2), "ms_per_step": round(ms / steps, 4),
             "avg_us": round(1e6 * sec / n, 2), "gbs": round(by / sec / 1e9, 1),
             "hbm_frac": round(by / sec / 1e9 / HBM_PEAK_GBS, 4)}
        if ops > 0:
            e["g_butterflies_per_s"] = round(ops / sec / 1e9, 1)
            e["alu_frac"] = round(ops / sec / BUTTERFLY_PEAK, 4)
        out[fam] = e
    return out


def step_distribution(fn, reps: int = 30, warmup: int = 3) -> dict:
    """Per-step GPU time from events around each step on the current stream
    (3 warm-ups, 30 timed repetitions): mean, std, p50, p99 in ms."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return {"reps": reps, "mean_ms": round(float(t.mean()), 4), "std_ms": round(float(t.std()), 4),
            "p50_ms": round(float(np.percentile(t, 50)), 4), "p99_ms": round(float(np.percentile(t, 99)), 4)}


ROT_SIZES = [(13, 3), (14, 8), (14, 4), (15, 8)]      # (log2 N, data limbs)


def rotation_microbench(P, batch: int = 128, hoisted: int = 24) -> dict:
    """Rotations/s at several ring sizes: one rotation of one ciphertext,
    `hoisted` rotations of one ciphertext sharing one ModUp, and one rotation
    of `batch` ciphertexts per launch.  Keys and inputs come from the
    library's own client and are resident before timing."""
    import torch
    out = {}
    for log_n, nl in ROT_SIZES:
        ctx = P.Context(log_n, [60] + [40] * (nl - 1), 60, 2.0 ** 40)
        sk = P.keygen_secret(ctx, 21)
        steps = list(range(1, hoisted + 1))
        keys = [P.gen_switch_key(ctx, sk, 22, steps=r) for r in steps]
        z = np.random.default_rng(23).uniform(-1, 1, ctx.slots)
        pt = ctx.encode(z, ctx.scale, nl, mont=False)
        ctb = P.encrypt_sk(ctx, sk, pt[None].expand(batch, nl, ctx.n).contiguous(), 24, ctx.scale)
        ct1 = P.Ciphertext(ctb.data[:1].clone(), ctx.scale)
        ws1 = ctx.workspace(nl, 1)
        dt1 = timed(lambda: ctx.rotate(ct1, 1, keys[0], ws1), 50, 5)
        wsh = ctx.workspace(nl, hoisted)
        dth = timed(lambda: ctx.rotate_hoisted(ct1, steps, keys, wsh), 10, 2)
        wsb = ctx.workspace(nl, batch)
        dtb = timed(lambda: ctx.rotate(ctb, 1, keys[0], wsb), 5, 1)
        out[f"N=2^{log_n},limbs={nl}"] = {
            "single_per_s": round(50 / dt1, 1),
            f"hoisted{hoisted}_per_s": round(10 * hoisted / dth, 1),
            f"batched{batch}_per_s": round(5 * batch / dtb, 1),
            "key_mb": round(nl * 2 * (nl + 1) * ctx.n * 8 / 1e6, 2)}
        del ctx, sk, keys, ctb, ct1, ws1, wsh, wsb
        torch.cuda.empty_cache()
    return out


# plan variants measured beside the default plan: (name, deferred ModDown, doubling FC sum)
PLAN_VARIANTS = [("deferred ModDown", True, False), ("doubling FC sum", False, True),
                 ("deferred ModDown + doubling FC sum", True, True)]


def batched_leg(P, W, name: str, B: int, per_ct: int, steps: int, tune: bool, lazy: bool, unit: str,
                fc_doubling: bool = False) -> dict:
    """One batched configuration (B ciphertexts of per_ct samples, hoisted,
    graph replay, tuned) in the default plan or a variant: samples/s,
    per-family kernel table and the dominant family's roofline."""
    import torch
    plan = " + ".join([n for n, on in (("deferred ModDown", lazy), ("doubling FC sum", fc_doubling)) if on]) \
        or "default"
    print(f"[bench] setup batched {name} ({B} ciphertexts x {per_ct}, {plan} plan)", file=sys.stderr, flush=True)
    sb = setup(P, W, name, batch=B, tune=tune, mode=P.EVAL_HOISTED | P.EVAL_GRAPH, lazy=lazy,
               fc_doubling=fc_doubling)
    nb, ctb, outb = sb["net"], sb["ct"], sb["outs"]
    stepb = lambda: nb.eval(ctb, outb)
    dtb = timed(stepb, steps, 2)
    rate = steps * B * per_ct / dtb
    dist = step_distribution(stepb, reps=steps, warmup=0)
    errb = max_error(P, W, sb)
    out = {unit: round(rate, 2), "ms_per_launch": round(1e3 * dtb / steps, 2), "launches_timed": steps,
           "launch_distribution": dist, "per_launch": B * per_ct,
           "plan": plan, "max_abs_err_vs_fp64": errb, "tuning": sb["tuning"]}
    sbs = family_stats(P, stepb, 1)
    out["kernel_families"] = family_table(sbs, 1)
    out["roofline"] = roofline_entry(sbs)
    tr = measured_traffic(out["roofline"]["kernel"], name + ("_variant" if lazy else ""))
    if tr is not None:
        out["roofline"]["traffic"] = round(tr["bytes_per_launch"])
        out["roofline"]["traffic_over_algorithmic"] = tr["measured_over_algorithmic"]
    print(f"[bench] batched {name} ({plan}): {rate:.1f} {unit}, max |err| {errb:.2e}", file=sys.stderr, flush=True)
    del sb, nb, ctb, outb, stepb
    torch.cuda.empty_cache()
    return out


def drop_level_bench(P, W, reps: int = 20) -> dict:
    """Drop-Level as Section IV-A writes it on the CIFAR-shaped ring (N =
    2^15, 11 limbs): one ciphertext brought to the network's 8 limbs by three
    products with encrypted all-ones vectors (ones at scale q_l, input scale
    kept), against the limb discard the network uses."""
    import torch
    cfg = W.config("cifar_cnn")
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    sk = P.keygen_secret(ctx, 31)
    rlk = P.gen_switch_key(ctx, sk, 32, relin=True)
    nl = len(ctx.primes)
    z = np.random.default_rng(33).uniform(0, 1, ctx.slots)
    ct = P.encrypt_sk(ctx, sk, ctx.encode(z, ctx.scale, nl, mont=False)[None], 34, ctx.scale)
    ones = []
    for k in range(3):
        q = float(ctx.primes[nl - 1 - k])
        ones.append(P.encrypt_sk(ctx, sk, ctx.encode(np.ones(ctx.slots), q, nl, mont=False)[None], 35 + k, q))
    out = ctx.drop_level(ct, ones, rlk)
    torch.cuda.synchronize()
    err = float(np.abs(P.decrypt_slots(ctx, sk, out, np.arange(64, dtype=np.uint32))[0] - z[:64]).max())
    dt = timed(lambda: ctx.drop_level(ct, ones, rlk), reps, 2)
    dtm = timed(lambda: ctx.mod_drop(ct, nl - 3), reps, 2)
    return {"ms_per_drop": round(1e3 * dt / reps, 4), "limbs": f"{nl} -> {nl - 3}", "products": 3,
            "scale_kept": out.scale == ct.scale, "max_abs_err": err,
            "limb_discard_ms": round(1e3 * dtm / reps, 4), "paper_cpu_seconds_m5": 0.155}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_children(jobs: list, timeout: float) -> list:
    """Run oracle timing children (python -m oracle.timing ...) side by side,
    one thread each; returns their JSON results in order."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    root = os.path.dirname(os.path.abspath(__file__))
    procs = [subprocess.Popen([sys.executable, "-m", "oracle.timing", *args], cwd=root, env=env,
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for args in jobs]
    out = []
    for p in procs:
        so, se = p.communicate(timeout=timeout)
        if p.returncode != 0:
            raise RuntimeError(f"oracle timing child failed ({p.returncode}): {se[-2000:]}")
        out.append(json.loads(so.strip().splitlines()[-1]))
    return out


def cpu_baseline(W, max_procs: int = 16) -> dict:
    """The oracle (scalar C, `%` on 128-bit products, untuned), timed on the
    host's cores, each run in a process of its own on one thread, keys made
    before the timer:
      conv1 (one conv layer, N = 2^13): median of 5 runs, one after another;
      LeNet-1 (N = 2^14): median of 5 runs, five processes side by side;
      batched LeNet-1: one ten-image ciphertext per process, min(cores, 16)
        processes side by side; images/s over what ran (ten images per
        process over the slowest process's time), no extrapolation."""
    nproc = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    procs = max(1, min(avail, max_procs))
    t0 = time.perf_counter()
    c1 = _oracle_children([["--workload", "conv1", "--reps", "5"]], 600)[0]
    c2 = _oracle_children([["--workload", "lenet1"] for _ in range(5)], 900)
    c3 = _oracle_children([["--workload", "lenet1_batched", "--ct-index", str(i)] for i in range(procs)], 900)
    wall = time.perf_counter() - t0
    s1 = float(np.median(c1["seconds"]))
    s2_all = [c["seconds"][0] for c in c2]
    s2 = float(np.median(s2_all))
    s3 = [c["seconds"][0] for c in c3]
    imgs = sum(c["samples"] for c in c3)
    return {"value": round(1.0 / s2, 5), "unit": "inferences/s", "cores": 1, "kind": "oracle",
            "sample": ("LeNet-1 shape, N=2^14, 8 limbs, 288 rotations: median of 5 whole encrypted inferences, "
                       "each one thread in its own process, the 5 side by side"),
            "nproc": nproc, "cores_available": avail, "cpu_model": _cpu_model(),
            "conv1_median_s": round(s1, 3), "conv1_runs_s": [round(x, 3) for x in c1["seconds"]],
            "lenet1_median_s": round(s2, 3), "lenet1_runs_s": [round(x, 3) for x in s2_all],
            "batched": {"images_per_s": round(imgs / max(s3), 4), "processes": procs, "ciphertexts": procs,
                        "images": imgs, "slowest_s": round(max(s3), 3), "fastest_s": round(min(s3), 3)},
            "leg_wall_s": round(wall, 1)}


# The paper's own single-inference times (seconds; SEAL on one Xeon Gold 5220
# core, scale 2^32, trained models): context only, different parameters.
PAPER_MODEL_SECONDS = {"m1": 16.247, "m3": 29.105, "m4": 740.128, "m6": 12.309, "m7": 5.119}
MODEL_NAMES = ["m1", "m3", "m4", "m6", "m7", "cifar_cnn", "lenet1_padded"]
MODEL_LOG_N: dict = {}
# multi-channel workloads also measured with one input ciphertext per channel
CHANNEL_CT_MODELS = ["cifar_cnn"]


def models_bench(P, W, steps: int = 3) -> dict:
    """Each of the paper's other model shapes at its full ring: plain
    evaluation of one ciphertext (graph replay, tuned), inferences/s and the
    largest deviation of the decrypted outputs from the FP64 CNN."""
    import torch
    out = {}
    for name in MODEL_NAMES:
        print(f"[bench] model {name}", file=sys.stderr, flush=True)
        st = setup(P, W, name, batch=1, mode=P.EVAL_PLAIN | P.EVAL_GRAPH, log_n=MODEL_LOG_N.get(name))
        net, ct, outs = st["net"], st["ct"], st["outs"]
        dt = timed(lambda: net.eval(ct, outs), steps, 1)
        err = max_error(P, W, st)
        cfg = st["cfg"]
        out[name] = {"inferences_per_s": round(steps / dt, 3), "ms_per_inference": round(1e3 * dt / steps, 2),
                     "max_abs_err_vs_fp64": err, "log_n": cfg["log_n"], "depth": net.depth,
                     "rotation_keys": len(net.rotations()), "desc": cfg["desc"]}
        if name in PAPER_MODEL_SECONDS:
            out[name]["paper_cpu_seconds"] = PAPER_MODEL_SECONDS[name]
        del st, net, ct, outs
        torch.cuda.empty_cache()
    for name in CHANNEL_CT_MODELS:
        print(f"[bench] model {name}, one input ciphertext per channel", file=sys.stderr, flush=True)
        st = setup(P, W, name, batch=1, mode=P.EVAL_PLAIN | P.EVAL_GRAPH, log_n=MODEL_LOG_N.get(name),
                   channel_cts=True)
        net, ct, outs = st["net"], st["ct"], st["outs"]
        dt = timed(lambda: net.eval(ct, outs), steps, 1)
        out[name + "_channel_cts"] = {"inferences_per_s": round(steps / dt, 3),
                                      "ms_per_inference": round(1e3 * dt / steps, 2),
                                      "max_abs_err_vs_fp64": max_error(P, W, st), "log_n": st["cfg"]["log_n"],
                                      "input_ciphertexts": net.n_inputs, "rotation_keys": len(net.rotations())}
        del st, net, ct, outs
        torch.cuda.empty_cache()
    return out


def headline(res: dict) -> dict:
    """The compact result line (about 2 KB): the headline rate, the batched
    multiple, rotations/s, serving latency, the dominant kernel's roofline
    and the CPU baseline; everything else stays in the detail file."""
    keep = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "max_abs_err_vs_fp64"]
    h = {k: res[k] for k in keep if k in res}
    d = res.get("plain_step_distribution")
    if d:
        h["plain_p50_ms"], h["plain_p99_ms"] = d["p50_ms"], d["p99_ms"]
    if "plain_hoisted_inferences_per_s" in res:
        h["plain_hoisted_inferences_per_s"] = res["plain_hoisted_inferences_per_s"]
    b = res.get("batched")
    if b:
        h["batched"] = {"images_per_s": b["images_per_s"], "multiple_of_plain": b.get("multiple_of_plain"),
                        "images_per_launch": b["per_launch"], "launches_timed": b["launches_timed"],
                        "launch_ms_mean": b["launch_distribution"]["mean_ms"],
                        "launch_ms_p50": b["launch_distribution"]["p50_ms"],
                        "launch_ms_p99": b["launch_distribution"]["p99_ms"],
                        "max_abs_err_vs_fp64": b["max_abs_err_vs_fp64"]}
        if b.get("roofline"):
            h["batched"]["top_kernel"] = {k: b["roofline"][k] for k in ("kernel", "frac", "traffic")}
    for key, unit in (("batched_variant", "images_per_s"), ("batched_cnn1d", "sequences_per_s"),
                      ("batched_cnn1d_variant", "sequences_per_s")):
        v = res.get(key)
        if v:
            h[key] = {unit: v[unit], "plan": v["plan"], "launch_ms_p99": v["launch_distribution"]["p99_ms"]}
            if "multiple_of_plain" in v:
                h[key]["multiple_of_plain"] = v["multiple_of_plain"]
    if "rotations_per_s" in res:
        h["rotations_per_s"] = res["rotations_per_s"]
    sw = res.get("rotation_sweep")
    if sw:
        h["rotations_per_s_single_hoisted24_batched128"] = {
            k.replace("N=2^", "").replace(",limbs=", "/"): [v["single_per_s"], v["hoisted24_per_s"],
                                                           v["batched128_per_s"]] for k, v in sw.items()}
    sv = res.get("serving")
    if sv:
        h["serving"] = {"saturation_requests_per_s": sv["saturation_requests_per_s"],
                        "requests_per_level": sv["requests_per_level"],
                        "p50_p99_ms": {k: [v["p50_ms"], v["p99_ms"]] for k, v in sv["load_levels"].items()}}
    if "roofline" in res:
        h["roofline"] = {k: res["roofline"][k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac",
                                                         "traffic", "avg_us", "alu_frac") if k in res["roofline"]}
    cb = res.get("cpu_baseline")
    if cb:
        h["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample", "nproc",
                                                "cores_available", "cpu_model", "conv1_median_s",
                                                "lenet1_median_s") if k in cb}
        if "batched" in cb:
            h["cpu_baseline"]["batched_images_per_s"] = cb["batched"]["images_per_s"]
            h["cpu_baseline"]["batched_processes"] = cb["batched"]["processes"]
    if "detail_path" in res:
        h["detail"] = res["detail_path"]
    return h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batched-cts", type=int, default=128, help="ciphertexts per batched launch (10 images each)")
    ap.add_argument("--batched-steps", type=int, default=5, help="timed batched launches (after 2 warm-ups)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--only-plain", action="store_true", help="skip every extra measurement (for profiling)")
    ap.add_argument("--no-rotation-sweep", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="default launch parameters instead of the tuned ones")
    ap.add_argument("--models", action="store_true", help="also time the paper's other model shapes")
    ap.add_argument("--no-lazy", action="store_true",
                    help="skip the plan variants (deferred ModDown, doubling FC sum)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per load level of the serving measurement (0 skips it)")
    ap.add_argument("--detail", default=os.path.join(tempfile.gettempdir(), "unihenn_bench_detail.json"),
                    help="file for the full result (kernel tables, tuning, per-model figures)")
    ap.add_argument("--only-batched", action="store_true",
                    help="only the batched LeNet-1 leg in the default plan (for profiling)")
    ap.add_argument("--ntt-probe", type=int, default=0, metavar="ROWS",
                    help="only time forward+inverse NTTs of ROWS limb rows at N=2^14 (kernel throughput)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB three times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.ntt_probe:
        import torch
        import paper_2402_03060_amd as P
        ctx = P.Context(14, [60] + [40] * 7, 60, 2.0 ** 40)
        rows = args.ntt_probe - args.ntt_probe % 8
        t = torch.randint(0, 2 ** 39, (rows // 8, 8, ctx.n), dtype=torch.int64, device="cuda")
        ref = t.clone()
        for _ in range(2):
            ctx.to_ntt(t, 8, rows // 8)
            ctx.from_ntt(t, 8, rows // 8)
        torch.cuda.synchronize()
        reps = args.steps
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.to_ntt(t, 8, rows // 8)
            ctx.from_ntt(t, 8, rows // 8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bfly = 2 * reps * rows * (ctx.n // 2) * 14
        print(json.dumps({"ntt_probe_rows": rows, "roundtrips": reps, "seconds": dt,
                          "butterflies_per_s": bfly / dt, "frac_of_alu_peak": bfly / dt / BUTTERFLY_PEAK,
                          "roundtrip_exact": bool(torch.equal(t, ref))}))
        return
    if args.copy_probe:
        import torch
        x = torch.ones(32 * 1024 * 1024, dtype=torch.int64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": x.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported in this build "
              "(the path shards by ciphertext with replicated keys; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2402_03060_amd as P
    import workloads as W

    log = lambda m: print("[bench] " + m, file=sys.stderr, flush=True)
    if args.only_batched:
        # evaluations made: batched_steps + 2 timed, batched_steps for the
        # distribution, 1 for the kernel families
        r = batched_leg(P, W, "lenet1_batched", args.batched_cts, 10, args.batched_steps, not args.no_tune, False,
                        "images_per_s")
        out = {"images_per_s": r["images_per_s"], "ms_per_launch": r["ms_per_launch"],
               "evaluations": 2 * args.batched_steps + 3, "roofline": r["roofline"]}
        with open(args.detail, "w") as f:
            json.dump(dict(r, evaluations=out["evaluations"]), f, indent=1)
        print(json.dumps(out))
        return
    log("setup plain LeNet-1 (N=2^14)")
    st = setup(P, W, "lenet1", batch=1, tune=not args.no_tune, mode=P.EVAL_PLAIN | P.EVAL_GRAPH)
    net, ct, outs = st["net"], st["ct"], st["outs"]
    step = lambda: net.eval(ct, outs)
    dt = timed(step, args.steps, args.warmup)
    value = args.steps / dt
    err = max_error(P, W, st)
    log(f"plain: {value:.2f} inf/s, max |err| {err:.2e}")
    res = {
        "metric": "encrypted LeNet-1-shape inferences/s, batched vs plain; rotations/s; p99 latency",
        "value": round(value, 3), "unit": "inferences/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * dt / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic, seeded: U[0,1] 28x28 images, weights N(0,0.1^2), biases N(0,0.01^2)",
        "config": {"workload": "plain LeNet-1 shape (conv 1->4 K5, sq, pool2, conv 4->12 K5, sq, pool2, flatten, "
                               "FC 192->10), CKKS N=2^14, primes 60+7x40 (+60 special), scale 2^40, one image per "
                               "ciphertext, one key switch per rotation, one HIP graph per inference"},
        "max_abs_err_vs_fp64": err,
        "tuning": st["tuning"],
    }
    if args.only_plain:
        print(json.dumps(headline(res)))
        return

    stats = family_stats(P, step, args.steps)
    fams = {k: v for k, v in stats.items() if v[0] and v[1] > 0}
    rf = roofline_entry(fams)
    tr = measured_traffic(rf["kernel"])
    if tr is not None:
        rf["traffic"] = round(tr["bytes_per_launch"])
        rf["traffic_over_algorithmic"] = tr["measured_over_algorithmic"]
    res["roofline"] = rf
    res["kernel_families"] = family_table(stats, args.steps)
    res["plain_step_distribution"] = step_distribution(step)

    # hoisted evaluation of the same single-image workload
    net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
    dth = timed(step, args.steps, 1)
    res["plain_hoisted_inferences_per_s"] = round(args.steps / dth, 3)
    net.set_mode(P.EVAL_PLAIN | P.EVAL_GRAPH)

    if not args.no_lazy:
        # the same single-image workload in the plan variants
        res["plain_variants"] = {}
        for vname, lazy, dbl in PLAN_VARIANTS:
            log(f"setup plain LeNet-1, {vname}")
            sl = setup(P, W, "lenet1", batch=1, tune=not args.no_tune, mode=P.EVAL_PLAIN | P.EVAL_GRAPH, lazy=lazy,
                       fc_doubling=dbl)
            nlz, ctl, outl = sl["net"], sl["ct"], sl["outs"]
            stepl = lambda: nlz.eval(ctl, outl)
            dtl = timed(stepl, args.steps, args.warmup)
            nlz.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
            dtlh = timed(stepl, args.steps, 1)
            nlz.set_mode(P.EVAL_PLAIN | P.EVAL_GRAPH)
            fv = family_table(family_stats(P, stepl, args.steps), args.steps)
            res["plain_variants"][vname] = {
                "inferences_per_s": round(args.steps / dtl, 3), "ms_per_step": round(1e3 * dtl / args.steps, 3),
                "hoisted_inferences_per_s": round(args.steps / dtlh, 3),
                "multiple_of_default_plan": round(dt / dtl, 3), "rotation_keys": len(nlz.rotations()),
                "max_abs_err_vs_fp64": max_error(P, W, sl), "tuning": sl["tuning"], "kernel_families": fv}
            log(f"plain, {vname}: {args.steps / dtl:.2f} inf/s")
            del sl, nlz, ctl, outl, stepl
        torch.cuda.empty_cache()

    # rotations/s at the same size (one ciphertext, 8 limbs)
    ctx = st["ctx"]
    ws = ctx.workspace(8, 1)
    key = st["keys"][1]
    full = ctx.empty_ct(1, 8, ctx.scale)
    full.data.copy_(st["ct"].data)
    rot = lambda: ctx.rotate(full, 1, key, ws)
    dtr = timed(rot, 50, 5)
    res["rotations_per_s"] = round(50 / dtr, 1)
    if not args.no_rotation_sweep:
        log("rotation microbenchmark")
        del ws, full
        res["rotation_sweep"] = rotation_microbench(P)

    if not args.no_batched:
        B = args.batched_cts
        del st, step
        torch.cuda.empty_cache()
        # default plan, then deferred ModDown with the doubling FC sum
        plans = [(False, False)] + ([] if args.no_lazy else [(True, True)])
        for lazy, dbl in plans:
            r = batched_leg(P, W, "lenet1_batched", B, 10, args.batched_steps, not args.no_tune, lazy, "images_per_s",
                            fc_doubling=dbl)
            r["multiple_of_plain"] = round(r["images_per_s"] / value, 2)
            res["batched_variant" if lazy else "batched"] = r
        for lazy, dbl in plans:
            r = batched_leg(P, W, "cnn1d", 64, 8, args.batched_steps, not args.no_tune, lazy, "sequences_per_s",
                            fc_doubling=dbl)
            res["batched_cnn1d_variant" if lazy else "batched_cnn1d"] = r

    if args.models:
        res["models"] = models_bench(P, W)
        res["drop_level"] = drop_level_bench(P, W)

    if args.serve_requests:
        from paper_2402_03060_amd.serve import serving_benchmark
        res["serving"] = serving_benchmark(P, W, args.serve_requests, tuning_cache=TUNING_CACHE, log=log)

    if not args.no_cpu_baseline:
        log("CPU oracle baseline (conv1 x5, LeNet-1 x5, batched LeNet-1 on up to 16 processes)")
        res["cpu_baseline"] = cpu_baseline(W)
    res["paper_context"] = {"lenet1_seconds": 30.089, "ten_samples_m1_seconds": 16.247,
                            "hardware": "Intel Xeon Gold 5220 @ 2.2 GHz, SEAL single-threaded, N=2^14, scale 2^32"}
    res["detail_path"] = args.detail
    try:
        with open(args.detail, "w") as f:
            json.dump(res, f, indent=1)
        log(f"full result: {args.detail}")
    except OSError as e:
        log(f"could not write {args.detail}: {e}")
    print(json.dumps(headline(res)))


if __name__ == "__main__":
    main()
