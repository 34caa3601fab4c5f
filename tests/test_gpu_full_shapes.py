"""Bit-exact parity at the real shapes of the batched and serving workloads:
LeNet-1 with ten images per ciphertext at stride 784 in a batch of 128
ciphertexts, the 1D CNN with eight sequences at stride 1024 in a batch of 64
(both at N = 2^14), and the 3 x 32 x 32 CNN at N = 2^15 with its input at 11
limbs dropped to 8.  The GPU runs the launch settings the benchmark and the
server use (the tuning cache, hoisted graph replay) and the row-fused inner
product in plain mode; sampled batch positions must hash to the digests the
oracle wrote (tests/golden/make_full_shape_golden.py).  Positions the oracle
did not evaluate hold random residues: each batch entry is evaluated on its
own, so they must not disturb the sampled ones."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.run import OracleSession, build_net, seeded_keys

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_CACHE = os.path.join(os.path.dirname(HERE), "paper_2402_03060_amd", "tuning_cache.json")
PLANS = {"default": (False, False), "lazy_doubling": (True, True)}


def _digest(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint64).tobytes())
    return h.hexdigest()


def _golden(name: str) -> dict:
    with open(os.path.join(HERE, "golden", f"full_{name}.json")) as f:
        return json.load(f)


def _procs() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 8


def _setup(name: str, batch: int | None = None):
    """Oracle client (keys from per-key seeded generators, encryptions of the
    sampled positions) and the GPU context with those keys and a batch of
    `batch` (default: the golden's) ciphertexts."""
    import paper_2402_03060_amd as P
    rec = _golden(name)
    cfg = W.config(name)
    sess = OracleSession(cfg, key_seed=rec["key_seed"])
    ck = sess.ck
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    assert ctx.primes == ck.primes and ctx.special == ck.special
    per_key, keys = {}, {}
    for r, k in seeded_keys(cfg, rec["key_seed"], rec["rotations"], rec["key_levels"], procs=_procs()):
        per_key[r] = _digest([k])
        keys[r] = ctx.import_evk(k)
    h = hashlib.sha256()
    for r in sorted(k for k in per_key if k is not None):
        h.update(per_key[r].encode())
    h.update(per_key[None].encode())
    assert h.hexdigest() == rec["keys_sha256"]
    rlk = keys.pop(None)
    onet = build_net(cfg, ck.slots)
    B, S = batch or rec["batch"], rec["samples_per_ct"]
    xs_all = W.gen_inputs(cfg["input"], S * B)
    rng = np.random.default_rng(2024)
    arr = np.empty((B, 2, ck.n_data, ck.n), dtype=np.uint64)
    for b in range(B):
        if b in rec["positions"]:
            ct = ck.encrypt(onet.input_vector(xs_all[b * S:(b + 1) * S]), rec["encrypt_seed_base"] + b)
            assert _digest([ct.data]) == rec["inputs_sha256"][str(b)], b
            arr[b] = ct.data
        else:
            for c in range(2):
                for i, q in enumerate(ck.primes):
                    arr[b, c, i] = rng.integers(0, q, ck.n, dtype=np.uint64)
    gin = ctx.import_ct(arr, ctx.scale)
    return rec, cfg, ctx, keys, rlk, gin


def _check(P, ctx, net, gin, rec, plan, what):
    outs = net.eval(gin)
    prec = rec["plans"][plan]
    assert [o.scale for o in outs] == prec["output_scales"], what
    got = [ctx.export_ct(o) for o in outs]
    for b in rec["positions"]:
        assert _digest([g[b] for g in got]) == prec["outputs_sha256"][str(b)], (what, b)


def _net(P, ctx, cfg, rec, keys, rlk, plan, max_batch):
    lazy, dbl = PLANS[plan]
    net = P.Net(ctx, cfg["input"], cfg["layers"], W.gen_params(cfg["layers"]), samples=rec["samples_per_ct"],
                stride=rec["sample_stride"], max_batch=max_batch, lazy=lazy, fc_doubling=dbl)
    assert sorted(net.rotations()) == rec["plans"][plan]["rotations"]
    net.bind_keys({r: keys[r] for r in net.rotations()}, rlk)
    return net


@pytest.fixture
def cache(tmp_path):
    """A copy of the tuning cache: a setting missing from it is tuned and
    written to the copy only."""
    import shutil
    dst = tmp_path / "tuning_cache.json"
    shutil.copy(TUNING_CACHE, dst)
    return str(dst)


@pytest.mark.parametrize("name", ["lenet1_batched", "cnn1d"])
def test_batched_full_shape_bit_exact(name, monkeypatch, cache):
    """Both plans in hoisted graph replay at the tuned launch settings of the
    whole batch, then the default plan in plain mode with the row-fused
    inner product on every group."""
    import torch
    import paper_2402_03060_amd as P
    monkeypatch.setenv("UNIHENN_KS_FUSE_MIN_WG", "0")
    rec, cfg, ctx, keys, rlk, gin = _setup(name)
    for plan in PLANS:
        net = _net(P, ctx, cfg, rec, keys, rlk, plan, rec["batch"])
        net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
        net.autotune(rec["batch"], cache_path=cache)
        _check(P, ctx, net, gin, rec, plan, (plan, "hoisted graph, tuned"))
        if plan == "default":
            net.set_mode(P.EVAL_PLAIN | P.EVAL_GRAPH)
            net.set_tuning(ks_group=4, ks_order=2)
            _check(P, ctx, net, gin, rec, plan, (plan, "plain, row-fused"))
        del net
        torch.cuda.empty_cache()


def test_cifar_cnn_full_ring_bit_exact(monkeypatch, cache):
    """N = 2^15, 11 limbs dropped to 8, in a batch of 4 as the server forms
    them: the default plan in plain graph replay at the tuned settings and
    with the row-fused inner product on every group (NTT splits 7 and 8), and
    deferred ModDown + doubling FC sum in hoisted graph replay as the server
    runs it."""
    import torch
    import paper_2402_03060_amd as P
    monkeypatch.setenv("UNIHENN_KS_FUSE_MIN_WG", "0")
    rec, cfg, ctx, keys, rlk, gin = _setup("cifar_cnn", batch=4)
    net = _net(P, ctx, cfg, rec, keys, rlk, "default", 4)
    net.set_mode(P.EVAL_PLAIN | P.EVAL_GRAPH)
    net.autotune(1, cache_path=cache)
    _check(P, ctx, net, gin, rec, "default", "plain graph, tuned")
    for split in (7, 8):
        net.set_tuning(ks_group=64, ks_order=2, ntt_split=split, ntt_tile_log=11)
        _check(P, ctx, net, gin, rec, "default", ("plain, row-fused", split))
    del net
    torch.cuda.empty_cache()
    net = _net(P, ctx, cfg, rec, keys, rlk, "lazy_doubling", 4)
    net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
    net.autotune(4, cache_path=cache)
    _check(P, ctx, net, gin, rec, "lazy_doubling", "hoisted graph, tuned")
