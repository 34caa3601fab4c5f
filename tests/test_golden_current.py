"""The stored oracle digests still describe what the oracle does now: the
rotation sets and key levels of the full-shape records and the digest of
each record's first encrypted input are recomputed from the oracle (the
whole evaluations take tens of minutes; tests/golden/make_full_shape_golden.py
rewrites them)."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.run import OracleSession, build_net

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _digest(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint64).tobytes())
    return h.hexdigest()


@pytest.mark.slow
@pytest.mark.parametrize("name", ["lenet1_batched", "cnn1d", "cifar_cnn"])
def test_full_shape_golden_setup_is_current(name):
    with open(os.path.join(GOLD, f"full_{name}.json")) as f:
        rec = json.load(f)
    cfg = W.config(name)
    assert rec["log_n"] == cfg["log_n"] and rec["prime_bits"] == cfg["prime_bits"]
    assert rec["samples_per_ct"] == cfg["samples_per_ct"] and rec["sample_stride"] == cfg["sample_stride"]
    sess = OracleSession(cfg, key_seed=rec["key_seed"])
    nets = {"default": build_net(cfg, sess.ck.slots), "lazy_doubling": build_net(cfg, sess.ck.slots, fc_doubling=True)}
    assert rec["key_levels"] == nets["default"].depth + 1
    for plan, net in nets.items():
        assert rec["plans"][plan]["rotations"] == net.rotation_set()
    assert rec["rotations"] == sorted(set(nets["default"].rotation_set()) | set(nets["lazy_doubling"].rotation_set()))
    S = cfg["samples_per_ct"]
    b = rec["positions"][0]
    xs = W.gen_inputs(cfg["input"], S * (b + 1))[b * S:(b + 1) * S]
    ct = sess.ck.encrypt(nets["default"].input_vector(xs), rec["encrypt_seed_base"] + b)
    assert _digest([ct.data]) == rec["inputs_sha256"][str(b)]
    # decrypted outputs the oracle recorded stay within the bound against FP64
    for plan in rec["plans"].values():
        assert plan["max_abs_err_vs_fp64"] < 1e-3
