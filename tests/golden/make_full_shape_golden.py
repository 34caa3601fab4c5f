"""Writes full_<target>.json: the oracle's encrypted evaluations at the real
shapes of the batched and serving workloads, summarised as SHA-256 digests of
coefficient-form residues.  Calls only the CPU oracle.

    python tests/golden/make_full_shape_golden.py [--target NAME] [--procs P]

Targets (each its own ring, keys and plans):
  lenet1_batched  LeNet-1 shape, N = 2^14, ten images per ciphertext at
                  stride 784 (Section III-B packing), positions of a batch of
                  128 ciphertexts;
  cnn1d           the 1D CNN, N = 2^14, eight sequences per ciphertext at
                  stride 1024, positions of a batch of 64;
  cifar_cnn       the 3 x 32 x 32 CNN, N = 2^15, 60 + 10 x 40-bit chain with
                  a 60-bit special prime, input at 11 limbs dropped to 8.
Ciphertext b of a batch packs samples b S .. b S + S - 1 of the seeded inputs
and is encrypted with seed SEED_ENCRYPT + b.  Keys come from per-key seeded
generators (oracle.run.seeded_keys) with the rows of the network's input
level formed.  Each target is evaluated in the default plan and with deferred
ModDown + the doubling FC sum (the plans the benchmark and the server run).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.run import (KEY_SEED_STRIDE, OracleSession, build_net, decrypt_outputs, reference_outputs,  # noqa: E402
                        run_encrypted, seeded_keys)

HERE = os.path.dirname(os.path.abspath(__file__))


def out_path(name: str) -> str:
    return os.path.join(HERE, f"full_{name}.json")


TARGETS = {
    "lenet1_batched": {"batch": 128, "positions": [0, 1, 64, 127]},
    "cnn1d": {"batch": 64, "positions": [0, 63]},
    "cifar_cnn": {"batch": 1, "positions": [0]},
}
PLANS = {"default": (False, False), "lazy_doubling": (True, True)}


def digest(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint64).tobytes())
    return h.hexdigest()


def keys_digest(per_key: dict) -> str:
    """Digest over the per-key digests in order of rotation (relin last)."""
    h = hashlib.sha256()
    for r in sorted(k for k in per_key if k is not None):
        h.update(per_key[r].encode())
    h.update(per_key[None].encode())
    return h.hexdigest()


def compute(name: str, procs: int) -> dict:
    t0 = time.time()
    spec = TARGETS[name]
    cfg = W.config(name)
    sess = OracleSession(cfg)
    S = cfg["samples_per_ct"]
    nets = {p: build_net(cfg, sess.ck.slots, fc_doubling=dbl) for p, (_, dbl) in PLANS.items()}
    levels = nets["default"].depth + 1
    rots = sorted(set(nets["default"].rotation_set()) | set(nets["lazy_doubling"].rotation_set()))
    per_key = {}
    for r, k in seeded_keys(cfg, W.SEED_KEYS, rots, levels, procs=procs):
        per_key[r] = digest([k])
        sess.set_key(r, k, keep_coeff=False)
    print(f"[{name}] {len(rots)} keys in {time.time() - t0:.0f} s", flush=True)
    xs_all = W.gen_inputs(cfg["input"], S * spec["batch"])
    rec = {"workload": cfg["desc"], "log_n": cfg["log_n"], "prime_bits": cfg["prime_bits"],
           "special_bits": cfg["special_bits"], "samples_per_ct": S, "sample_stride": cfg["sample_stride"],
           "batch": spec["batch"], "positions": spec["positions"], "key_seed": W.SEED_KEYS,
           "key_seed_stride": KEY_SEED_STRIDE, "key_levels": levels, "rotations": rots,
           "keys_sha256": keys_digest(per_key), "encrypt_seed_base": W.SEED_ENCRYPT, "plans": {}}
    rec["inputs_sha256"] = {}
    for pname, (lazy, dbl) in PLANS.items():
        net = nets[pname]
        prec = {"rotations": net.rotation_set(), "outputs_sha256": {}, "output_scales": None,
                "max_abs_err_vs_fp64": 0.0}
        for b in spec["positions"]:
            xs = xs_all[b * S:(b + 1) * S]
            ct, outs, _ = run_encrypted(sess, net, xs, enc_seed=W.SEED_ENCRYPT + b, lazy=lazy)
            cts = ct if isinstance(ct, list) else [ct]
            rec["inputs_sha256"][str(b)] = digest([c.data for c in cts])
            prec["outputs_sha256"][str(b)] = digest([o.data for o in outs])
            prec["output_scales"] = [o.scale for o in outs]
            prec["output_limbs"] = [int(o.data.shape[1]) for o in outs]
            got = decrypt_outputs(sess, net, outs)
            ref = reference_outputs(net, xs)
            prec["max_abs_err_vs_fp64"] = max(prec["max_abs_err_vs_fp64"], float(np.abs(got - ref).max()))
            print(f"[{name}] {pname} position {b}: {time.time() - t0:.0f} s", flush=True)
        rec["plans"][pname] = prec
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--target", choices=sorted(TARGETS), action="append")
    ap.add_argument("--procs", type=int, default=8, help="key-generation worker processes")
    a = ap.parse_args()
    for name in a.target or sorted(TARGETS):
        rec = compute(name, a.procs)
        with open(out_path(name), "w") as f:
            json.dump(rec, f, indent=1)
        print(name, json.dumps(rec["plans"]["default"]["outputs_sha256"]))


if __name__ == "__main__":
    main()
