"""Writes lenet1_full.json: the oracle's encrypted LeNet-1 evaluation at the
full ring size (N = 2^14, 60 + 7 x 40-bit chain, 60-bit special prime) on the
first seeded input image, summarised as SHA-256 digests of the coefficient-form
residues.  Calls only the CPU oracle.

    python tests/golden/make_lenet1_golden.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.run import OracleSession, build_net, decrypt_outputs, reference_outputs, run_encrypted  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lenet1_full.json")


def digest(arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint64).tobytes())
    return h.hexdigest()


def compute() -> dict:
    cfg = W.config("lenet1")
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    ct, outs, _ = run_encrypted(sess, net, xs)
    got = decrypt_outputs(sess, net, outs)[0]
    ref = reference_outputs(net, xs)[0]
    rec = {
        "workload": "LeNet-1 shape, N = 2^14, one image per ciphertext",
        "key_seed": W.SEED_KEYS, "encrypt_seed": W.SEED_ENCRYPT, "input_index": 0,
        "rotations": net.rotation_set(),
        "input_sha256": digest([ct.data]),
        "keys_sha256": digest([sess.key_coeff[r] for r in sorted(sess.key_coeff)] + [sess.rlk_coeff]),
        "n_outputs": len(outs),
        "output_scales": [o.scale for o in outs],
        "output_limbs": [int(o.data.shape[1]) for o in outs],
        "outputs_sha256": digest([o.data for o in outs]),
        "max_abs_err_vs_fp64": float(np.abs(got - ref).max()),
    }
    return rec


def main():
    rec = compute()
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec)[:400])


if __name__ == "__main__":
    main()
