"""Times the oracle on whole encrypted evaluations of one workload.

TEST INFRASTRUCTURE ONLY: run by the benchmark's CPU-baseline leg as child
processes (one thread each).  The product library never imports this.

    python -m oracle.timing --workload lenet1 --reps 5
    python -m oracle.timing --workload lenet1_batched --ct-index 3

Keys are made before any timer starts.  Each repetition encrypts the packed
inputs of ciphertext `ct-index` (samples_per_ct inputs) and evaluates the
network in the oracle (client encryption included, decryption not).  Prints
one JSON line: the workload, the seconds of every repetition and the number
of threads the process ran on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--reps", type=int, default=1)
    ap.add_argument("--ct-index", type=int, default=0, help="which ciphertext of the seeded inputs")
    a = ap.parse_args()
    import workloads as W
    from oracle.run import OracleSession, build_net, run_encrypted
    cfg = W.config(a.workload)
    S = cfg["samples_per_ct"]
    t0 = time.perf_counter()
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    sess.ensure_keys(net.rotation_set())
    keys_s = time.perf_counter() - t0
    xs = W.gen_inputs(cfg["input"], S * (a.ct_index + 1))[S * a.ct_index:]
    secs = []
    for r in range(a.reps):
        t0 = time.perf_counter()
        run_encrypted(sess, net, xs, enc_seed=W.SEED_ENCRYPT + a.ct_index)
        secs.append(time.perf_counter() - t0)
    print(json.dumps({"workload": a.workload, "ct_index": a.ct_index, "samples": S, "seconds": secs,
                      "keygen_seconds": keys_s, "threads": 1, "rotations_per_eval": len(net.rotation_set())}))


if __name__ == "__main__":
    main()
