"""Encrypted end-to-end runs of the oracle network (client + evaluator).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU-baseline leg).
"""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle.ckks import OracleCKKS
from oracle.network import CkksEval, LazyCkksEval, Net, cnn_fp64, read_outputs


class OracleSession:
    """Keys and context for one ring; keys for a set of rotations + relin."""

    def __init__(self, ring: dict, key_seed: int = W.SEED_KEYS):
        self.ck = OracleCKKS(ring["log_n"], ring["prime_bits"], ring["special_bits"], ring["log_scale"])
        self.ck.keygen(key_seed)
        self.key_coeff: dict[int, np.ndarray] = {}
        self.key_handle: dict[int, object] = {}
        self.rlk_coeff = None
        self.rlk = None

    def ensure_keys(self, rotations, relin: bool = True):
        for r in rotations:
            r = r % self.ck.slots
            if r and r not in self.key_handle:
                k = self.ck.rotation_key(r)
                self.key_coeff[r] = k
                self.key_handle[r] = self.ck.load_key(k)
        if relin and self.rlk is None:
            self.rlk_coeff = self.ck.relin_key()
            self.rlk = self.ck.load_key(self.rlk_coeff)


def build_net(cfg: dict, n_slots: int, params=None, fc_doubling: bool = False, channel_cts: bool = False) -> Net:
    params = W.gen_params(cfg["layers"]) if params is None else params
    return Net(cfg["input"], cfg["layers"], params, n_slots, cfg["samples_per_ct"], cfg["sample_stride"],
               fc_doubling=fc_doubling, channel_cts=channel_cts)


def run_encrypted(sess: OracleSession, net: Net, xs: np.ndarray, enc_seed: int = W.SEED_ENCRYPT,
                  lazy: bool = False):
    """Encrypt the packed inputs, drop to the network depth, evaluate (with
    lazy: deferred ModDown, LazyCkksEval).
    Returns (input ciphertext, output ciphertexts, evaluator); with the net's
    channel_cts the input is a list of one ciphertext per channel, encrypted
    with seeds enc_seed, enc_seed + 1000, ..."""
    ck = sess.ck
    sess.ensure_keys(net.rotation_set())
    cts = [ck.encrypt(v, enc_seed + 1000 * i) for i, v in enumerate(net.input_vectors(xs))]
    xs_in = [ck.limb_drop(ct, net.depth + 1) for ct in cts]
    ev = (LazyCkksEval if lazy else CkksEval)(ck, sess.key_handle, sess.rlk)
    outs = net.run(ev, xs_in)
    return (cts if net.channel_cts else cts[0]), outs, ev


def decrypt_outputs(sess: OracleSession, net: Net, outs) -> np.ndarray:
    return read_outputs(net, [sess.ck.decrypt(o) for o in outs])


def reference_outputs(net: Net, xs: np.ndarray) -> np.ndarray:
    return np.array([cnn_fp64(x, net.layers, net.params).reshape(-1) for x in xs])
