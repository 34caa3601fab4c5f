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

    def set_key(self, r: int | None, key: np.ndarray, keep_coeff: bool = True):
        """Use a key made elsewhere (seeded_keys): rotation r, or the
        relinearisation key when r is None; keep_coeff=False keeps only the
        evaluator's copy."""
        if r is None:
            self.rlk_coeff = key if keep_coeff else None
            self.rlk = self.ck.load_key(key)
        else:
            r = r % self.ck.slots
            if keep_coeff:
                self.key_coeff[r] = key
            self.key_handle[r] = self.ck.load_key(key)

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


# ---- keys from per-key seeded generators (made in parallel processes) ----
KEY_SEED_STRIDE = 1_000_003


def seeded_key_seed(key_seed: int, r: int | None) -> int:
    """Seed of one key's own generator: rotation r (>= 1), or relinearisation
    (r None, seed offset 0)."""
    return key_seed * KEY_SEED_STRIDE + (0 if r is None else int(r))


_worker_ck = None


def _key_worker_init(ring: dict, key_seed: int):
    global _worker_ck
    _worker_ck = OracleCKKS(ring["log_n"], ring["prime_bits"], ring["special_bits"], ring["log_scale"])
    _worker_ck.keygen(key_seed)


def _key_worker(job):
    key_seed, r, levels = job
    k = _worker_ck.seeded_key(seeded_key_seed(key_seed, r), r=r, levels=levels)
    # only the formed rows travel back: digits and limbs below `levels`, then P
    nd = _worker_ck.n_data
    packed = np.concatenate([k[:levels, :, :levels], k[:levels, :, nd:nd + 1]], axis=2)
    return r, packed


def unpack_seeded_key(packed: np.ndarray, n_data: int) -> np.ndarray:
    """The full key layout [n_data][2][n_data + 1][N] of a packed key
    [levels][2][levels + 1][N] (rows not formed are zero)."""
    lv, n = packed.shape[0], packed.shape[-1]
    k = np.zeros((n_data, 2, n_data + 1, n), dtype=np.uint64)
    k[:lv, :, :lv] = packed[:, :, :lv]
    k[:lv, :, n_data] = packed[:, :, lv]
    return k


def seeded_keys(ring: dict, key_seed: int, rotations, levels: int, procs: int = 8):
    """Yield (r, key) for each rotation in `rotations` and (None, relin key),
    each key from its own seeded generator (OracleCKKS.seeded_key) with only
    the rows of `levels` limbs formed, made by `procs` worker processes (each
    a child process with its own copy of the client secret)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n_data = len(ring["prime_bits"])
    jobs = [(key_seed, int(r), levels) for r in rotations] + [(key_seed, None, levels)]
    with cf.ProcessPoolExecutor(max_workers=max(1, procs), mp_context=mp.get_context("spawn"),
                                initializer=_key_worker_init, initargs=(ring, key_seed)) as ex:
        for fut in cf.as_completed([ex.submit(_key_worker, j) for j in jobs]):
            r, packed = fut.result()
            yield r, unpack_seeded_key(packed, n_data)


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
