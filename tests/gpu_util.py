"""Helpers shared by the GPU parity tests: oracle sessions (client role) and
conversion of their keys and ciphertexts into the library's device form."""
from __future__ import annotations

import numpy as np

import workloads as W
from oracle.ckks import Ciphertext as OCt
from oracle.ckks import OracleCKKS


def oracle_ring(name_or_ring, key_seed: int = W.SEED_KEYS) -> OracleCKKS:
    ring = W.TINY_RINGS[name_or_ring] if isinstance(name_or_ring, str) else name_or_ring
    ck = OracleCKKS(ring["log_n"], ring["prime_bits"], ring["special_bits"], ring["log_scale"])
    ck.keygen(key_seed)
    return ck


def gpu_ctx_for(ck: OracleCKKS, ring: dict):
    from paper_2402_03060_amd import Context
    ctx = Context(ring["log_n"], ring["prime_bits"], ring["special_bits"], 2.0 ** ring["log_scale"])
    assert ctx.primes == ck.primes and ctx.special == ck.special
    return ctx


def random_ct(ck: OracleCKKS, nl: int, seed: int, batch: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.stack([np.stack([np.stack([rng.integers(0, q, ck.n, dtype=np.uint64) for q in ck.primes[:nl]])
                               for _ in range(2)]) for _ in range(batch)])


def ocat(arr: np.ndarray, scale: float = 1.0) -> OCt:
    return OCt(np.ascontiguousarray(arr), scale)
