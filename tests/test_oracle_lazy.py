"""Pins of the oracle's deferred-ModDown evaluator (extended ciphertexts over
{q_0..q_{l}, P}) against things other than itself: brute-force integer
arithmetic on tiny rings (schoolbook products, direct substitution, CRT with
exact rounding), the already pinned eager rotation, and the FP64 CNN.
No GPU."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle.ckks import Ciphertext, ExtCiphertext, OracleCKKS
from tests import bigint_ref as R


@pytest.fixture(scope="module")
def tiny():
    ring = W.TINY_RINGS["n16"]
    ck = OracleCKKS(ring["log_n"], ring["prime_bits"], ring["special_bits"], ring["log_scale"])
    ck.keygen(W.SEED_KEYS)
    return ck


@pytest.fixture(scope="module")
def mid():
    ring = W.TINY_RINGS["n1024"]
    ck = OracleCKKS(ring["log_n"], ring["prime_bits"], ring["special_bits"], ring["log_scale"])
    ck.keygen(W.SEED_KEYS)
    return ck


def _rand_ct(ck, rng, nl, ext=False):
    mods = ck.primes[:nl] + ([ck.special] if ext else [])
    return np.stack([np.stack([rng.integers(0, q, ck.n, dtype=np.uint64) for q in mods]) for _ in range(2)])


def test_rotate_ext_bruteforce(tiny):
    """(P tau_g(c0) + sum_j d_j evk_{j,0}, sum_j d_j evk_{j,1}) on integers,
    d_j the centered residues of tau_g(c1) mod q_j, reduced mod q_i and P."""
    rng = np.random.default_rng(41)
    r = 3
    key = tiny.rotation_key(r)
    h = tiny.load_key(key)
    g = tiny.galois_elt(r)
    N = tiny.n
    for nl in [3, 2]:
        ct = _rand_ct(tiny, rng, nl)
        got = tiny.rotate_ext(Ciphertext(ct, 1.0), r, h).data
        mods = tiny.primes[:nl] + [tiny.special]
        key_limbs = list(range(nl)) + [key.shape[2] - 1]
        tc1 = [R.substitute([int(x) for x in ct[1, j]], g, N, tiny.primes[j]) for j in range(nl)]
        for c in range(2):
            U = [0] * N
            for j in range(nl):
                dj = [R.centered(x, tiny.primes[j]) for x in tc1[j]]
                ev = [R.crt([int(key[j, c, li, t]) for li in key_limbs], mods)[0] for t in range(N)]
                U = [u + p for u, p in zip(U, R.negacyclic(dj, ev, N))]
            for i, q in enumerate(mods):
                exp = [u % q for u in U]
                if c == 0 and i < nl:
                    tc0 = R.substitute([int(x) for x in ct[0, i]], g, N, q)
                    exp = [(e + tiny.special * t) % q for e, t in zip(exp, tc0)]
                assert [int(x) for x in got[c, i]] == exp


def test_moddown_bruteforce(tiny):
    """ModDown = round(E / P) of the CRT integer of (E mod q_i, E mod P), mod q_i."""
    rng = np.random.default_rng(42)
    for nl in [3, 1]:
        data = _rand_ct(tiny, rng, nl, ext=True)
        out = tiny.moddown(ExtCiphertext(data, 1.0)).data
        mods = tiny.primes[:nl] + [tiny.special]
        for c in range(2):
            for t in range(tiny.n):
                x, _ = R.crt([int(data[c, i, t]) for i in range(nl + 1)], mods)
                v = R.round_div(x, tiny.special)
                for i in range(nl):
                    assert int(out[c, i, t]) == v % tiny.primes[i]


def test_mac_matrix_ext_schoolbook(tiny):
    """Extended MAC limb by limb, the P limb included, against schoolbook
    negacyclic products."""
    rng = np.random.default_rng(43)
    nl = 2
    mods = tiny.primes[:nl] + [tiny.special]
    cts = [ExtCiphertext(_rand_ct(tiny, rng, nl, ext=True), 1.0) for _ in range(3)]
    pts = [[np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in mods]) for _ in range(3)]
           for _ in range(2)]
    pts[0][1] = None
    accs = tiny.mac_matrix_ext(cts, pts)
    for o in range(2):
        for c in range(2):
            for i, q in enumerate(mods):
                exp = [0] * tiny.n
                for t in range(3):
                    if pts[o][t] is None:
                        continue
                    p = R.negacyclic([int(x) for x in pts[o][t][i]], [int(x) for x in cts[t].data[c, i]], tiny.n, q)
                    exp = [(a + b) % q for a, b in zip(exp, p)]
                assert [int(x) for x in accs[o][c, i]] == exp


def test_add_and_to_ext(tiny):
    rng = np.random.default_rng(44)
    nl = 3
    a = ExtCiphertext(_rand_ct(tiny, rng, nl, ext=True), 1.0)
    b = ExtCiphertext(_rand_ct(tiny, rng, nl, ext=True), 1.0)
    s = tiny.add_ext(a, b).data
    x = _rand_ct(tiny, rng, nl)
    e = tiny.to_ext(Ciphertext(x, 1.0)).data
    for i, q in enumerate(tiny.primes[:nl] + [tiny.special]):
        assert np.array_equal(s[:, i], (a.data[:, i] + b.data[:, i]) % np.uint64(q))
        exp = [(tiny.special * int(v)) % q for v in x[:, i].ravel()] if i < nl else [0] * (2 * tiny.n)
        assert [int(v) for v in e[:, i].ravel()] == exp


def test_moddown_inverts_to_ext_and_rotate_ext(mid):
    """ModDown(P ct) = ct and ModDown(rotate_ext(ct, r)) = Rot(ct, r), bit for
    bit (P tau(c0) divides exactly)."""
    z = W.gen_slots(mid.slots, 1, seed=45)[0]
    ct = mid.limb_drop(mid.encrypt(z, 46), 3)
    assert np.array_equal(mid.moddown(mid.to_ext(ct)).data, ct.data)
    for r in [1, 7, -5]:
        k = mid.load_key(mid.rotation_key(r))
        assert np.array_equal(mid.moddown(mid.rotate_ext(ct, r, k)).data, mid.rotate(ct, r, k).data)


def test_encode_ext_carries_residue_mod_p(mid):
    """The plaintext's limb nl is the same integer polynomial mod P: the
    centered CRT of the data limbs, reduced mod P."""
    z = W.gen_slots(mid.slots, 1, seed=47)[0]
    nl = 3
    ws = [0.25, -1.5]
    e = mid.encode_scaled_ext(z, ws, mid.delta, nl)
    p = mid.encode_scaled(z, ws, mid.delta, nl)
    assert np.array_equal(e[:, :nl], p)
    for w in range(len(ws)):
        ints = mid.crt_centered(p[w])
        assert [int(v) for v in e[w, nl]] == [v % mid.special for v in ints]


def test_one_moddown_per_sum_stays_close(mid):
    """sum_t pt_t * Rot(ct, r_t) with one ModDown of the extended sum differs
    in its bits from the eager sum (which rounds once per term), decrypts
    within 1e-7 of it, and both decrypt to the slot-wise result."""
    z = W.gen_slots(mid.slots, 1, seed=48)[0]
    ct = mid.limb_drop(mid.encrypt(z, 49), 3)
    rs = [0, 1, 5, 33]
    keys = {r: mid.load_key(mid.rotation_key(r)) for r in rs if r}
    ws = [0.5, -0.25, 0.75, 1.0]
    mask = np.ones(mid.slots)
    pts = mid.encode_scaled(mask, ws, mid.delta, ct.nl)
    ptx = mid.encode_scaled_ext(mask, ws, mid.delta, ct.nl)
    eager = [ct if r == 0 else mid.rotate(ct, r, keys[r]) for r in rs]
    lazy = [mid.to_ext(ct) if r == 0 else mid.rotate_ext(ct, r, keys[r]) for r in rs]
    acc_e = mid.mac_matrix(eager, [list(pts)])[0]
    acc_l = mid.moddown(ExtCiphertext(mid.mac_matrix_ext(lazy, [list(ptx)])[0], ct.scale)).data
    assert not np.array_equal(acc_e, acc_l)
    sc = ct.scale * mid.delta
    de = mid.decrypt(mid.rescale(Ciphertext(acc_e, sc)))
    dl = mid.decrypt(mid.rescale(Ciphertext(acc_l, sc)))
    exp = sum(w * np.roll(z, -r) for w, r in zip(ws, rs))
    assert np.abs(de - exp).max() < 1e-6
    assert np.abs(dl - exp).max() < 1e-6
    assert np.abs(de - dl).max() < 1e-7


def test_lazy_conv1_config():
    """Conv + square (the conv1 configuration, N = 2^13) with deferred
    ModDown: same primitive counts, outputs within 1e-3 of FP64, and a
    result that differs in its bits from the eager evaluator."""
    from oracle.run import OracleSession, build_net, decrypt_outputs, reference_outputs, run_encrypted
    cfg = W.config("conv1")
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, ev = run_encrypted(sess, net, xs, lazy=True)
    assert ev.count.as_dict() == {"rot": 24, "mac": 100, "rescale": 8, "relin": 4}
    got = decrypt_outputs(sess, net, outs)
    assert all(isinstance(o, Ciphertext) and o.nl == 1 for o in outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3
    _, eager, _ = run_encrypted(sess, net, xs)
    assert not np.array_equal(eager[0].data, outs[0].data)


@pytest.mark.slow
def test_lazy_lenet1_small_ring():
    """LeNet-1 at N = 2^11: pooling sums and the flatten and FC sums stay
    extended; outputs within 1e-3 of the FP64 CNN."""
    from oracle.run import OracleSession, build_net, decrypt_outputs, reference_outputs, run_encrypted
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, _ = run_encrypted(sess, net, xs, lazy=True)
    assert all(o.nl == 1 for o in outs)
    got = decrypt_outputs(sess, net, outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3


def test_lazy_relu_after_pooling():
    """Approximate ReLU right after pooling receives an extended sum: its
    first product stays extended, its Mul(C) takes the ModDown.  Outputs
    within 1e-3 of the FP64 CNN (N = 2^11)."""
    from oracle.network import Net, read_outputs, cnn_fp64
    from oracle.run import OracleSession, run_encrypted
    inp = {"c": 1, "h": 12, "w": 12, "dist": "uniform01"}
    layers = [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1}, {"kind": "avgpool", "c": 2},
              W.RELU, W.FLATTEN, {"kind": "fc", "din": 50, "dout": 4}]
    ring = dict(W.config("lenet1"), log_n=11)
    sess = OracleSession(ring)
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    net = Net(inp, layers, params, sess.ck.slots)
    _, outs, _ = run_encrypted(sess, net, xs, lazy=True)
    got = read_outputs(net, [sess.ck.decrypt(o) for o in outs])
    assert np.abs(got[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-3
