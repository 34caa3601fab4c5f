"""Pins of the CPU oracle against things other than itself: number theory,
schoolbook products, exact big-integer CRT and rounding, a decimal evaluation
of the encoding sum, slot-level invariants and the paper's printed facts.
No GPU."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.ckks import OracleCKKS, gen_primes
from tests import bigint_ref as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


# ---------------------------------------------------------------- primes
@pytest.mark.parametrize("name", ["conv1", "lenet1", "cifar_cnn"])
def test_prime_chain(name):
    cfg = W.config(name)
    bits = cfg["prime_bits"] + [cfg["special_bits"]]
    ps = gen_primes(cfg["log_n"], bits)
    two_n = 2 << cfg["log_n"]
    assert len(set(ps)) == len(ps)
    for i, (p, b) in enumerate(zip(ps, bits)):
        assert p.bit_length() == b and p % two_n == 1 and R.is_prime(p)
        # largest: every candidate above it that is = 1 mod 2N is composite or used earlier
        c = p + two_n
        while c < (1 << b):
            assert (not R.is_prime(c)) or c in ps[:i]
            c += two_n


def test_prime_chain_survey_values():
    """Cross-check with the chain computed independently when the work was
    surveyed (same selection rule)."""
    assert gen_primes(13, [60, 40, 40, 60]) == [1152921504606830593, 1099511480321, 1099510890497,
                                                1152921504606748673]
    assert gen_primes(14, [60] + [40] * 7 + [60])[-1] == 1152921504606683137


# ---------------------------------------------------------------- ring arithmetic
def test_poly_mul_schoolbook(tiny):
    rng = np.random.default_rng(5)
    N = tiny.n
    for mi, q in enumerate(tiny.primes + [tiny.special]):
        a = [int(x) for x in rng.integers(0, q, N, dtype=np.uint64)]
        b = [int(x) for x in rng.integers(0, q, N, dtype=np.uint64)]
        out = np.zeros(N, dtype=np.uint64)
        from oracle.ckks import lib, _p64
        lib().or_poly_mul(tiny.ctx, mi, _p64(np.array(a, dtype=np.uint64)), _p64(np.array(b, dtype=np.uint64)),
                          _p64(out))
        assert [int(x) for x in out] == R.negacyclic(a, b, N, q)


def test_automorphism_substitution(tiny):
    rng = np.random.default_rng(6)
    N = tiny.n
    a = np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in tiny.primes])
    for r in [1, 2, 3, -1]:
        g = tiny.galois_elt(r)
        assert g == pow(5, r % (N // 2), 2 * N)
        out = tiny.automorphism(a, g)
        for i, q in enumerate(tiny.primes):
            assert [int(x) for x in out[i]] == R.substitute([int(x) for x in a[i]], g, N, q)


# ---------------------------------------------------------------- encoding
def test_encode_matches_decimal_closed_form(tiny):
    """Rounded integers equal round-half-away of the 60-digit decimal value."""
    rng = np.random.default_rng(7)
    N = tiny.n
    z = rng.uniform(-1, 1, N // 2)
    scale = 2.0 ** 30
    pt = tiny.encode(z, scale, len(tiny.primes))
    exact = R.encode_exact(z, N, scale)
    hi, lo = tiny.real_transform(z)
    for j in range(N):
        v = R.round_half_away(exact[j])
        for i, q in enumerate(tiny.primes):
            assert int(pt[i, j]) == v % q
        # the binary128 transform agrees with the decimal one far below 1/2 ulp of the scaled value
        assert abs(float(exact[j] / int(scale) - R.Decimal(hi[j]) - R.Decimal(lo[j]))) < 1e-28


def test_encode_scaled_is_encode_of_product(tiny):
    rng = np.random.default_rng(8)
    z = np.zeros(tiny.slots)
    z[[0, 3, 5]] = 1.0
    ws = rng.normal(0, 0.1, 5)
    batch = tiny.encode_scaled(z, ws, 2.0 ** 30, 2)
    for w, pt in zip(ws, batch):
        assert np.array_equal(pt, tiny.encode(w * z, 2.0 ** 30, 2))


def test_decode_encode_roundtrip(mid):
    z = W.gen_slots(mid.slots, 1, seed=9)[0]
    pt = mid.encode(z, mid.delta, 2)
    back = mid.decode(pt, mid.delta)
    assert np.abs(back - z).max() < 1e-9


def test_encode_rotation_equivariance(mid):
    """Encode(roll(z, -r)) == tau_{5^r}(Encode(z)), bit for bit."""
    z = W.gen_slots(mid.slots, 1, seed=10)[0]
    pt = mid.encode(z, mid.delta, 3)
    for r in [1, 7, mid.slots // 4, -3]:
        assert np.array_equal(mid.encode(np.roll(z, -r), mid.delta, 3), mid.automorphism(pt, mid.galois_elt(r)))


# ---------------------------------------------------------------- encryption
def test_encrypt_decrypt(mid):
    z = W.gen_slots(mid.slots, 1, seed=11)[0]
    ct = mid.encrypt(z, 12)
    assert np.abs(mid.decrypt(ct) - z).max() < 1e-7


# ---------------------------------------------------------------- key switching
def _ks_bruteforce(ck, d, key, nl):
    """round((sum_j centered(d mod q_j) * evk_j) / P) mod q_i, on integers."""
    N = ck.n
    mods = ck.primes[:nl] + [ck.special]
    key_limbs = list(range(nl)) + [key.shape[2] - 1]
    out = np.zeros((2, nl, N), dtype=np.uint64)
    for c in range(2):
        U = [0] * N
        for j in range(nl):
            dj = [R.centered(int(x), ck.primes[j]) for x in d[j]]
            ev = [R.crt([int(key[j, c, li, t]) for li in key_limbs], mods)[0] for t in range(N)]
            prod = R.negacyclic(dj, ev, N)
            U = [u + p for u, p in zip(U, prod)]
        M = 1
        for m in mods:
            M *= m
        for t in range(N):
            v = R.round_div(U[t] % M, ck.special)
            for i in range(nl):
                out[c, i, t] = v % ck.primes[i]
    return out


def test_keyswitch_bruteforce(tiny):
    rng = np.random.default_rng(13)
    key = tiny.rotation_key(1)
    h = tiny.load_key(key)
    for nl in [3, 2]:
        d = np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes[:nl]])
        assert np.array_equal(tiny.keyswitch(d, h), _ks_bruteforce(tiny, d, key, nl))


def test_rescale_bruteforce(tiny):
    rng = np.random.default_rng(14)
    from oracle.ckks import Ciphertext
    for nl in [3, 2]:
        data = np.stack([np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes[:nl]])
                         for _ in range(2)])
        out = tiny.rescale(Ciphertext(data, 1.0)).data
        ql = tiny.primes[nl - 1]
        for c in range(2):
            for t in range(tiny.n):
                x, _ = R.crt([int(data[c, i, t]) for i in range(nl)], tiny.primes[:nl])
                v = R.round_div(x, ql)
                for i in range(nl - 1):
                    assert int(out[c, i, t]) == v % tiny.primes[i]


def test_keyswitch_noise_bound(mid):
    """KS(d) decrypts to d * t plus an error below N sum_j (q_j/2) 19 / P + N."""
    rng = np.random.default_rng(15)
    r = 5
    key = mid.load_key(mid.rotation_key(r))
    nl = len(mid.primes)
    d = np.stack([rng.integers(0, q, mid.n, dtype=np.uint64) for q in mid.primes])
    ks = mid.keyswitch(d, key)
    from oracle.ckks import Ciphertext
    m = mid.decrypt_residues(Ciphertext(ks, 1.0))
    # expected d * tau_g(s), limb by limb
    g = mid.galois_elt(r)
    s = [int(x) for x in mid.sk.s]
    ts = R.substitute(s, g, mid.n, 1 << 80)
    ts = [x - (1 << 80) if x > (1 << 79) else x for x in ts]
    bound = mid.n * sum(q / 2 for q in mid.primes) * 19 / mid.special + mid.n
    worst = 0
    for i in range(1):  # limb 0 only: q_0 is 60-bit and holds the error
        q = mid.primes[i]
        exp = R.negacyclic([int(x) for x in d[i]], ts, mid.n, q)
        err = max(abs(R.centered(int(a) - b, q)) for a, b in zip(m[i], exp))
        worst = max(worst, err)
    assert worst <= bound


def test_rotation_decrypts_to_left_roll(mid):
    z = W.gen_slots(mid.slots, 1, seed=16)[0]
    ct = mid.encrypt(z, 17)
    for r in [1, 5, -3, mid.slots // 4]:
        k = mid.load_key(mid.rotation_key(r))
        out = mid.decrypt(mid.rotate(ct, r, k))
        assert np.abs(out - np.roll(z, -r)).max() < 1e-6


def test_hoisted_equals_plain(mid):
    z = W.gen_slots(mid.slots, 1, seed=18)[0]
    ct = mid.limb_drop(mid.encrypt(z, 19), 3)
    rs = [1, 28, -4, 100]
    keys = [mid.load_key(mid.rotation_key(r)) for r in rs]
    hs = mid.rotate_hoisted(ct, rs, keys)
    for r, k, h in zip(rs, keys, hs):
        assert np.array_equal(h.data, mid.rotate(ct, r, k).data)


def test_square_relin_rescale(mid):
    z = W.gen_slots(mid.slots, 1, seed=20)[0]
    ct = mid.encrypt(z, 21)
    rlk = mid.load_key(mid.relin_key())
    sq = mid.rescale(mid.square_relin(ct, rlk))
    assert sq.nl == len(mid.primes) - 1
    assert np.abs(mid.decrypt(sq) - z * z).max() < 1e-6


def test_mul_relin(mid):
    """Mul(C): equals the square when both operands are the same ciphertext
    (bit for bit), is symmetric (bit for bit), and decrypts to the slotwise
    product."""
    z1 = W.gen_slots(mid.slots, 1, seed=23)[0]
    z2 = W.gen_slots(mid.slots, 1, seed=24)[0]
    a, b = mid.encrypt(z1, 25), mid.encrypt(z2, 26)
    rlk = mid.load_key(mid.relin_key())
    assert np.array_equal(mid.mul_relin(a, a, rlk).data, mid.square_relin(a, rlk).data)
    ab, ba = mid.mul_relin(a, b, rlk), mid.mul_relin(b, a, rlk)
    assert np.array_equal(ab.data, ba.data)
    r = mid.rescale(ab)
    assert np.abs(mid.decrypt(r) - z1 * z2).max() < 1e-6


def test_mul_relin_tensor_bruteforce(tiny):
    """The tensor part, checked with schoolbook negacyclic products: with a
    zero relinearisation contribution (c1 parts zero) the product is
    (a0 b0, a0 b1 + a1 b0) exactly."""
    rng = np.random.default_rng(27)
    nl = len(tiny.primes)
    a = np.stack([np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes]),
                  np.zeros((nl, tiny.n), dtype=np.uint64)])
    b = np.stack([np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes]) for _ in range(2)])
    from oracle.ckks import Ciphertext
    rlk = tiny.load_key(tiny.relin_key())
    out = tiny.mul_relin(Ciphertext(a, 1.0), Ciphertext(b, 1.0), rlk)
    for i, q in enumerate(tiny.primes):
        a0 = [int(x) for x in a[0, i]]
        e0 = R.negacyclic(a0, [int(x) for x in b[0, i]], tiny.n, q)
        e1 = R.negacyclic(a0, [int(x) for x in b[1, i]], tiny.n, q)
        assert [int(x) for x in out.data[0, i]] == e0
        assert [int(x) for x in out.data[1, i]] == e1


def test_mac_schoolbook(tiny):
    rng = np.random.default_rng(22)
    nl = 2
    from oracle.ckks import Ciphertext
    cts = [Ciphertext(np.stack([np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes[:nl]])
                                for _ in range(2)]), 1.0) for _ in range(3)]
    pts = [[np.stack([rng.integers(0, q, tiny.n, dtype=np.uint64) for q in tiny.primes[:nl]]) for _ in range(3)]
           for _ in range(2)]
    pts[1][2] = None
    accs = tiny.mac_matrix(cts, pts)
    for o in range(2):
        for c in range(2):
            for i, q in enumerate(tiny.primes[:nl]):
                exp = [0] * tiny.n
                for t in range(3):
                    if pts[o][t] is None:
                        continue
                    p = R.negacyclic([int(x) for x in pts[o][t][i]], [int(x) for x in cts[t].data[c, i]], tiny.n, q)
                    exp = [(a + b) % q for a, b in zip(exp, p)]
                assert [int(x) for x in accs[o][c, i]] == exp


# ---------------------------------------------------------------- paper facts
def test_paper_facts():
    facts = json.load(open(os.path.join(GOLD, "paper_facts.json")))
    from oracle.network import network_depth, Net, SlotEval
    # Table of M2 (LeNet-1): per-layer #Mult and total 7
    cfg = W.config("lenet1")
    per = facts["lenet1_mults"]
    layers = cfg["layers"]
    acc = 0
    for i, lay in enumerate(layers):
        d = network_depth(cfg["input"], layers[: i + 1])
        assert d - acc == per[i]["mult"], (i, lay)
        acc = d
    assert acc == facts["lenet1_total_mults"]
    # Tables of M1 and M3 to M7: per-layer #Mult and totals
    for name, rows in facts["model_mults"].items():
        cfg = W.config(name)
        layers = cfg["layers"]
        assert len(layers) == len(rows), name
        acc = 0
        for i in range(len(layers)):
            d = network_depth(cfg["input"], layers[: i + 1])
            assert d - acc == rows[i]["mult"], (name, i, rows[i]["layer"])
            acc = d
        assert acc == facts["model_total_mults"][name]
    assert tuple(facts["approx_relu"][k] for k in ("c0", "c1", "c2")) == __import__("oracle.network").network.RELU_APPROX
    # FC 64 -> 10: the first loop of Algorithm 2 runs DAT_out = 10 times, not 64
    fc = facts["fc_64_10"]
    ev = SlotEval(4096)
    inp = {"c": 1, "h": 1, "w": fc["din"], "dist": "normal"}
    lays = [W.FLATTEN, {"kind": "fc", "din": fc["din"], "dout": fc["dout"]}]
    net = Net(inp, lays, W.gen_params(lays), 4096)
    net.run(ev, [np.zeros(4096)])
    D = fc["dout"]
    assert ev.count.mac == 2 * D - 1            # the loop body's two products, V2 empty at o = 0
    assert ev.count.mac // 2 + 1 == fc["loop_iterations"]
    # packing example: input i is shifted right by (i - 1) * 800 slots
    ex = facts["packing_800"]
    inp = {"c": 1, "h": 1, "w": 784, "dist": "uniform01"}
    net = Net(inp, [], [], 8192, samples=3, stride=ex["stride"])
    v = net.input_vector(np.ones((3, 1, 1, 784)))
    for i in range(1, 4):
        assert v[(i - 1) * ex["stride"]] == 1.0 and v[(i - 1) * ex["stride"] + 784] == 0.0


def test_drop_level_by_encrypted_ones(mid):
    """Drop-Level as Section IV-A writes it: two products with encryptions of
    all-ones vectors take a 4-limb ciphertext to 2 limbs; with the ones at
    scale q_l (the prime each rescale divides by) the scale is unchanged
    exactly, and the slots decrypt to the input's."""
    z = W.gen_slots(mid.slots, 1, seed=61)[0]
    ct = mid.encrypt(z, 62)
    rlk = mid.load_key(mid.relin_key())
    ones = []
    for k in range(2):
        q = float(mid.primes[ct.nl - 1 - k])
        ones.append(mid.encrypt_pt(mid.encode(np.ones(mid.slots), q, mid.n_data), 63 + k, q))
    out = mid.drop_level(ct, ones, rlk)
    assert out.nl == ct.nl - 2
    assert out.scale == ct.scale
    assert np.abs(mid.decrypt(out) - z).max() < 1e-6


# ---------------------------------------------------------------- samplers
# The client's samplers (ternary secret, rounded Gaussian errors of sigma 3.2
# redrawn past |e| = 19, uniform residues) pinned by their distributions.
def _draws(kind: int, n: int, seed: int, q: int = 0) -> np.ndarray:
    import ctypes
    from oracle.ckks import lib
    L = lib()
    p = L.or_prng_new(seed)
    out = np.zeros(n, dtype=np.int64)
    L.or_sample(p, kind, q, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    L.or_prng_free(p)
    return out


def test_sampler_ternary_is_uniform_on_three_values():
    n = 300_000
    x = _draws(0, n, 7)
    vals, counts = np.unique(x, return_counts=True)
    assert vals.tolist() == [-1, 0, 1]
    # each frequency within 6 standard errors (sqrt(2/9 / n) = 0.00086) of 1/3
    assert np.all(np.abs(counts / n - 1 / 3) < 0.0052), counts


def test_sampler_gauss_sigma_shape_and_bound():
    from scipy.stats import chi2, norm
    n = 1_000_000
    x = _draws(1, n, 8)
    assert np.abs(x).max() <= 19
    # rounding a N(0, 3.2^2) variable adds 1/12 to its variance
    sd = np.sqrt(3.2 ** 2 + 1 / 12)
    assert abs(x.mean()) < 6 * sd / np.sqrt(n)
    assert abs(x.std() - sd) < 6 * sd / np.sqrt(2 * n)
    # probability of each value against the rounded normal law (tails merged)
    ks = np.arange(-10, 11)
    exp = norm.cdf((ks + 0.5) / 3.2) - norm.cdf((ks - 0.5) / 3.2)
    obs = np.array([(x == k).sum() for k in ks], dtype=np.float64)
    tail_exp = 1.0 - exp.sum()
    tail_obs = n - obs.sum()
    stat = ((obs - n * exp) ** 2 / (n * exp)).sum() + (tail_obs - n * tail_exp) ** 2 / (n * tail_exp)
    assert chi2.sf(stat, len(ks)) > 1e-6, stat


def test_sampler_gauss_redraw_boundary():
    """With u2 = 0 (cos = 1) or u2 = 1/2 (cos = -1) the candidate is
    +-3.2 sqrt(-2 ln u1): 19.4 rounds to 19 and is kept, 19.6 rounds to 20
    and is redrawn, on both sides."""
    import ctypes
    from oracle.ckks import lib
    L = lib()
    e = ctypes.c_int(0)
    for u2, sign in ((0.0, 1), (0.5, -1)):
        for target, keep in ((19.4, True), (19.6, False), (3.0, True)):
            u1 = float(np.exp(-((target / 3.2) ** 2) / 2))
            ok = L.or_gauss_candidate(u1, u2, ctypes.byref(e))
            assert bool(ok) == keep, (u2, target)
            if keep:
                assert e.value == sign * int(round(target))


def test_sampler_uniform_range_and_spread():
    q = 1099510054913                       # a 40-bit prime of the chain
    n = 200_000
    x = _draws(2, n, 9, q).astype(np.uint64)
    assert int(x.min()) >= 0 and int(x.max()) < q
    u = x.astype(np.float64) / q
    assert abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / n)
    counts = np.histogram(u, bins=16, range=(0, 1))[0]
    assert np.all(np.abs(counts / n - 1 / 16) < 6 * np.sqrt(15 / 256 / n)), counts


def test_seeded_keys_partial_rows_equal_whole_key(mid):
    """Keys from their own seeded generator: the rows formed for `levels`
    limbs equal the whole key's rows, the others are zero, and a rotation
    (and a relinearised square) at that many limbs gives the same
    ciphertext with either key, which decrypts to the rolled slots."""
    nd = mid.n_data
    lv = 2
    for r in (3, None):
        whole = mid.seeded_key(1234, r=r)
        part = mid.seeded_key(1234, r=r, levels=lv)
        assert not np.array_equal(whole, mid.seeded_key(1235, r=r))
        for d in range(nd):
            for i in range(nd + 1):
                used = d < lv and (i < lv or i == nd)
                if used:
                    assert np.array_equal(part[d, :, i], whole[d, :, i]), (d, i)
                else:
                    assert not part[d, :, i].any(), (d, i)
    z = W.gen_slots(mid.slots, 1, seed=21)[0]
    ct = mid.limb_drop(mid.encrypt(z, 22), lv)
    kw, kp = mid.load_key(mid.seeded_key(77, r=3)), mid.load_key(mid.seeded_key(77, r=3, levels=lv))
    a, b = mid.rotate(ct, 3, kw), mid.rotate(ct, 3, kp)
    assert np.array_equal(a.data, b.data)
    assert np.abs(mid.decrypt(a) - np.roll(z, -3)).max() < 1e-6
    rw, rp = mid.load_key(mid.seeded_key(78)), mid.load_key(mid.seeded_key(78, levels=lv))
    assert np.array_equal(mid.square_relin(ct, rw).data, mid.square_relin(ct, rp).data)
