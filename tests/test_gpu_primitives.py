"""GPU parity of the CKKS primitives against the CPU oracle: every output is
compared in coefficient form, residue by residue (bit-exact)."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import gpu_ctx_for, ocat, oracle_ring, random_ct

pytestmark = pytest.mark.gpu

RINGS = {
    "n16": W.TINY_RINGS["n16"],
    "n1024": W.TINY_RINGS["n1024"],
    "n8192": {"log_n": 13, "prime_bits": [60, 40, 40], "special_bits": 60, "log_scale": 40},
}


@pytest.fixture(scope="module", params=list(RINGS))
def pair(request):
    ring = RINGS[request.param]
    ck = oracle_ring(ring)
    ctx = gpu_ctx_for(ck, ring)
    return ck, ctx, ring


@pytest.mark.parametrize("log_n", [4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16])
def test_ntt_roundtrip_all_sizes(log_n):
    import torch
    from paper_2402_03060_amd import Context, device_u64, host_u64
    bits = [60, 40, 40]
    ctx = Context(log_n, bits, 60, 2.0 ** 40)
    rng = np.random.default_rng(log_n)
    a = np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes]) for _ in range(3)])
    t = device_u64(a)
    ctx.to_ntt(t, 3, 3)
    ntt = host_u64(t.clone())
    ctx.from_ntt(t, 3, 3)
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(t), a)
    for i, q in enumerate(ctx.primes):
        assert int(ntt[:, i].max()) < q  # canonical residues


@pytest.mark.parametrize("log_n", [11, 13, 14, 15])
def test_ntt_every_tuning_setting_identical(log_n):
    """Every NTT split / tile the tuner can choose gives the same forward
    transform as the default one, and inverts exactly."""
    import torch
    from paper_2402_03060_amd import Context, device_u64, host_u64
    ctx = Context(log_n, [60, 40, 40], 60, 2.0 ** 40)
    rng = np.random.default_rng(1000 + log_n)
    a = np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes]) for _ in range(5)])
    t = device_u64(a)
    ctx.to_ntt(t, 3, 5)
    ref = host_u64(t)
    default = ctx.tuning()
    tried = 0
    for l1 in range(3, log_n - 2):
        if l1 > 8 or log_n - l1 > 8:
            continue
        for tile in (11, 12):
            ctx.set_tuning(ntt_split=l1, ntt_tile_log=tile)
            t = device_u64(a)
            ctx.to_ntt(t, 3, 5)
            assert np.array_equal(host_u64(t), ref), (l1, tile)
            ctx.from_ntt(t, 3, 5)
            torch.cuda.synchronize()
            assert np.array_equal(host_u64(t), a), (l1, tile)
            tried += 1
    assert tried >= 4
    ctx.set_tuning(ntt_split=default["ntt_split"], ntt_tile_log=default["ntt_tile_log"])
    info = ctx.autotune(batch=2)
    assert 3 <= info["ntt_split"] <= 8 and info["ntt_tile_log"] in (11, 12) and info["ntt_ms"] > 0
    t = device_u64(a)
    ctx.to_ntt(t, 3, 5)
    assert np.array_equal(host_u64(t), ref)


def test_mac_parity(pair):
    ck, ctx, _ = pair
    nl = len(ck.primes)
    cts = [random_ct(ck, nl, 100 + t)[0] for t in range(3)]
    pts = [np.stack([np.random.default_rng(200 + t).integers(0, q, ck.n, dtype=np.uint64) for q in ck.primes])
           for t in range(3)]
    exp = ck.mac_matrix([ocat(c) for c in cts], [pts])[0]
    g = ctx.mul_plain_acc([ctx.import_ct(c, 1.0) for c in cts], [ctx.import_pt(p) for p in pts])
    assert np.array_equal(ctx.export_ct(g)[0], exp)


@pytest.mark.parametrize("steps", [1, 3, -2, 5])
def test_rotate_parity(pair, steps):
    ck, ctx, _ = pair
    z = W.gen_slots(ck.slots, 1, seed=31)[0]
    ct = ck.encrypt(z, 32)
    key = ck.rotation_key(steps)
    hk = ck.load_key(key)
    gkey = ctx.import_evk(key)
    for nl in sorted({len(ck.primes), 2}):
        oct_ = ck.limb_drop(ct, nl)
        exp = ck.rotate(oct_, steps, hk)
        ws = ctx.workspace(nl, 1)
        got = ctx.rotate(ctx.import_ct(oct_.data, oct_.scale), steps, gkey, ws)
        assert np.array_equal(ctx.export_ct(got)[0], exp.data)


def test_rotate_hoisted_parity(pair):
    ck, ctx, _ = pair
    z = W.gen_slots(ck.slots, 1, seed=33)[0]
    ct = ck.encrypt(z, 34)
    rs = [1, 2, -1, 0]
    keys = {r: ck.rotation_key(r) for r in rs if r}
    gct = ctx.import_ct(ct.data, ct.scale)
    ws = ctx.workspace(len(ck.primes), 1)
    outs = ctx.rotate_hoisted(gct, rs, [ctx.import_evk(keys[r]) if r else None for r in rs], ws)
    for r, o in zip(rs, outs):
        exp = ck.rotate(ct, r, ck.load_key(keys[r])).data if r else ct.data
        assert np.array_equal(ctx.export_ct(o)[0], exp)


def test_rescale_parity(pair):
    ck, ctx, _ = pair
    nl = len(ck.primes)
    a = random_ct(ck, nl, 41, batch=2)
    ws = ctx.workspace(nl, 2)
    got = ctx.export_ct(ctx.rescale(ctx.import_ct(a, 1.0), ws))
    for b in range(2):
        assert np.array_equal(got[b], ck.rescale(ocat(a[b])).data)


def test_square_relin_parity(pair):
    ck, ctx, _ = pair
    z = W.gen_slots(ck.slots, 1, seed=35)[0]
    ct = ck.encrypt(z, 36)
    rk = ck.relin_key()
    exp = ck.square_relin(ct, ck.load_key(rk))
    ws = ctx.workspace(len(ck.primes), 1)
    got = ctx.square_relin(ctx.import_ct(ct.data, ct.scale), ctx.import_evk(rk), ws)
    assert np.array_equal(ctx.export_ct(got)[0], exp.data)
    assert got.scale == exp.scale


def test_mul_relin_parity(pair):
    """Mul(C) + relinearisation of two ciphertexts, with the second operand
    also one level above the first (its top limb ignored)."""
    ck, ctx, _ = pair
    nl = len(ck.primes)
    za, zb = W.gen_slots(ck.slots, 2, seed=37)
    a, b = ck.encrypt(za, 38), ck.encrypt(zb, 39)
    rk = ck.relin_key()
    rlk = ck.load_key(rk)
    g_rlk = ctx.import_evk(rk)
    ws = ctx.workspace(nl, 1)
    exp = ck.mul_relin(a, b, rlk)
    got = ctx.mul_relin(ctx.import_ct(a.data, a.scale), ctx.import_ct(b.data, b.scale), g_rlk, ws)
    assert np.array_equal(ctx.export_ct(got)[0], exp.data)
    assert got.scale == exp.scale
    if nl > 1:
        a2 = ck.limb_drop(a, nl - 1)
        exp2 = ck.mul_relin(a2, ck.limb_drop(b, nl - 1), rlk)
        got2 = ctx.mul_relin(ctx.import_ct(a2.data, a2.scale), ctx.import_ct(b.data, b.scale), g_rlk, ws)
        assert np.array_equal(ctx.export_ct(got2)[0], exp2.data)


def test_add_and_add_plain_parity(pair):
    ck, ctx, _ = pair
    nl = len(ck.primes)
    a, b = random_ct(ck, nl, 51)[0], random_ct(ck, nl, 52)[0]
    got = ctx.export_ct(ctx.add(ctx.import_ct(a, 1.0), ctx.import_ct(b, 1.0)))[0]
    assert np.array_equal(got, ck.add(ocat(a), ocat(b)).data)
    pt = np.stack([np.random.default_rng(53).integers(0, q, ck.n, dtype=np.uint64) for q in ck.primes])
    got = ctx.export_ct(ctx.add_plain(ctx.import_ct(a, 1.0), ctx.import_pt(pt, mont=False)))[0]
    assert np.array_equal(got, ck.add_plain(ocat(a), pt).data)


@pytest.mark.parametrize("kind", ["dense", "mask", "bias_scale"])
def test_encode_parity(pair, kind):
    ck, ctx, _ = pair
    nl = len(ck.primes)
    rng = np.random.default_rng(61)
    if kind == "dense":
        z, scale = rng.uniform(-1, 1, ck.slots), ck.delta
    elif kind == "mask":
        z = np.zeros(ck.slots)
        z[rng.choice(ck.slots, size=max(1, ck.slots // 7), replace=False)] = rng.normal(0, 0.1)
        scale = ck.delta
    else:
        z = np.zeros(ck.slots)
        z[: max(1, ck.slots // 3)] = rng.normal(0, 0.01)
        scale = ck.delta * 1.0000013283  # a non-power-of-two scale, as after a rescale
    exp = ck.encode(z, scale, nl)
    for mont in (False, True):
        got = ctx.export_pt(ctx.encode(z, scale, nl, mont=mont), mont=mont)
        assert np.array_equal(got, exp)


def test_mod_drop(pair):
    ck, ctx, _ = pair
    nl = len(ck.primes)
    a = random_ct(ck, nl, 71, batch=2)
    got = ctx.export_ct(ctx.mod_drop(ctx.import_ct(a, 1.0), 1))
    assert np.array_equal(got, a[:, :, :1, :])


def test_drop_level_parity(pair):
    """Drop-Level by encrypted all-ones vectors (Section IV-A as written):
    every limb count it can drop, bit for bit against the oracle's products
    and rescales; ones at scale q_l keep the scale exactly."""
    ck, ctx, _ = pair
    nl = len(ck.primes)
    z = W.gen_slots(ck.slots, 1, seed=71)[0]
    ct = ck.encrypt(z, 72)
    rk = ck.relin_key()
    rlk, g_rlk = ck.load_key(rk), ctx.import_evk(rk)
    ones = []
    for k in range(nl - 1):
        q = float(ck.primes[nl - 1 - k])
        ones.append(ck.encrypt_pt(ck.encode(np.ones(ck.slots), q, nl), 73 + k, q))
    g_in = ctx.import_ct(ct.data, ct.scale)
    g_ones = [ctx.import_ct(o.data, o.scale) for o in ones]
    for n in range(1, nl):
        exp = ck.drop_level(ct, ones[:n], rlk)
        got = ctx.drop_level(g_in, g_ones[:n], g_rlk)
        assert np.array_equal(ctx.export_ct(got)[0], exp.data), n
        assert got.n_limbs == nl - n and got.scale == exp.scale == ct.scale


def test_largest_ring_rotation():
    """The largest ring the library takes (N = 2^16, three primes), where the
    oracle is too slow for a test: the product client's keys and ciphertext,
    and rotations by 1 and by N/4 - 1 slots decrypting to the rolled slots
    (a property that holds at any size)."""
    import paper_2402_03060_amd as P
    ctx = P.Context(16, [60, 40, 40], 60, 2.0 ** 40)
    sk = P.keygen_secret(ctx, 93)
    z = np.random.default_rng(94).uniform(-1, 1, ctx.slots)
    ct = P.encrypt_sk(ctx, sk, ctx.encode(z, ctx.scale, 3, mont=False)[None], 95, ctx.scale)
    ws = ctx.workspace(3, 1)
    probe = np.arange(0, ctx.slots, 997, dtype=np.uint32)
    for r in (1, ctx.slots // 2 - 1):
        key = P.gen_switch_key(ctx, sk, 96, steps=r)
        got = P.decrypt_slots(ctx, sk, ctx.rotate(ct, r, key, ws), probe)[0]
        assert np.abs(got - np.roll(z, -r)[probe]).max() < 1e-6, r


def test_import_export_ct_entry_points(pair):
    """unihenn_import_ct / unihenn_export_ct: from host and device memory,
    out of place and in place, equal the in-place transforms and invert each
    other; bad descriptors are EINVAL with the destination untouched."""
    import ctypes as C
    import torch
    import paper_2402_03060_amd as P
    from paper_2402_03060_amd import device_u64, host_u64
    ck, ctx, ring = pair
    rng = np.random.default_rng(321)
    nl = len(ctx.primes) - 1
    a = np.stack([np.stack([np.stack([rng.integers(0, q, ctx.n, dtype=np.uint64) for q in ctx.primes[:nl]])
                            for _ in range(2)]) for _ in range(3)])
    ref = device_u64(a)
    ctx.to_ntt(ref, nl, 6)
    ct = ctx.import_ct(a, 1.0)                       # host source, out of place
    assert torch.equal(ct.data, ref)
    dev = device_u64(a)
    ct2 = P.Ciphertext(torch.empty_like(dev), 1.0)
    d2 = ct2.desc()
    P._check(P.lib().unihenn_import_ct(ctx.h, dev.data_ptr(), C.byref(d2), P._stream()))   # device source
    d3 = P.Ciphertext(dev, 1.0).desc()
    P._check(P.lib().unihenn_import_ct(ctx.h, dev.data_ptr(), C.byref(d3), P._stream()))   # in place
    torch.cuda.synchronize()
    assert torch.equal(ct2.data, ref) and torch.equal(dev, ref)
    assert np.array_equal(ctx.export_ct(ct), a)
    P._check(P.lib().unihenn_export_ct(ctx.h, C.byref(d3), dev.data_ptr(), P._stream()))  # in place
    torch.cuda.synchronize()
    assert np.array_equal(host_u64(dev), a)
    bad = P.Ciphertext(torch.full_like(dev, 7), 1.0)
    db = bad.desc()
    db.n_limbs = len(ctx.primes) + 3
    assert P.lib().unihenn_import_ct(ctx.h, ref.data_ptr(), C.byref(db), P._stream()) == P.EINVAL
    db = bad.desc()
    db.batch = 0
    assert P.lib().unihenn_export_ct(ctx.h, C.byref(db), ref.data_ptr(), P._stream()) == P.EINVAL
    torch.cuda.synchronize()
    assert bool((bad.data == 7).all())


def test_workspace_size_entry_point():
    import ctypes as C
    import workloads as W
    import paper_2402_03060_amd as P
    cfg = W.config("conv1")
    cfg["log_n"] = 11
    ctx = P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])
    net = P.Net(ctx, cfg["input"], cfg["layers"], W.gen_params(cfg["layers"]), max_batch=3)
    w = net.workspace_size()
    assert w > 0 and w == net.workspace_size(1)
    fixed, per_slot = net.memory()
    assert per_slot * 3 >= w                          # the slots' shares cover the workspace
    b = C.c_size_t(0)
    assert P.lib().unihenn_workspace_size(ctx.h, net.h, 4, C.byref(b)) == P.EINVAL
    assert P.lib().unihenn_workspace_size(ctx.h, net.h, 0, C.byref(b)) == P.EINVAL
