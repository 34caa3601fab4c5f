"""GPU network parity: whole networks and single conv layers evaluated by the
HIP library on keys and ciphertexts made by the CPU oracle (client role),
compared with the oracle's evaluation residue by residue; and the product's
own client end to end against the FP64 CNN."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle.network import input_layout, read_outputs
from oracle.run import OracleSession, build_net, decrypt_outputs, reference_outputs, run_encrypted

pytestmark = pytest.mark.gpu


def _gpu_net(P, ctx, cfg, sess, net_oracle, batch=1, lazy=False):
    net = P.Net(ctx, cfg["input"], cfg["layers"], net_oracle.params, samples=cfg["samples_per_ct"],
                stride=cfg["sample_stride"], max_batch=batch, lazy=lazy, fc_doubling=net_oracle.fc_doubling)
    assert net.depth == net_oracle.depth
    assert sorted(net.rotations()) == net_oracle.rotation_set()
    keys = {r: ctx.import_evk(sess.key_coeff[r]) for r in net.rotations()}
    rlk = ctx.import_evk(sess.rlk_coeff)
    net.bind_keys(keys, rlk)
    return net


def _ctx(P, cfg):
    return P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])


def _run_parity(cfg, n_cts=1, seeds=(W.SEED_ENCRYPT,), lazy=False, modes=None, fc_doubling=False):
    """GPU outputs equal to the oracle's, residue by residue, in every mode
    (default: plain and hoisted); lazy: both sides plan deferred ModDown;
    fc_doubling: both sides sum the FC's rotated copies by doubling."""
    import paper_2402_03060_amd as P
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots, fc_doubling=fc_doubling)
    xs_all = W.gen_inputs(cfg["input"], cfg["samples_per_ct"] * n_cts)
    expected, cts = [], []
    for b in range(n_cts):
        xs = xs_all[b * cfg["samples_per_ct"]:(b + 1) * cfg["samples_per_ct"]]
        ct, outs, _ = run_encrypted(sess, onet, xs, enc_seed=seeds[b % len(seeds)] + b, lazy=lazy)
        expected.append([o.data for o in outs])
        cts.append(ct)
    ctx = _ctx(P, cfg)
    assert ctx.primes == sess.ck.primes
    gnet = _gpu_net(P, ctx, cfg, sess, onet, batch=n_cts, lazy=lazy)
    gin = ctx.import_ct(np.stack([c.data for c in cts]), cts[0].scale)
    results = {}
    for mode in (modes or (P.EVAL_PLAIN, P.EVAL_HOISTED)):
        gnet.set_mode(mode)
        outs = gnet.eval(gin)
        got = [ctx.export_ct(o) for o in outs]
        for b in range(n_cts):
            for k in range(len(outs)):
                assert np.array_equal(got[k][b], expected[b][k]), (mode, b, k)
        results[mode] = got
    return sess, onet, gnet, ctx, xs_all


def test_conv1_config_bit_exact():
    """One conv layer (4 filters 5x5) + square at N = 2^13: the full-size
    single-layer workload."""
    _run_parity(W.config("conv1"))


def test_lenet1_small_ring_bit_exact():
    """Every layer kind (conv, square, pool, flatten after pooling, FC) at N = 2^11."""
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    _run_parity(cfg)


@pytest.mark.parametrize("n_cts", [2, 5])
def test_lenet1_packed_batch_bit_exact(n_cts):
    """Two images per ciphertext at stride 784 and several ciphertexts per
    launch (5: a full batch chunk of 4 plus a ragged one)."""
    cfg = W.config("lenet1_batched")
    cfg["log_n"] = 12
    cfg["samples_per_ct"] = 2
    _run_parity(cfg, n_cts=n_cts)


def test_cnn1d_small_ring_bit_exact():
    """1D convolutions with stride 2 and the row-interval flatten at N = 2^12,
    two sequences at stride 1024."""
    cfg = W.config("cnn1d")
    cfg["log_n"] = 12
    cfg["samples_per_ct"] = 2
    _run_parity(cfg)


@pytest.mark.parametrize("name,log_n", [("m3", 12), ("m1", 11), ("m6", 11), ("m7", 11), ("m4", 11),
                                        ("lenet1_padded", 11)])
def test_paper_model_shapes_bit_exact(name, log_n):
    """The paper's other model shapes on small rings: approximate ReLU with
    Mul(C) (M3), stride-3 and stride-2 convolutions with FC -> square -> FC
    (M1, M6), 1D convolutions of stride 2 (M7), LeNet-5 with its 16 -> 120
    convolution and a flatten of 1 x 1 maps (M4)."""
    cfg = W.config(name)
    cfg["log_n"] = log_n
    _run_parity(cfg)


def test_conv_layer_entry_point():
    """unihenn_conv (Algorithm 1 alone) on the LeNet-1 second conv at N = 2^11."""
    import paper_2402_03060_amd as P
    from oracle.network import CkksEval, Layout
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots)
    sess.ensure_keys(onet.rotation_set())
    ck = sess.ck
    ev = CkksEval(ck, sess.key_handle, sess.rlk)
    # four input channels at the level and scale conv2 sees in the network
    xs = W.gen_slots(ck.slots, 4, seed=81, lo=0, hi=0.5)
    nl = onet.depth + 1 - 2
    cts = [ck.limb_drop(ck.encrypt(x, 90 + i), nl) for i, x in enumerate(xs)]
    ctx = _ctx(P, cfg)
    gnet = _gpu_net(P, ctx, cfg, sess, onet)
    # the plan's scale for conv2's input: conv1 (MAC, rescale), square (rescale), pool
    s = ck.delta * ck.delta / ck.primes[nl + 1]
    s = s * s / ck.primes[nl]
    cts = [type(c)(c.data, s) for c in cts]
    L = Layout("map", 4, 12, 12, 2, 28, [0, 1, 2, 3], [0, 0, 0, 0], "avgpool", 0.25)
    exp, L2 = onet._conv(ev, cts, L, cfg["layers"][3], onet.params[3])
    gins = [ctx.import_ct(c.data, s) for c in cts]
    outs, interval = gnet.conv(3, gins, 12, nl - 1)
    assert interval == L2.I == 2
    for o in range(12):
        assert np.array_equal(ctx.export_ct(outs[o])[0], exp[o].data)


def test_full_size_rotation_lenet1_ring():
    """One rotation and one rescale at the LeNet-1 size (N = 2^14, 8 limbs),
    launch configuration of the benchmark."""
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    sess = OracleSession(cfg)
    ck = sess.ck
    z = W.gen_slots(ck.slots, 1, seed=91)[0]
    ct = ck.encrypt(z, 92)
    key = ck.rotation_key(28)
    exp = ck.rotate(ct, 28, ck.load_key(key))
    ctx = _ctx(P, cfg)
    ws = ctx.workspace(8, 1)
    g = ctx.rotate(ctx.import_ct(ct.data, ct.scale), 28, ctx.import_evk(key), ws)
    assert np.array_equal(ctx.export_ct(g)[0], exp.data)
    r = ctx.rescale(g, ws)
    assert np.array_equal(ctx.export_ct(r)[0], ck.rescale(exp).data)


@pytest.mark.parametrize("name", ["conv1", "lenet1", "cnn1d", "cifar_cnn"])
def test_product_client_end_to_end(name):
    """The library's own client (GPU keygen, encryption, decryption) around
    the full-size network: outputs within 1e-3 of the FP64 CNN."""
    import paper_2402_03060_amd as P
    cfg = W.config(name)
    ctx = _ctx(P, cfg)
    params = W.gen_params(cfg["layers"])
    S = cfg["samples_per_ct"]
    B = 2
    net = P.Net(ctx, cfg["input"], cfg["layers"], params, samples=S, stride=cfg["sample_stride"], max_batch=B)
    sk = P.keygen_secret(ctx, 5)
    keys = {r: P.gen_switch_key(ctx, sk, 6, steps=r) for r in net.rotations()}
    rlk = P.gen_switch_key(ctx, sk, 7, relin=True)
    net.bind_keys(keys, rlk)
    xs = W.gen_inputs(cfg["input"], S * B)
    from oracle.network import Net as ONet
    onet = ONet(cfg["input"], cfg["layers"], params, ctx.slots, S, cfg["sample_stride"])
    pts = []
    for b in range(B):
        v = onet.input_vector(xs[b * S:(b + 1) * S])
        pts.append(ctx.encode(v, ctx.scale, net.in_limbs, mont=False))
    import torch
    ct = P.encrypt_sk(ctx, sk, torch.stack(pts), 8, ctx.scale)
    net.set_mode(P.EVAL_HOISTED)
    outs = net.eval(ct)
    pos = net.output_slots()
    ref = reference_outputs(onet, xs)
    for b in range(B):
        for s in range(S):
            ids = pos[s] >> np.uint64(32)
            slots = (pos[s] & np.uint64(0xffffffff)).astype(np.uint32)
            vals = np.zeros(len(slots))
            for k in np.unique(ids):
                sel = ids == k
                vals[sel] = P.decrypt_slots(ctx, sk, outs[int(k)], slots[sel])[b]
            assert np.abs(vals - ref[b * S + s]).max() < 1e-3


def test_graph_replay_matches_eager():
    """The captured evaluation, replayed several times with eager evaluations
    and synchronisations in between, equals the eager result every time."""
    import torch
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 2)
    cts = [run_encrypted(sess, onet, xs[b:b + 1], enc_seed=200 + b)[0] for b in range(2)]
    ctx = _ctx(P, cfg)
    net = _gpu_net(P, ctx, cfg, sess, onet, batch=2)
    gin = ctx.import_ct(np.stack([c.data for c in cts]), cts[0].scale)
    other = ctx.import_ct(np.stack([cts[1].data, cts[0].data]), cts[0].scale)
    for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED):
        net.set_mode(mode)
        eager = [ctx.export_ct(o) for o in net.eval(gin)]
        net.set_mode(mode | P.EVAL_GRAPH)
        outs = net.alloc_outputs(2)
        for rep in range(3):
            net.eval(gin, outs)
            torch.cuda.synchronize()
            got = [ctx.export_ct(o) for o in outs]
            for a, b in zip(got, eager):
                assert np.array_equal(a, b), (mode, rep)
            # eager work between replays (different buffers -> direct launches)
            net.set_mode(mode)
            swapped = [ctx.export_ct(o) for o in net.eval(other)]
            assert np.array_equal(swapped[0][0], eager[0][1])
            net.set_mode(mode | P.EVAL_GRAPH)


def test_graph_cache_several_shapes():
    """Graphs captured for two batch sizes and two output sets stay valid
    while the evaluation alternates between them."""
    import torch
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 3)
    cts = [run_encrypted(sess, onet, xs[b:b + 1], enc_seed=300 + b)[0] for b in range(3)]
    ctx = _ctx(P, cfg)
    net = _gpu_net(P, ctx, cfg, sess, onet, batch=3)
    gin3 = ctx.import_ct(np.stack([c.data for c in cts]), cts[0].scale)
    net.set_mode(P.EVAL_HOISTED)
    eager = [ctx.export_ct(o) for o in net.eval(gin3)]
    net.set_mode(P.EVAL_HOISTED | P.EVAL_GRAPH)
    staging = ctx.empty_ct(3, gin3.n_limbs, gin3.scale)
    outs_a, outs_b = net.alloc_outputs(3), net.alloc_outputs(3)
    plan = [(3, outs_a), (1, outs_a), (2, outs_b), (3, outs_a), (1, outs_b), (2, outs_b), (3, outs_b)]
    for rep, (b, outs) in enumerate(plan):
        perm = [(rep + i) % 3 for i in range(b)]
        staging.data[:b].copy_(gin3.data[perm])
        o = [P.Ciphertext(x.data[:b], 0.0) for x in outs]
        net.eval(P.Ciphertext(staging.data[:b], gin3.scale), o)
        torch.cuda.synchronize()
        got = [ctx.export_ct(x) for x in o]
        for k in range(len(got)):
            for i, src in enumerate(perm):
                assert np.array_equal(got[k][i], eager[k][src]), (rep, b, k, i)


def _digest(arrays) -> str:
    import hashlib
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype=np.uint64).tobytes())
    return h.hexdigest()


def test_lenet1_full_size_golden():
    """Full-size LeNet-1 (N = 2^14, 8 limbs, 81 rotation keys + relin) on
    oracle keys and an oracle ciphertext: the GPU outputs hash to the digest
    the oracle wrote (tests/golden/make_lenet1_golden.py), in plain graph
    replay and hoisted modes, and in plain mode under the row-fused inner
    product at the benchmark's launch shapes (groups of 32 and 64, NTT
    splits 6 and 7: large groups fused, small ones not)."""
    import json
    import os
    import paper_2402_03060_amd as P
    with open(os.path.join(os.path.dirname(__file__), "golden", "lenet1_full.json")) as f:
        rec = json.load(f)
    cfg = W.config("lenet1")
    sess = OracleSession(cfg, key_seed=rec["key_seed"])
    onet = build_net(cfg, sess.ck.slots)
    assert onet.rotation_set() == rec["rotations"]
    sess.ensure_keys(onet.rotation_set())
    assert _digest([sess.key_coeff[r] for r in sorted(sess.key_coeff)] + [sess.rlk_coeff]) == rec["keys_sha256"]
    xs = W.gen_inputs(cfg["input"], 1)
    ct = sess.ck.encrypt(onet.input_vector(xs), rec["encrypt_seed"])
    assert _digest([ct.data]) == rec["input_sha256"]
    ctx = _ctx(P, cfg)
    gnet = _gpu_net(P, ctx, cfg, sess, onet)
    gin = ctx.import_ct(ct.data, ct.scale)
    for mode in (P.EVAL_PLAIN | P.EVAL_GRAPH, P.EVAL_HOISTED):
        gnet.set_mode(mode)
        outs = gnet.eval(gin)
        assert [o.scale for o in outs] == rec["output_scales"]
        got = [ctx.export_ct(o)[0] for o in outs]
        assert [g.shape[1] for g in got] == rec["output_limbs"]
        assert _digest(got) == rec["outputs_sha256"], mode
    for group, split in ((32, 6), (32, 7), (64, 6)):
        gnet.set_tuning(ks_group=group, ks_order=2, ntt_split=split, ntt_tile_log=11)
        gnet.set_mode(P.EVAL_PLAIN | P.EVAL_GRAPH)
        got = [ctx.export_ct(o)[0] for o in gnet.eval(gin)]
        assert _digest(got) == rec["outputs_sha256"], ("row-fused", group, split)


def test_autotune_keeps_results_and_caches(tmp_path, monkeypatch):
    """The tuner's settings (group sizes, workgroup targets, NTT split and
    tile, the inner product's workgroup order including the row-fused one)
    leave the network outputs bit-identical to the oracle's; a second call
    with the same cache file applies the stored setting."""
    import json
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1_batched")
    cfg["log_n"] = 12
    cfg["samples_per_ct"] = 2
    n_cts = 3
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots)
    xs_all = W.gen_inputs(cfg["input"], cfg["samples_per_ct"] * n_cts)
    expected, cts = [], []
    for b in range(n_cts):
        ct, outs, _ = run_encrypted(sess, onet, xs_all[2 * b:2 * b + 2], enc_seed=400 + b)
        expected.append([o.data for o in outs])
        cts.append(ct)
    ctx = _ctx(P, cfg)
    net = _gpu_net(P, ctx, cfg, sess, onet, batch=n_cts)
    gin = ctx.import_ct(np.stack([c.data for c in cts]), cts[0].scale)

    def check(tag):
        for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED | P.EVAL_GRAPH):
            net.set_mode(mode)
            got = [ctx.export_ct(o) for o in net.eval(gin)]
            for b in range(n_cts):
                for k in range(len(got)):
                    assert np.array_equal(got[k][b], expected[b][k]), (tag, mode, b, k)

    for setting in ({"ks_group": 1}, {"ks_group": 2, "mac_min_wg": 512}, {"ks_min_wg": 8192, "mac_min_wg": 8192},
                    {"ntt_split": 5, "ntt_tile_log": 12}, {"ntt_split": 7, "ntt_tile_log": 11, "ks_group": 4},
                    {"ks_group": 4, "ks_order": 1}, {"ks_group": 1, "ks_order": 1, "ks_min_wg": 512},
                    {"ks_group": 4, "ks_order": 2}, {"ks_group": 1, "ks_order": 2, "ntt_split": 5, "ntt_tile_log": 12},
                    {"ks_group": 8, "ks_order": 2, "ntt_split": 4, "ntt_tile_log": 11},
                    {"ks_group": 64, "ks_order": 2}, {"ks_group": 64, "ks_order": 1}):
        net.set_tuning(**setting)
        check(setting)
    with pytest.raises(P.UnihennError):
        net.set_tuning(ks_order=3)
    # the row-fused kernel on every group, however small (by default small
    # groups stay unfused)
    monkeypatch.setenv("UNIHENN_KS_FUSE_MIN_WG", "0")
    ctx = _ctx(P, cfg)
    net = _gpu_net(P, ctx, cfg, sess, onet, batch=n_cts)
    gin = ctx.import_ct(np.stack([c.data for c in cts]), cts[0].scale)
    for setting in ({"ks_group": 4, "ks_order": 2}, {"ks_group": 1, "ks_order": 2, "ntt_split": 5, "ntt_tile_log": 12},
                    {"ks_group": 8, "ks_order": 2, "ntt_split": 4, "ntt_tile_log": 11}):
        net.set_tuning(**setting)
        check(("fused everywhere", setting))
    cache = str(tmp_path / "tuning.json")
    net.set_mode(P.EVAL_HOISTED)
    first = net.autotune(cache_path=cache)
    check("tuned")
    entries = json.load(open(cache))
    assert len(entries) == 1
    net.set_tuning(ks_group=1, mac_min_wg=512, ks_min_wg=512, ntt_split=4, ntt_tile_log=12)
    net.set_mode(P.EVAL_HOISTED)          # the cache key includes the mode
    second = net.autotune(cache_path=cache)
    for k in ("ntt_split", "ntt_tile_log", "mac_min_wg", "ks_min_wg", "ks_group", "ks_order"):
        assert second[k] == first[k], k
    now = net.tuning()
    for k in ("ntt_split", "ntt_tile_log", "mac_min_wg", "ks_min_wg", "ks_group", "ks_order"):
        assert now[k] == first[k], k
    check("cached")


def _channel_parity(cfg, inp, layers, params, lazy):
    import paper_2402_03060_amd as P
    from oracle.network import Net as ONet
    sess = OracleSession(cfg)
    onet = ONet(inp, layers, params, sess.ck.slots, channel_cts=True)
    xs = W.gen_inputs(inp, 1)
    cts, outs, _ = run_encrypted(sess, onet, xs, lazy=lazy)
    ctx = _ctx(P, cfg)
    gnet = P.Net(ctx, inp, layers, params, max_batch=1, lazy=lazy, channel_cts=True)
    assert gnet.n_inputs == inp["c"] and gnet.depth == onet.depth
    assert sorted(gnet.rotations()) == onet.rotation_set()
    keys = {r: ctx.import_evk(sess.key_coeff[r]) for r in gnet.rotations()}
    gnet.bind_keys(keys, ctx.import_evk(sess.rlk_coeff))
    gins = [ctx.import_ct(c.data[None], c.scale) for c in cts]
    for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED, P.EVAL_HOISTED | P.EVAL_GRAPH):
        gnet.set_mode(mode)
        got = [ctx.export_ct(o)[0] for o in gnet.eval(gins)]
        for g, e in zip(got, outs):
            assert np.array_equal(g, e.data), mode
    with pytest.raises(ValueError):
        gnet.eval(gins[0])


@pytest.mark.parametrize("lazy", [False, True])
def test_channel_cts_small_bit_exact(lazy):
    """A three-channel input as three ciphertexts (PLAN_CHANNEL_CTS) at
    N = 2^11, default and deferred-ModDown plans."""
    inp = {"c": 3, "h": 12, "w": 12, "dist": "uniform01"}
    layers = [{"kind": "conv", "ch_in": 3, "ch_out": 2, "k": 3, "s": 1}, W.SQUARE, {"kind": "avgpool", "c": 2},
              W.FLATTEN, {"kind": "fc", "din": 50, "dout": 4}]
    _channel_parity(dict(W.config("lenet1"), log_n=11), inp, layers, W.gen_params(layers), lazy)


def test_channel_cts_cifar_shape_where_one_ciphertext_cannot():
    """The CIFAR-shaped CNN at N = 2^12: 3 x 32 x 32 does not fit 2048 slots
    in one ciphertext, it does as three (one plane each)."""
    import paper_2402_03060_amd as P
    cfg = W.config("cifar_cnn")
    cfg["log_n"] = 12
    params = W.gen_params(cfg["layers"])
    ctx = _ctx(P, cfg)
    with pytest.raises(P.UnihennError):
        P.Net(ctx, cfg["input"], cfg["layers"], params, max_batch=1)
    _channel_parity(cfg, cfg["input"], cfg["layers"], params, False)


def test_literal_drop_level_feeds_the_network():
    """A LeNet-1 input encrypted on a longer chain (10 data primes, N = 2^11)
    is brought to the network's 8 limbs by Drop-Level as written (two
    products with encrypted all-ones vectors); the network's outputs equal
    the oracle's on its own dropped input, bit for bit."""
    import paper_2402_03060_amd as P
    from oracle.network import CkksEval
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    cfg["prime_bits"] = [60] + [40] * 9
    sess = OracleSession(cfg)
    ck = sess.ck
    onet = build_net(cfg, ck.slots)
    sess.ensure_keys(onet.rotation_set())
    xs = W.gen_inputs(cfg["input"], 1)
    ct = ck.encrypt(onet.input_vector(xs), 81)
    nl = ck.n_data
    ones = [ck.encrypt_pt(ck.encode(np.ones(ck.slots), float(ck.primes[nl - 1 - k]), nl), 82 + k,
                          float(ck.primes[nl - 1 - k])) for k in range(2)]
    dropped = ck.drop_level(ct, ones, sess.rlk)
    assert dropped.nl == onet.depth + 1 and dropped.scale == ct.scale
    exp = onet.run(CkksEval(ck, sess.key_handle, sess.rlk), [dropped])
    ctx = _ctx(P, cfg)
    g_rlk = ctx.import_evk(sess.rlk_coeff)
    g_drop = ctx.drop_level(ctx.import_ct(ct.data, ct.scale), [ctx.import_ct(o.data, o.scale) for o in ones], g_rlk)
    assert np.array_equal(ctx.export_ct(g_drop)[0], dropped.data)
    gnet = _gpu_net(P, ctx, cfg, sess, onet)
    for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED):
        gnet.set_mode(mode)
        got = [ctx.export_ct(o)[0] for o in gnet.eval(g_drop)]
        for g, e in zip(got, exp):
            assert np.array_equal(g, e.data), mode
    got = decrypt_outputs(sess, onet, exp)
    assert np.abs(got - reference_outputs(onet, xs)).max() < 1e-3


def _custom_parity(log_n, inp, layers, samples=1, stride=0, lazy=False):
    """GPU outputs equal to the oracle's for a network given by its layers
    (plain and hoisted modes)."""
    import paper_2402_03060_amd as P
    from oracle.network import Net as ONet
    ring = dict(W.config("lenet1"), log_n=log_n)
    sess = OracleSession(ring)
    params = W.gen_params(layers)
    onet = ONet(inp, layers, params, sess.ck.slots, samples, stride)
    xs = W.gen_inputs(inp, samples)
    ct, outs, _ = run_encrypted(sess, onet, xs, lazy=lazy)
    ctx = _ctx(P, ring)
    gnet = P.Net(ctx, inp, layers, params, samples=samples, stride=stride, max_batch=1, lazy=lazy)
    assert gnet.depth == onet.depth and sorted(gnet.rotations()) == onet.rotation_set()
    keys = {r: ctx.import_evk(sess.key_coeff[r]) for r in gnet.rotations()}
    gnet.bind_keys(keys, ctx.import_evk(sess.rlk_coeff))
    gin = ctx.import_ct(ct.data[None], ct.scale)
    for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED):
        gnet.set_mode(mode)
        got = [ctx.export_ct(o)[0] for o in gnet.eval(gin)]
        for g, e in zip(got, outs):
            assert np.array_equal(g, e.data), mode
    return gnet


@pytest.mark.parametrize("name", ["same_pool", "two_padded", "strided_first", "1d"])
@pytest.mark.parametrize("lazy", [False, True])
def test_padding_bit_exact(name, lazy):
    """Zero-padded convolutions over Section VI's reserved space (a lead of
    zero slots, a wider row pitch) at N = 2^11, default and deferred-ModDown
    plans, against the oracle."""
    from tests.test_oracle_network import PAD_NETS
    inp, layers = PAD_NETS[name]
    _custom_parity(11, inp, layers, lazy=lazy)


def test_padding_packed_samples_bit_exact():
    """Three padded samples per ciphertext at stride 512 (N = 2^12)."""
    from tests.test_oracle_network import PAD_NETS
    inp, layers = PAD_NETS["two_padded"]
    _custom_parity(12, inp, layers, samples=3, stride=512)


def test_padding_rejected_by_the_planner():
    """The planner refuses padded reads that would not be zero: no margin
    columns, too short a lead, a pooled input."""
    import paper_2402_03060_amd as P
    from tests.test_oracle_network import PAD_INPUT, PAD_NETS
    ctx = _ctx(P, dict(W.config("lenet1"), log_n=11))
    layers = PAD_NETS["same_pool"][1]
    params = W.gen_params(layers)
    for inp in (dict(PAD_INPUT, pitch=12), dict(PAD_INPUT, lead=13)):
        with pytest.raises(P.UnihennError):
            P.Net(ctx, inp, layers, params)
    pooled = [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1}, {"kind": "avgpool", "c": 2},
              {"kind": "conv", "ch_in": 2, "ch_out": 2, "k": 3, "s": 1, "pad": 1}, W.FLATTEN,
              {"kind": "fc", "din": 50, "dout": 2}]
    with pytest.raises(P.UnihennError):
        P.Net(ctx, PAD_INPUT, pooled, W.gen_params(pooled))


@pytest.mark.parametrize("name", ["k1", "k2s2", "fc_wide"])
def test_degenerate_shapes_bit_exact(name):
    """1 x 1 kernels, stride equal to the kernel, an FC wider than its input
    and an FC to a single output (N = 2^11)."""
    from tests.test_oracle_network import DEGENERATE_INPUT, DEGENERATE_NETS
    _custom_parity(11, DEGENERATE_INPUT, DEGENERATE_NETS[name])
    _custom_parity(11, DEGENERATE_INPUT, DEGENERATE_NETS[name], lazy=True)
