"""GPU parity of the deferred-ModDown plan (PLAN_LAZY_MODDOWN): the HIP
library against the oracle's LazyCkksEval, residue by residue, in the plain,
hoisted and graph-replay modes; the plan's bookkeeping (extended registers,
plaintexts with the P limb) across every layer kind."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle.network import Net as OracleNet
from oracle.network import cnn_fp64, read_outputs
from oracle.run import OracleSession, run_encrypted
from tests.test_gpu_network import _ctx, _run_parity

pytestmark = pytest.mark.gpu


def _all_modes(P):
    return (P.EVAL_PLAIN, P.EVAL_HOISTED, P.EVAL_HOISTED | P.EVAL_GRAPH, P.EVAL_PLAIN | P.EVAL_GRAPH)


def test_lazy_conv1_config_bit_exact():
    """Conv (4 filters 5 x 5) + square at N = 2^13: 24 extended rotations
    and the identity term in one extended multi-output sum, four ModDowns."""
    import paper_2402_03060_amd as P
    _run_parity(W.config("conv1"), lazy=True, modes=_all_modes(P))


def test_lazy_lenet1_small_ring_bit_exact():
    """Every layer kind at N = 2^11: pooling sums and the flatten / FC sums
    stay extended; conv2 and flatten rotate the ModDown of a pooled sum."""
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    _run_parity(cfg, lazy=True, modes=_all_modes(P))


@pytest.mark.parametrize("n_cts", [2, 5])
def test_lazy_lenet1_packed_batch_bit_exact(n_cts):
    cfg = W.config("lenet1_batched")
    cfg["log_n"] = 12
    cfg["samples_per_ct"] = 2
    _run_parity(cfg, n_cts=n_cts, lazy=True)


@pytest.mark.parametrize("name,log_n", [("cnn1d", 12), ("m3", 12), ("m1", 11), ("m6", 11), ("m7", 11),
                                        ("m4", 11)])
def test_lazy_models_bit_exact(name, log_n):
    """1D stride-2 convolutions and the row-interval flatten (cnn1d, M7),
    approximate ReLU (M3), stride-3 / stride-2 convolutions with FC -> square
    -> FC (M1, M6), LeNet-5's 1 x 1 flatten (M4)."""
    cfg = W.config(name)
    cfg["log_n"] = log_n
    if name == "cnn1d":
        cfg["samples_per_ct"] = 2
    _run_parity(cfg, lazy=True)


def test_lazy_relu_after_pooling_bit_exact():
    """Approximate ReLU right after pooling: its first product takes the
    extended pooled sum, its Mul(C) the sum's ModDown."""
    import paper_2402_03060_amd as P
    inp = {"c": 1, "h": 12, "w": 12, "dist": "uniform01"}
    layers = [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1}, {"kind": "avgpool", "c": 2},
              W.RELU, W.FLATTEN, {"kind": "fc", "din": 50, "dout": 4}]
    ring = dict(W.config("lenet1"), log_n=11)
    sess = OracleSession(ring)
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    onet = OracleNet(inp, layers, params, sess.ck.slots)
    ct, outs, _ = run_encrypted(sess, onet, xs, lazy=True)
    got_o = read_outputs(onet, [sess.ck.decrypt(o) for o in outs])
    assert np.abs(got_o[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-3
    ctx = _ctx(P, ring)
    gnet = P.Net(ctx, inp, layers, params, max_batch=1, lazy=True)
    keys = {r: ctx.import_evk(sess.key_coeff[r]) for r in gnet.rotations()}
    gnet.bind_keys(keys, ctx.import_evk(sess.rlk_coeff))
    for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED):
        gnet.set_mode(mode)
        got = [ctx.export_ct(o)[0] for o in gnet.eval(ctx.import_ct(ct.data[None], ct.scale))]
        for g, e in zip(got, outs):
            assert np.array_equal(g, e.data)


def test_lazy_plan_differs_and_rejects_extended_conv_input():
    """The lazy plan changes bits (so both plans are really exercised), and
    the single-layer conv entry refuses a layer whose input is an extended
    pooled sum in the plan."""
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    from oracle.run import build_net
    onet = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, eager, _ = run_encrypted(sess, onet, xs)
    _, lazy, _ = run_encrypted(sess, onet, xs, lazy=True)
    assert not np.array_equal(eager[0].data, lazy[0].data)
    ctx = _ctx(P, cfg)
    gnet = P.Net(ctx, cfg["input"], cfg["layers"], onet.params, max_batch=1, lazy=True)
    keys = {r: ctx.import_evk(sess.key_coeff[r]) for r in gnet.rotations()}
    gnet.bind_keys(keys, ctx.import_evk(sess.rlk_coeff))
    nl = onet.depth + 1 - 2
    ins = [ctx.import_ct(sess.ck.limb_drop(sess.ck.encrypt(np.zeros(sess.ck.slots), 5 + i), nl).data, 1.0)
           for i in range(4)]
    with pytest.raises(P.UnihennError):
        gnet.conv(3, ins, 12, nl - 1)


@pytest.mark.parametrize("fuse_min_wg", [None, "0"])
def test_lazy_workgroup_orders_and_groups_identical(monkeypatch, fuse_min_wg):
    """Every workgroup order of the extended inner product (the row-fused one
    on the plain path, also forced onto every group), at several group
    sizes, gives the oracle's residues (LeNet-1 at N = 2^11, hoisted and
    plain)."""
    if fuse_min_wg is not None:
        monkeypatch.setenv("UNIHENN_KS_FUSE_MIN_WG", fuse_min_wg)
    import paper_2402_03060_amd as P
    from oracle.run import build_net
    from tests.test_gpu_network import _gpu_net
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    onet = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    ct, outs, _ = run_encrypted(sess, onet, xs, lazy=True)
    ctx = _ctx(P, cfg)
    gnet = _gpu_net(P, ctx, cfg, sess, onet, lazy=True)
    gin = ctx.import_ct(ct.data[None], ct.scale)
    for setting in ({"ks_group": 8, "ks_order": 1}, {"ks_group": 32, "ks_order": 1, "ks_min_wg": 512},
                    {"ks_group": 3, "ks_order": 0}, {"ks_group": 8, "ks_order": 2}, {"ks_group": 64, "ks_order": 2},
                    {"ks_group": 3, "ks_order": 2, "ntt_tile_log": 12}):
        gnet.set_tuning(**setting)
        for mode in (P.EVAL_PLAIN, P.EVAL_HOISTED):
            gnet.set_mode(mode)
            got = [ctx.export_ct(o)[0] for o in gnet.eval(gin)]
            for g, e in zip(got, outs):
                assert np.array_equal(g, e.data), (setting, mode)


@pytest.mark.parametrize("name,log_n,lazy", [("lenet1", 11, False), ("lenet1", 11, True), ("cnn1d", 12, False),
                                             ("cnn1d", 12, True)])
def test_fc_doubling_bit_exact(name, log_n, lazy):
    """Algorithm 2's closing sum by doubling (PLAN_FC_DOUBLING), alone and with
    deferred ModDown, against the oracle's fc_doubling mode: LeNet-1 (20
    copies, 5 rotations) and the 1D CNN (189 copies, 12 rotations; two
    sequences per ciphertext)."""
    import paper_2402_03060_amd as P
    cfg = W.config(name)
    cfg["log_n"] = log_n
    if name == "cnn1d":
        cfg["samples_per_ct"] = 2
    _run_parity(cfg, lazy=lazy, fc_doubling=True, modes=_all_modes(P))
