"""Oracle network: layer algorithms (Algorithms 1 and 2, average pooling,
flatten) checked against a direct FP64 CNN, without encryption (slot
simulation) and with encryption (CPU CKKS oracle).  No GPU."""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W
from oracle.network import (Net, PlanError, SlotEval, check_packing, cnn_fp64, footprint, network_depth,
                            read_outputs, shapes)
from oracle.run import OracleSession, build_net, decrypt_outputs, reference_outputs, run_encrypted


def _slot_run(name, samples=None, stride=None):
    cfg = W.config(name)
    n_slots = 2 ** (cfg["log_n"] - 1)
    params = W.gen_params(cfg["layers"])
    S = cfg["samples_per_ct"] if samples is None else samples
    st = cfg["sample_stride"] if stride is None else stride
    xs = W.gen_inputs(cfg["input"], S)
    net = Net(cfg["input"], cfg["layers"], params, n_slots, S, st)
    ev = SlotEval(n_slots)
    outs = net.run(ev, [net.input_vector(xs)])
    got = read_outputs(net, outs)
    ref = np.array([cnn_fp64(x, cfg["layers"], params).reshape(-1) for x in xs])
    return got, ref, ev.count.as_dict(), net


@pytest.mark.parametrize("name", list(W.CONFIGS))
def test_slot_simulation_matches_fp64_cnn(name):
    got, ref, _, _ = _slot_run(name)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() < 1e-12


def test_lenet1_operation_counts():
    """Exact primitive counts of Algorithms 1 and 2, pooling and flatten for
    LeNet-1: conv rotations CH_in K^2 minus the zero shifts, conv products
    CH_in CH_out K^2, pooling c^2 - 1 rotations per channel, flatten W_in +
    H_in products and rotations per channel plus CH - 1 packing rotations,
    FC 2 DAT_out - 1 products and 2 (DAT_out - 1) + ceil(DAT_in / DAT_out) - 1
    rotations."""
    _, _, cnt, net = _slot_run("lenet1")
    conv_rot = (1 * 25 - 1) + (4 * 25 - 4)
    conv_mac = 1 * 4 * 25 + 4 * 12 * 25
    pool_rot = 3 * 4 + 3 * 12
    flat_rot = 12 * (3 + 3) + 11
    flat_mac = 12 * (4 + 4)
    fc_rot = 2 * 9 + math.ceil(192 / 10) - 1
    fc_mac = 2 * 10 - 1
    assert cnt["rot"] == conv_rot + pool_rot + flat_rot + fc_rot == 288
    assert cnt["mac"] == conv_mac + flat_mac + fc_mac == 1415
    assert cnt["relin"] == 4 + 12
    assert cnt["rescale"] == 4 + 4 + 12 + 12 + 12 + 12 + 1 == 57
    assert len(net.rotation_set()) == 81


@pytest.mark.parametrize("name,expect", [("conv1", 2), ("lenet1", 7), ("cnn1d", 6), ("cifar_cnn", 7)])
def test_depth(name, expect):
    cfg = W.config(name)
    assert network_depth(cfg["input"], cfg["layers"]) == expect


def test_theorem1_conv_does_not_grow():
    """H_img >= H_out(i) * prod_{j<=i} S_j whenever K >= S >= 1 (Theorem 1 and
    its corollary for widths), over random conv stacks."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        H = int(rng.integers(8, 64))
        h, prod = H, 1
        for _ in range(int(rng.integers(1, 4))):
            K = int(rng.integers(1, 6))
            S = int(rng.integers(1, K + 1))
            if h < K:
                break
            h = (h - K) // S + 1
            prod *= S
            assert H >= h * prod


def test_stride_larger_than_kernel_rejected():
    inp = {"c": 1, "h": 28, "w": 28, "dist": "uniform01"}
    with pytest.raises(PlanError):
        footprint(inp, [{"kind": "conv", "ch_in": 1, "ch_out": 1, "k": 2, "s": 3}])


def test_cnn1d_packing_as_written_overflows():
    """32 sequences at stride 128 cannot hold the 944-slot flatten output or
    the 945-slot FC width; 8 at stride 1024 fit."""
    cfg = W.config("cnn1d")
    assert footprint(cfg["input"], cfg["layers"]) == 945
    with pytest.raises(PlanError):
        check_packing(cfg["input"], cfg["layers"], 8192, 32, 128)
    assert check_packing(cfg["input"], cfg["layers"], 8192, 8, 1024) == 1024


def test_packed_equals_single_slot_sim():
    got10, ref10, _, _ = _slot_run("lenet1_batched")
    got1, ref1, _, _ = _slot_run("lenet1", samples=1)
    assert np.abs(got10[0] - got1[0]).max() < 1e-12
    assert np.abs(got10 - ref10).max() < 1e-12


def test_shapes_lenet1():
    cfg = W.config("lenet1")
    assert shapes(cfg["input"], cfg["layers"])[-2:] == [(192,), (10,)]


# ---------------------------------------------------------------- encrypted
def test_encrypted_conv1_config():
    cfg = W.config("conv1")
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, ev = run_encrypted(sess, net, xs)
    assert ev.count.as_dict() == {"rot": 24, "mac": 100, "rescale": 8, "relin": 4}
    got = decrypt_outputs(sess, net, outs)
    assert all(o.nl == 1 for o in outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3


def test_encrypted_packing_isolation():
    """Five images packed at stride 784 decrypt to the same outputs as each
    image alone (conv + square at N = 2^13)."""
    cfg = W.config("conv1")
    sess = OracleSession(cfg)
    cfgp = dict(cfg, samples_per_ct=5, sample_stride=784)
    netp = build_net(cfgp, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 5)
    _, outs, _ = run_encrypted(sess, netp, xs)
    packed = decrypt_outputs(sess, netp, outs)
    ref = reference_outputs(netp, xs)
    assert np.abs(packed - ref).max() < 1e-3
    net1 = build_net(cfg, sess.ck.slots)
    _, outs1, _ = run_encrypted(sess, net1, xs[2:3])
    single = decrypt_outputs(sess, net1, outs1)
    assert np.abs(packed[2] - single[0]).max() < 1e-3


@pytest.mark.slow
def test_encrypted_lenet1_small_ring():
    """LeNet-1 shape end to end at N = 2^11 (1024 slots hold the 784-slot
    footprint) with the same 60 + 7 x 40 + 60 chain: 7 levels consumed,
    logits within 1e-3 of FP64."""
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, ev = run_encrypted(sess, net, xs)
    assert outs[0].nl == 1
    assert ev.count.rescale == 57
    got = decrypt_outputs(sess, net, outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3


@pytest.mark.slow
def test_lenet1_full_size_golden_is_current():
    """The oracle still produces the committed full-size LeNet-1 digests
    (keys, input, outputs), so the GPU golden test compares against the
    oracle as it stands."""
    import importlib.util
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(here, "lenet1_full.json")) as f:
        rec = json.load(f)
    spec = importlib.util.spec_from_file_location("make_lenet1_golden", os.path.join(here, "make_lenet1_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert json.loads(json.dumps(mod.compute())) == rec
    assert rec["max_abs_err_vs_fp64"] < 1e-3


def test_relu_after_pooling_folds_the_factor():
    """Approximate ReLU right after average pooling applies f to the
    average: the deferred 1/c^2 enters as b/c^2 and c/c^4 (Section IV-C)."""
    inp = {"c": 1, "h": 12, "w": 12, "dist": "uniform01"}
    layers = [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1}, {"kind": "avgpool", "c": 2},
              W.RELU, W.FLATTEN, {"kind": "fc", "din": 50, "dout": 4}]
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    net = Net(inp, layers, params, 1024)
    ev = SlotEval(1024)
    got = read_outputs(net, net.run(ev, [net.input_vector(xs)]))
    ref = cnn_fp64(xs[0], layers, params).reshape(-1)
    assert np.abs(got[0] - ref).max() < 1e-12
    assert network_depth(inp, layers) == 1 + 2 + 2 + 1


@pytest.mark.slow
@pytest.mark.parametrize("name,log_n", [("m3", 12), ("m7", 11), ("m6", 11)])
def test_encrypted_models_small_ring(name, log_n):
    """Approximate ReLU (M3), 1D convolutions of stride 2 with FC -> square ->
    FC (M7), and a stride-2 2D model (M6) end to end on the CPU CKKS oracle:
    every level consumed, outputs within 1e-3 of the FP64 CNN."""
    cfg = W.config(name)
    cfg["log_n"] = log_n
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, ev = run_encrypted(sess, net, xs)
    assert all(o.nl == 1 for o in outs)
    got = decrypt_outputs(sess, net, outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3


# ------------------------------------------------------------ doubling FC sum
def _doubling_rotations(reps: int) -> int:
    return (reps.bit_length() - 1) + bin(reps).count("1") - 1


@pytest.mark.parametrize("name", list(W.CONFIGS))
def test_fc_doubling_slot_simulation(name):
    """The doubling form of Algorithm 2's closing sum gives the FP64 CNN slot
    for slot on every workload, and saves exactly
    (reps - 1) - (floor(log2 reps) + popcount(reps) - 1) rotations per FC."""
    cfg = W.config(name)
    n_slots = 2 ** (cfg["log_n"] - 1)
    params = W.gen_params(cfg["layers"])
    S, st = cfg["samples_per_ct"], cfg["sample_stride"]
    xs = W.gen_inputs(cfg["input"], S)
    ref = np.array([cnn_fp64(x, cfg["layers"], params).reshape(-1) for x in xs])
    counts = []
    for dbl in (False, True):
        net = Net(cfg["input"], cfg["layers"], params, n_slots, S, st, fc_doubling=dbl)
        ev = SlotEval(n_slots)
        got = read_outputs(net, net.run(ev, [net.input_vector(xs)]))
        assert np.abs(got - ref).max() < 1e-12
        counts.append(ev.count.rot)
    saved = 0
    for lay in cfg["layers"]:
        if lay["kind"] == "fc":
            reps = math.ceil(lay["din"] / lay["dout"])
            saved += (reps - 1) - _doubling_rotations(reps)
    assert counts[0] - counts[1] == saved


def test_fc_doubling_counts_lenet1_cnn1d():
    """LeNet-1's 192 -> 10 FC sums 20 copies with 4 + 2 - 1 = 5 rotations
    (19 before); the 1D CNN's 944 -> 5 FC sums 189 copies with 7 + 6 - 1 = 12
    (188 before)."""
    assert _doubling_rotations(20) == 5 and _doubling_rotations(189) == 12
    assert _doubling_rotations(1) == 0 and _doubling_rotations(2) == 1 and _doubling_rotations(3) == 2


@pytest.mark.slow
@pytest.mark.parametrize("lazy", [False, True])
def test_encrypted_lenet1_fc_doubling(lazy):
    """LeNet-1 at N = 2^11 with the doubling FC sum (and with deferred
    ModDown): within 1e-3 of the FP64 CNN."""
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    sess = OracleSession(cfg)
    net = build_net(cfg, sess.ck.slots, fc_doubling=True)
    xs = W.gen_inputs(cfg["input"], 1)
    _, outs, ev = run_encrypted(sess, net, xs, lazy=lazy)
    assert ev.count.rot == 274
    got = decrypt_outputs(sess, net, outs)
    assert np.abs(got - reference_outputs(net, xs)).max() < 1e-3


# ------------------------------------------------- one ciphertext per channel
@pytest.mark.parametrize("name", ["cifar_cnn", "m5"])
def test_channel_cts_slot_simulation(name):
    """Multi-channel inputs given as one ciphertext per channel (each plane
    at offset 0) reproduce the FP64 CNN like the single-ciphertext layout."""
    cfg = W.config(name)
    n_slots = 2 ** (cfg["log_n"] - 1)
    params = W.gen_params(cfg["layers"])
    xs = W.gen_inputs(cfg["input"], 1)
    net = Net(cfg["input"], cfg["layers"], params, n_slots, channel_cts=True)
    ev = SlotEval(n_slots)
    got = read_outputs(net, net.run(ev, net.input_vectors(xs)))
    ref = np.array([cnn_fp64(x, cfg["layers"], params).reshape(-1) for x in xs])
    assert np.abs(got - ref).max() < 1e-12


def test_channel_cts_fit_where_one_ciphertext_cannot():
    """3 x 32 x 32 inputs need 3072 slots in one ciphertext; at N = 2^12
    (2048 slots) only the per-channel layout (1024 slots each) fits."""
    cfg = W.config("cifar_cnn")
    with pytest.raises(PlanError):
        check_packing(cfg["input"], cfg["layers"], 2048, 1, 2048)
    assert footprint(cfg["input"], cfg["layers"], channel_cts=True) <= 2048


SMALL3 = ({"c": 3, "h": 12, "w": 12, "dist": "uniform01"},
          [{"kind": "conv", "ch_in": 3, "ch_out": 2, "k": 3, "s": 1}, W.SQUARE, {"kind": "avgpool", "c": 2},
           W.FLATTEN, {"kind": "fc", "din": 50, "dout": 4}])


@pytest.mark.parametrize("lazy", [False, True])
def test_encrypted_channel_cts_small(lazy):
    """A three-channel input as three ciphertexts (N = 2^11), eager and with
    deferred ModDown: within 1e-3 of the FP64 CNN."""
    inp, layers = SMALL3
    ring = dict(W.config("lenet1"), log_n=11)
    sess = OracleSession(ring)
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    net = Net(inp, layers, params, sess.ck.slots, channel_cts=True)
    cts, outs, _ = run_encrypted(sess, net, xs, lazy=lazy)
    assert len(cts) == 3
    got = read_outputs(net, [sess.ck.decrypt(o) for o in outs])
    assert np.abs(got[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-3


# ------------------------------------------------------------ padding
PAD_INPUT = {"c": 1, "h": 12, "w": 12, "dist": "uniform01", "pitch": 13, "lead": 14}
PAD_NETS = {
    # "same" padding, then pooling and the flatten after pooling
    "same_pool": (PAD_INPUT, [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1, "pad": 1}, W.SQUARE,
                              {"kind": "avgpool", "c": 2}, W.FLATTEN, {"kind": "fc", "din": 72, "dout": 5}]),
    # two padded convolutions, the second of stride 2 on a convolution output
    "two_padded": (PAD_INPUT, [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1, "pad": 1}, W.SQUARE,
                               {"kind": "conv", "ch_in": 2, "ch_out": 3, "k": 3, "s": 2, "pad": 1}, W.SQUARE,
                               W.FLATTEN, {"kind": "fc", "din": 108, "dout": 5}]),
    # a padded stride-2 convolution first: the next one reads at interval 2
    "strided_first": ({"c": 1, "h": 12, "w": 12, "dist": "uniform01", "pitch": 14, "lead": 30},
                      [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 2, "pad": 1}, W.SQUARE,
                       {"kind": "conv", "ch_in": 2, "ch_out": 2, "k": 3, "s": 1, "pad": 1}, W.FLATTEN,
                       {"kind": "fc", "din": 72, "dout": 4}]),
    # 1D convolutions padded along the width
    "1d": ({"c": 1, "h": 1, "w": 32, "dist": "normal", "pitch": 34, "lead": 2},
           [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1, "dims": 1, "pad": 1}, W.SQUARE,
            {"kind": "conv", "ch_in": 2, "ch_out": 2, "k": 3, "s": 2, "dims": 1, "pad": 1}, W.FLATTEN,
            {"kind": "fc", "din": 32, "dout": 4}]),
}


@pytest.mark.parametrize("name", list(PAD_NETS))
@pytest.mark.parametrize("samples", [1, 3])
def test_padding_slot_simulation(name, samples):
    """Zero-padded convolutions (Section VI's reserved space: a lead of zero
    slots per sample and a wider row pitch) give the FP64 CNN on zero-padded
    inputs, slot for slot, alone and with three packed samples."""
    inp, layers = PAD_NETS[name]
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, samples)
    n_slots, stride = (2048, 0) if samples == 1 else (4096, 1024)
    net = Net(inp, layers, params, n_slots, samples, stride)
    ev = SlotEval(n_slots)
    got = read_outputs(net, net.run(ev, net.input_vectors(xs)))
    ref = np.array([cnn_fp64(x, layers, params).reshape(-1) for x in xs])
    assert np.abs(got - ref).max() < 1e-12


def test_padding_fp64_reference_is_zero_padding():
    """The FP64 reference pads with zeros: a 1 x 1 kernel of weight 1 and
    padding 1 returns the input inside a zero border."""
    x = np.arange(12.0).reshape(1, 3, 4)
    lay = {"kind": "conv", "ch_in": 1, "ch_out": 1, "k": 1, "s": 1, "pad": 1}
    out = cnn_fp64(x, [lay], [(np.ones((1, 1, 1, 1)), np.zeros(1))])
    assert out.shape == (1, 5, 6) and np.array_equal(out[0, 1:4, 1:5], x[0]) and out.sum() == x.sum()


@pytest.mark.parametrize("inp,layers,channel_cts,msg", [
    ({"c": 3, "h": 8, "w": 8, "dist": "uniform01", "pitch": 9, "lead": 10},
     [{"kind": "conv", "ch_in": 3, "ch_out": 2, "k": 3, "s": 1, "pad": 1}], False, "one ciphertext per input channel"),
    (dict(PAD_INPUT, pitch=12), PAD_NETS["same_pool"][1], False, "zero columns"),
    (dict(PAD_INPUT, lead=13), PAD_NETS["same_pool"][1], False, "leading space"),
    (PAD_INPUT, [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 3, "s": 1}, {"kind": "avgpool", "c": 2},
                 {"kind": "conv", "ch_in": 2, "ch_out": 2, "k": 3, "s": 1, "pad": 1}], False, "pooled map"),
])
def test_padding_rejected_where_the_reads_are_not_zero(inp, layers, channel_cts, msg):
    params = W.gen_params(layers)
    net = Net(inp, layers, params, 2048, channel_cts=channel_cts)
    with pytest.raises(PlanError, match=msg):
        net.run(SlotEval(2048), net.input_vectors(W.gen_inputs(inp, 1)))


def test_padding_channel_cts():
    """A padded convolution of a three-channel input given as one ciphertext
    per channel."""
    inp = {"c": 3, "h": 8, "w": 8, "dist": "uniform01", "pitch": 9, "lead": 10}
    layers = [{"kind": "conv", "ch_in": 3, "ch_out": 2, "k": 3, "s": 1, "pad": 1}, W.SQUARE, W.FLATTEN,
              {"kind": "fc", "din": 128, "dout": 4}]
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    net = Net(inp, layers, params, 2048, channel_cts=True)
    got = read_outputs(net, net.run(SlotEval(2048), net.input_vectors(xs)))
    assert np.abs(got[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-12


@pytest.mark.parametrize("lazy", [False, True])
def test_encrypted_padding(lazy):
    """The two-padded-convolution net encrypted at N = 2^11 (eager and with
    deferred ModDown): within 1e-3 of the FP64 CNN."""
    inp, layers = PAD_NETS["two_padded"]
    ring = dict(W.config("lenet1"), log_n=11)
    sess = OracleSession(ring)
    params = W.gen_params(layers)
    xs = W.gen_inputs(inp, 1)
    net = Net(inp, layers, params, sess.ck.slots)
    _, outs, _ = run_encrypted(sess, net, xs, lazy=lazy)
    got = read_outputs(net, [sess.ck.decrypt(o) for o in outs])
    assert np.abs(got[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-3


# ------------------------------------------------------- degenerate shapes
DEGENERATE_INPUT = {"c": 1, "h": 8, "w": 8, "dist": "uniform01"}
DEGENERATE_NETS = {
    # 1 x 1 kernels: Algorithm 1 with a single term per output (no rotation)
    "k1": [{"kind": "conv", "ch_in": 1, "ch_out": 3, "k": 1, "s": 1}, W.SQUARE, W.FLATTEN,
           {"kind": "fc", "din": 192, "dout": 4}],
    # stride equal to the kernel (Theorem 1's boundary K = S)
    "k2s2": [{"kind": "conv", "ch_in": 1, "ch_out": 2, "k": 2, "s": 2}, W.SQUARE, W.FLATTEN,
             {"kind": "fc", "din": 32, "dout": 3}],
    # FC wider than its input (one copy, no closing rotations) and an FC to one output
    "fc_wide": [{"kind": "conv", "ch_in": 1, "ch_out": 1, "k": 3, "s": 1}, W.SQUARE, W.FLATTEN,
                {"kind": "fc", "din": 36, "dout": 50}, W.SQUARE, {"kind": "fc", "din": 50, "dout": 1}],
}


@pytest.mark.parametrize("name", list(DEGENERATE_NETS))
def test_degenerate_shapes_slot_simulation(name):
    layers = DEGENERATE_NETS[name]
    params = W.gen_params(layers)
    xs = W.gen_inputs(DEGENERATE_INPUT, 1)
    net = Net(DEGENERATE_INPUT, layers, params, 1024)
    got = read_outputs(net, net.run(SlotEval(1024), net.input_vectors(xs)))
    assert np.abs(got[0] - cnn_fp64(xs[0], layers, params).reshape(-1)).max() < 1e-12
