"""The C ABI's error contract: each documented UNIHENN_E* code comes back
for its condition, before anything is enqueued, so the output buffers keep
their contents.  Conditions: a missing rotation or relinearisation key
(ENOKEY), an exhausted level (ELEVEL; a network deeper than the chain), MAC
terms at different scales (ESCALE; Section II-B's Add needs equal scales), a
convolution with kernel smaller than its stride (EINVAL; Theorem 1 needs
K >= S), packed samples whose footprint exceeds their stride (ESLOTS;
Section VI's sizing rule: the 1D CNN at 32 sequences of stride 128), and a
batch above the net's maximum (EINVAL)."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A5A5A


def _ctx(P, cfg):
    return P.Context(cfg["log_n"], cfg["prime_bits"], cfg["special_bits"], 2.0 ** cfg["log_scale"])


def _fresh_ct(P, ctx, batch, nl, scale):
    ct = ctx.empty_ct(batch, nl, scale)
    ct.data.fill_(SENTINEL)
    return ct


def _untouched(ct) -> bool:
    import torch
    torch.cuda.synchronize()
    return bool((ct.data == SENTINEL).all())


def _code(fn):
    import paper_2402_03060_amd as P
    with pytest.raises(P.UnihennError) as ei:
        fn()
    return ei.value.code


def _small_lenet(P):
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    ctx = _ctx(P, cfg)
    params = W.gen_params(cfg["layers"])
    net = P.Net(ctx, cfg["input"], cfg["layers"], params)
    return cfg, ctx, net


def test_enokey_eval_before_keys_and_missing_rotation():
    import paper_2402_03060_amd as P
    cfg, ctx, net = _small_lenet(P)
    x = ctx.import_ct(np.zeros((1, 2, net.in_limbs, ctx.n), dtype=np.uint64), ctx.scale)
    outs = [_fresh_ct(P, ctx, 1, 1, 0.0) for _ in range(net.n_out)]
    assert _code(lambda: net.eval(x, outs)) == P.ENOKEY
    assert all(_untouched(o) for o in outs)
    sk = P.keygen_secret(ctx, 5)
    rots = net.rotations()
    keys = {r: P.gen_switch_key(ctx, sk, 6, steps=r) for r in rots[1:]}     # one rotation key missing
    rlk = P.gen_switch_key(ctx, sk, 7, relin=True)
    assert _code(lambda: net.bind_keys(keys, rlk)) == P.ENOKEY
    keys[rots[0]] = P.gen_switch_key(ctx, sk, 6, steps=rots[0])
    assert _code(lambda: net.bind_keys(keys, None)) == P.ENOKEY          # no relinearisation key
    net.bind_keys(keys, rlk)
    net.eval(x, outs)                                                    # now accepted
    # a single rotation without its key
    ws = ctx.workspace(net.in_limbs, 1)
    assert _code(lambda: ctx.rotate(x, 3, None, ws)) == P.ENOKEY


def test_elevel_rescale_at_one_limb_and_network_deeper_than_the_chain():
    import paper_2402_03060_amd as P
    cfg = W.config("lenet1")
    cfg["log_n"] = 11
    ctx = _ctx(P, cfg)
    one = ctx.import_ct(np.zeros((1, 2, 1, ctx.n), dtype=np.uint64), ctx.scale)
    ws = ctx.workspace(1, 1)
    assert _code(lambda: ctx.rescale(one, ws)) == P.ELEVEL
    # LeNet-1 needs depth 7 + 1 limbs; a chain of four primes cannot hold it
    short = P.Context(11, [60, 40, 40, 40], 60, 2.0 ** 40)
    params = W.gen_params(cfg["layers"])
    assert _code(lambda: P.Net(short, cfg["input"], cfg["layers"], params)) == P.ELEVEL


def test_escale_mac_terms_at_different_scales():
    import paper_2402_03060_amd as P
    cfg = W.config("conv1")
    cfg["log_n"] = 11
    ctx = _ctx(P, cfg)
    nl = 2
    a = ctx.import_ct(np.ones((1, 2, nl, ctx.n), dtype=np.uint64), ctx.scale)
    b = ctx.import_ct(np.ones((1, 2, nl, ctx.n), dtype=np.uint64), ctx.scale * 2)
    pt = ctx.encode(np.ones(8), ctx.scale, nl)
    acc = _fresh_ct(P, ctx, 1, nl, 0.0)
    assert _code(lambda: ctx.mul_plain_acc([a, b], [pt, pt], acc)) == P.ESCALE
    assert _untouched(acc)
    ctx.mul_plain_acc([a, a], [pt, pt], acc)                             # equal scales are accepted
    # terms at different levels
    c = ctx.import_ct(np.ones((1, 2, nl + 1, ctx.n), dtype=np.uint64), ctx.scale)
    acc2 = _fresh_ct(P, ctx, 1, nl, 0.0)
    assert _code(lambda: ctx.mul_plain_acc([a, c], [pt, pt], acc2)) == P.ELEVEL
    assert _untouched(acc2)


def test_einval_kernel_smaller_than_stride():
    import paper_2402_03060_amd as P
    cfg = W.config("m1")
    cfg["log_n"] = 11
    ctx = _ctx(P, cfg)
    layers = [dict(cfg["layers"][0], k=2, s=3)] + cfg["layers"][1:2]
    params = W.gen_params(layers)
    with pytest.raises(P.UnihennError) as ei:
        P.Net(ctx, cfg["input"], layers, params)
    assert ei.value.code == P.EINVAL and "Theorem 1" in str(ei.value)


def test_eslots_cnn1d_as_written():
    """32 sequences per ciphertext at stride 128: the flatten output (944
    slots) and the FC's width (945) exceed the stride."""
    import paper_2402_03060_amd as P
    cfg = W.config("cnn1d")
    ctx = _ctx(P, cfg)
    params = W.gen_params(cfg["layers"])
    assert _code(lambda: P.Net(ctx, cfg["input"], cfg["layers"], params, samples=32, stride=128)) == P.ESLOTS
    # 8 sequences at stride 1024 fit
    P.Net(ctx, cfg["input"], cfg["layers"], params, samples=8, stride=1024)


def test_einval_batch_above_the_maximum():
    import paper_2402_03060_amd as P
    cfg, ctx, net = _small_lenet(P)
    sk = P.keygen_secret(ctx, 5)
    net.bind_keys({r: P.gen_switch_key(ctx, sk, 6, steps=r) for r in net.rotations()},
                  P.gen_switch_key(ctx, sk, 7, relin=True))
    x = ctx.import_ct(np.zeros((2, 2, net.in_limbs, ctx.n), dtype=np.uint64), ctx.scale)
    outs = [_fresh_ct(P, ctx, 2, 1, 0.0) for _ in range(net.n_out)]
    assert _code(lambda: net.eval(x, outs)) == P.EINVAL
    assert all(_untouched(o) for o in outs)
