"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module holds only data: ring-parameter choices, network shapes and
seeded random draws of inputs, weights and biases.  It contains none of the
method's arithmetic (no encoding, no layer algorithm, no modular math), so
that the CPU oracle and the HIP path can both take their inputs from it while
sharing no code with each other.

Stand-ins for the paper's datasets (Section V-B): MNIST-shaped 1x28x28
images with values uniform in [0, 1], ECG-shaped length-128 sequences with
values N(0, 1), and CIFAR-shaped 3x32x32 images uniform in [0, 1].  Weights
are N(0, 0.1^2) and biases N(0, 0.01^2).  Seeds: 1 weights, 2 biases,
3 inputs, 4 arrival times.
"""
from __future__ import annotations

import copy
import numpy as np

SEED_WEIGHTS = 1
SEED_BIASES = 2
SEED_INPUTS = 3
SEED_ARRIVALS = 4
SEED_KEYS = 11
SEED_ENCRYPT = 12


# Layer records use the paper's notation (Table 1, Algorithms 1 and 2):
#   conv:    ch_in, ch_out, k (kernel K), s (stride S)
#   square:  the x^2 activation
#   relu_approx: the degree-2 polynomial approximation of ReLU
#   avgpool: c (kernel size and stride)
#   flatten: the flatten-layer converter
#   fc:      din (DAT_in), dout (DAT_out)
def _conv(ci, co, k, s):
    return {"kind": "conv", "ch_in": ci, "ch_out": co, "k": k, "s": s}


def _conv1d(ci, co, k, s):
    # 1D convolution on an H = 1 input: a 1 x K kernel, stride S along x
    return {"kind": "conv", "ch_in": ci, "ch_out": co, "k": k, "s": s, "dims": 1}


SQUARE = {"kind": "square"}
FLATTEN = {"kind": "flatten"}
RELU = {"kind": "relu_approx"}   # the degree-2 approximation of ReLU (Section V-A)


def _pool(c):
    return {"kind": "avgpool", "c": c}


def _fc(din, dout):
    return {"kind": "fc", "din": din, "dout": dout}


# Ring parameters: log2 N, data-prime bit sizes [b_0 .. b_L], special-prime
# bit size, log2 of the scale.  "depth" is the multiplicative depth of the
# network; the ciphertext is limb-dropped to depth+1 data primes first.
CONFIGS = {
    "conv1": {
        "desc": "one conv layer (4 filters 5x5, stride 1) + square on a 1x28x28 image",
        "log_n": 13, "prime_bits": [60, 40, 40], "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01"},
        "layers": [_conv(1, 4, 5, 1), SQUARE],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "lenet1": {
        "desc": "LeNet-1 shape (Table M2): conv 1->4 K5, sq, pool2, conv 4->12 K5, sq, pool2, flatten, FC 192->10",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01"},
        "layers": [_conv(1, 4, 5, 1), SQUARE, _pool(2), _conv(4, 12, 5, 1), SQUARE, _pool(2),
                   FLATTEN, _fc(192, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "lenet1_batched": {
        "desc": "LeNet-1 shape, ten 28x28 images per ciphertext at stride 784, 128 ciphertexts per launch",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01"},
        "layers": [_conv(1, 4, 5, 1), SQUARE, _pool(2), _conv(4, 12, 5, 1), SQUARE, _pool(2),
                   FLATTEN, _fc(192, 10)],
        "samples_per_ct": 10, "sample_stride": 784, "cts_per_batch": 128,
    },
    "cnn1d": {
        "desc": "1D CNN: conv1d 1->8 k7, sq, conv1d 8->16 k5 s2, sq, flatten, FC 944->5 "
                "(8 sequences per ciphertext at stride 1024; 128 does not hold the 944-slot flatten output)",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 1, "w": 128, "dist": "normal"},
        "layers": [_conv1d(1, 8, 7, 1), SQUARE, _conv1d(8, 16, 5, 2), SQUARE, FLATTEN, _fc(944, 5)],
        "samples_per_ct": 8, "sample_stride": 1024, "cts_per_batch": 64,
    },
    "cifar_cnn": {
        "desc": "2D CNN on 3x32x32: conv 3->16 3x3, sq, pool2, conv 16->32 3x3 s2, sq, flatten, FC 1568->10",
        "log_n": 15, "prime_bits": [60] + [40] * 10, "special_bits": 60, "log_scale": 40,
        "input": {"c": 3, "h": 32, "w": 32, "dist": "uniform01"},
        "layers": [_conv(3, 16, 3, 1), SQUARE, _pool(2), _conv(16, 32, 3, 2), SQUARE, FLATTEN,
                   _fc(1568, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
}

# The paper's other model shapes (Section V, Tables of detailed parameters
# for M1 and M3 to M7), with synthetic weights.  M4 is LeNet-5, whose third
# convolution needs a 32 x 32 input (28 x 28 would leave no output); rings
# of 2^15 hold the depth-8 and depth-9 models at a 2^40 scale.
MODEL_CONFIGS = {
    "m1": {
        "desc": "M1: conv 1->8 K4 S3, sq, flatten, FC 648->64, sq, FC 64->10 (28x28)",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01"},
        "layers": [_conv(1, 8, 4, 3), SQUARE, FLATTEN, _fc(648, 64), SQUARE, _fc(64, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "m3": {
        "desc": "M3: conv 1->6 K3, approx ReLU, pool2, flatten, FC 1014->120, approx ReLU, FC 120->10 (28x28)",
        "log_n": 15, "prime_bits": [60] + [40] * 10, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01"},
        "layers": [_conv(1, 6, 3, 1), RELU, _pool(2), FLATTEN, _fc(1014, 120), RELU, _fc(120, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "m4": {
        "desc": "M4 (LeNet-5 with squares): conv 1->6 K5, sq, pool2, conv 6->16 K5, sq, pool2, conv 16->120 K5, "
                "sq, flatten, FC 120->84, sq, FC 84->10 (32x32)",
        "log_n": 15, "prime_bits": [60] + [40] * 10, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 32, "w": 32, "dist": "uniform01"},
        "layers": [_conv(1, 6, 5, 1), SQUARE, _pool(2), _conv(6, 16, 5, 1), SQUARE, _pool(2), _conv(16, 120, 5, 1),
                   SQUARE, FLATTEN, _fc(120, 84), SQUARE, _fc(84, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "m5": {
        "desc": "M5: conv 3->16 K3, sq, pool2, conv 16->64 K4, sq, pool2, conv 64->128 K3, sq, pool4, flatten, "
                "FC 128->10 (3x32x32)",
        "log_n": 15, "prime_bits": [60] + [40] * 10, "special_bits": 60, "log_scale": 40,
        "input": {"c": 3, "h": 32, "w": 32, "dist": "uniform01"},
        "layers": [_conv(3, 16, 3, 1), SQUARE, _pool(2), _conv(16, 64, 4, 1), SQUARE, _pool(2), _conv(64, 128, 3, 1),
                   SQUARE, _pool(4), FLATTEN, _fc(128, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "m6": {
        "desc": "M6: conv 1->6 K4 S2, sq, flatten, FC 294->64, sq, FC 64->10 (16x16)",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 16, "w": 16, "dist": "uniform01"},
        "layers": [_conv(1, 6, 4, 2), SQUARE, FLATTEN, _fc(294, 64), SQUARE, _fc(64, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
    "m7": {
        "desc": "M7: conv1d 1->2 k2 s2, sq, conv1d 2->4 k2 s2, flatten, FC 128->32, sq, FC 32->5 (length 128)",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 1, "w": 128, "dist": "normal"},
        "layers": [_conv1d(1, 2, 2, 2), SQUARE, _conv1d(2, 4, 2, 2), FLATTEN, _fc(128, 32), SQUARE, _fc(32, 5)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
}
CONFIGS.update(MODEL_CONFIGS)

# LeNet-1 with a "same"-padded first convolution (not one of the paper's
# models: the padded-convolution workload).  The sample keeps the padding
# space of Section VI: 2 zero columns per row (pitch 30) and a lead of
# 2 * 30 + 2 zero slots for the rows above the image.
PADDED_CONFIGS = {
    "lenet1_padded": {
        "desc": "LeNet-1 with conv1 padded: conv 1->4 K5 P2, sq, pool2, conv 4->12 K5, sq, pool2, flatten, FC 300->10",
        "log_n": 14, "prime_bits": [60] + [40] * 7, "special_bits": 60, "log_scale": 40,
        "input": {"c": 1, "h": 28, "w": 28, "dist": "uniform01", "pitch": 30, "lead": 62},
        "layers": [dict(_conv(1, 4, 5, 1), pad=2), SQUARE, _pool(2), _conv(4, 12, 5, 1), SQUARE, _pool(2), FLATTEN,
                   _fc(300, 10)],
        "samples_per_ct": 1, "sample_stride": 0, "cts_per_batch": 1,
    },
}
CONFIGS.update(PADDED_CONFIGS)

# Small rings used by unit and parity tests (same shapes of work, tiny N).
TINY_RINGS = {
    "n16": {"log_n": 4, "prime_bits": [50, 40, 40], "special_bits": 50, "log_scale": 30},
    "n64": {"log_n": 6, "prime_bits": [60, 40, 40, 40], "special_bits": 60, "log_scale": 40},
    "n1024": {"log_n": 10, "prime_bits": [60, 40, 40, 40], "special_bits": 60, "log_scale": 40},
}


def config(name: str) -> dict:
    return copy.deepcopy(CONFIGS[name])


def gen_params(layers, seed_w: int = SEED_WEIGHTS, seed_b: int = SEED_BIASES):
    """Weights N(0, 0.1^2) and biases N(0, 0.01^2) for every conv / fc layer,
    in layer order.  Returns a list aligned with `layers` (None for layers
    without parameters)."""
    rw = np.random.default_rng(seed_w)
    rb = np.random.default_rng(seed_b)
    out = []
    for L in layers:
        if L["kind"] == "conv":
            kh = 1 if L.get("dims") == 1 else L["k"]
            w = rw.normal(0.0, 0.1, size=(L["ch_out"], L["ch_in"], kh, L["k"]))
            b = rb.normal(0.0, 0.01, size=(L["ch_out"],))
            out.append((w, b))
        elif L["kind"] == "fc":
            w = rw.normal(0.0, 0.1, size=(L["dout"], L["din"]))
            b = rb.normal(0.0, 0.01, size=(L["dout"],))
            out.append((w, b))
        else:
            out.append(None)
    return out


def gen_inputs(inp: dict, count: int, seed: int = SEED_INPUTS) -> np.ndarray:
    """`count` inputs of shape (C, H, W)."""
    r = np.random.default_rng(seed)
    shape = (count, inp["c"], inp["h"], inp["w"])
    if inp["dist"] == "uniform01":
        return r.uniform(0.0, 1.0, size=shape)
    if inp["dist"] == "normal":
        return r.normal(0.0, 1.0, size=shape)
    raise ValueError(inp["dist"])


def gen_slots(n_slots: int, count: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Plain random real slot vectors, for primitive-level tests."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(count, n_slots))


def poisson_arrivals(rate_per_s: float, n: int, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=n)
    return np.cumsum(gaps)
