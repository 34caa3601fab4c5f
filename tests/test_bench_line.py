"""Host-side checks of bench.py: the compact result line stays short enough
for a log reader that keeps the last few KB of stdout, carries the fields
the benchmark contract names, and the benchmark's own FP64 forward pass
(used for max_abs_err_vs_fp64) equals the oracle's FP64 CNN on every
workload shape."""
from __future__ import annotations

import json

import numpy as np
import pytest

import bench
import workloads as W
from oracle.network import cnn_fp64

HEAD_LIMIT = 3000


def _fake_full_result() -> dict:
    fams = {f: {"launches_per_step": 12.0, "ms_per_step": 0.123, "avg_us": 10.2, "gbs": 2000.1, "hbm_frac": 0.25,
                "g_butterflies_per_s": 500.0, "alu_frac": 0.24}
            for f in ["ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col", "modup", "ks_inner", "moddown",
                      "rescale", "mac", "automorphism", "tensor", "add", "encode", "other", "ks_rowfused"]}
    tuning = {"ntt_split": 6, "ntt_tile_log": 11, "mac_min_wg": 2048, "ks_min_wg": 1024, "ks_group": 64,
              "ks_order": 2, "ntt_ms": 0.1234567, "net_ms": 3.456789}
    dist = {"reps": 30, "mean_ms": 3.5612, "std_ms": 0.0123, "p50_ms": 3.5601, "p99_ms": 3.6312}
    rf = {"bound": "hbm", "kernel": "ks_rowfused", "achieved": 3281.3, "peak": 8000.0, "unit": "GB/s", "frac": 0.4102,
          "traffic": 273821782, "launches": 160, "avg_us": 138.917, "bytes_per_launch": 319052176,
          "alu_frac": 0.3371, "traffic_over_algorithmic": 0.8582}
    batched = {"images_per_s": 6434.12, "ms_per_launch": 198.94, "launches_timed": 5, "launch_distribution":
               dict(dist, reps=5), "per_launch": 1280, "plan": "deferred ModDown + doubling FC sum",
               "max_abs_err_vs_fp64": 2.9e-07, "tuning": tuning, "kernel_families": fams, "roofline": rf,
               "multiple_of_plain": 22.91}
    levels = {str(f): {"completed": 10000, "seconds": 33.1, "throughput_per_s": 302.2, "p50_ms": 7.312,
                       "p99_ms": 40.123, "batches": 4000, "max_host_queue": 2,
                       "per_model": {m: {"n": 3000, "p50_ms": 5.0, "p99_ms": 30.0}
                                     for m in ("conv1", "cnn1d", "cifar_cnn")}, "offered_requests_per_s": 302.5}
              for f in (0.5, 0.8, 1.0)}
    sweep = {f"N=2^{a},limbs={b}": {"single_per_s": 13392.1, "hoisted24_per_s": 40123.4, "batched128_per_s": 98765.4,
                                    "key_mb": 18.87} for a, b in bench.ROT_SIZES}
    res = {
        "metric": "encrypted LeNet-1-shape inferences/s, batched vs plain; rotations/s; p99 latency",
        "value": 281.234, "unit": "inferences/s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": 3.556,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic, seeded: U[0,1] 28x28 images, weights N(0,0.1^2), biases N(0,0.01^2)",
        "config": {"workload": "plain LeNet-1 shape (conv 1->4 K5, sq, pool2, conv 4->12 K5, sq, pool2, flatten, "
                               "FC 192->10), CKKS N=2^14, primes 60+7x40 (+60 special), scale 2^40, one image per "
                               "ciphertext, one key switch per rotation, one HIP graph per inference"},
        "max_abs_err_vs_fp64": 1.28e-07, "tuning": tuning, "roofline": rf, "kernel_families": fams,
        "plain_step_distribution": dist, "plain_hoisted_inferences_per_s": 360.2,
        "plain_variants": {v: {"inferences_per_s": 294.0, "kernel_families": fams, "tuning": tuning}
                           for v, _, _ in bench.PLAN_VARIANTS},
        "rotations_per_s": 13392.1, "rotation_sweep": sweep,
        "batched": batched, "batched_variant": batched,
        "batched_cnn1d": dict(batched, sequences_per_s=4267.1), "batched_cnn1d_variant": dict(batched,
                                                                                             sequences_per_s=7052.3),
        "serving": {"models": {}, "plan": "deferred ModDown + doubling FC sum", "mix": {}, "arrival_seed": 4,
                    "hbm_budget_bytes": 233000000000, "requests_per_level": 10000,
                    "saturation_requests_per_s": 605.12, "load_levels": levels},
        "cpu_baseline": {"value": 0.06123, "unit": "inferences/s", "cores": 1, "kind": "oracle",
                         "sample": "LeNet-1 shape, N=2^14, 8 limbs, 288 rotations: median of 5 whole encrypted "
                                   "inferences, each one thread in its own process, the 5 side by side",
                         "nproc": 128, "cores_available": 16, "cpu_model": "AMD EPYC 9575F 64-Core Processor",
                         "conv1_median_s": 1.234, "conv1_runs_s": [1.2, 1.3, 1.2, 1.25, 1.22],
                         "lenet1_median_s": 16.3, "lenet1_runs_s": [16.1, 16.3, 16.5, 16.2, 16.4],
                         "batched": {"images_per_s": 9.81, "processes": 16, "ciphertexts": 16, "images": 160,
                                     "slowest_s": 16.3, "fastest_s": 15.9}, "leg_wall_s": 80.1},
        "detail_path": "/tmp/unihenn_bench_detail.json",
    }
    for k in ("batched_cnn1d", "batched_cnn1d_variant"):
        res[k].pop("images_per_s")
        res[k].pop("multiple_of_plain")
    return res


def test_headline_is_short_and_complete():
    head = bench.headline(_fake_full_result())
    line = json.dumps(head)
    assert len(line) <= HEAD_LIMIT, len(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in head, k
    assert "workload" in head["config"]
    assert head["batched"]["multiple_of_plain"] == 22.91
    assert head["serving"]["p50_p99_ms"]["1.0"] == [7.312, 40.123]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in head["roofline"]
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in head["cpu_baseline"]
    # the full result itself would not fit
    assert len(json.dumps(_fake_full_result())) > 4 * HEAD_LIMIT


def test_headline_of_a_plain_only_run():
    res = _fake_full_result()
    plain = {k: res[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                 "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                                 "max_abs_err_vs_fp64", "tuning")}
    head = bench.headline(plain)
    assert head["value"] == res["value"] and "roofline" not in head


def test_roofline_entry_is_hbm_on_algorithmic_bytes():
    stats = {"ks_rowfused": (160, 160 * 0.139, 160 * 3.19e8, 160 * 1e8), "mac": (20, 20 * 0.22, 20 * 1e9, 0.0)}
    rf = bench.roofline_entry(stats)
    assert rf["kernel"] == "ks_rowfused" and rf["bound"] == "hbm" and rf["unit"] == "GB/s"
    assert rf["achieved"] == pytest.approx(3.19e8 / 139e-6 / 1e9, rel=1e-3)
    assert rf["frac"] == pytest.approx(rf["achieved"] / 8000.0, rel=1e-3)
    assert 0 < rf["alu_frac"] < 1


@pytest.mark.parametrize("name", sorted(W.CONFIGS))
def test_bench_fp64_forward_equals_oracle_fp64(name):
    cfg = W.config(name)
    params = W.gen_params(cfg["layers"])
    xs = W.gen_inputs(cfg["input"], 2)
    for x in xs:
        ref = np.asarray(cnn_fp64(x, cfg["layers"], params)).reshape(-1)
        got = bench._fp64_cnn(x, cfg["layers"], params)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
