"""Summaries of rocprofv3 CSV output (kernel statistics and HBM counters).

    python -m paper_2402_03060_amd.profiling stats <kernel_stats.csv> --title T --command C -o out.txt
    python -m paper_2402_03060_amd.profiling busy <counter_collection.csv> --title T --command C -o out.txt
    python -m paper_2402_03060_amd.profiling traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes B --family ks_inner \
        --bench-json bench.json --evals 3 --title T --command C -o out.txt

`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of one kernel
family into bytes per launch, calibrated by what the same counters read for
plain device copies of known size, and compares them with the family's
algorithmic bytes per launch from the library's own launch statistics.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re

# kernel-name patterns of each family of the library's launch statistics
FAMILY_KERNELS = {
    "ntt_fwd_col": r"k_ntt_r8<\d+, \d+, true, false, false>|k_ntt_fwd<true",
    "ntt_fwd_row": r"k_ntt_r8<\d+, \d+, false, false, true>|k_ntt_fwd<false",
    "ntt_inv_row": r"k_ntt_r8<\d+, \d+, false, true, false>|k_intt_r8_gather<|k_ntt_inv<false",
    "ntt_inv_col": r"k_ntt_r8<\d+, \d+, true, true, true>|k_ntt_inv<true",
    "modup": r"k_ntt_r8_lift<\d+, \d+, 2>|k_modup",
    "ks_inner": r"k_group_inner<|k_ks_inner<|k_ntt_r8_ksrow<",
    "ks_rowfused": r"k_ks_rowmix<|k_ks_rowfp<",
    "moddown": r"k_ntt_r8_lift<\d+, \d+, 0>|k_ntt_r8_finish<\d+, \d+, 0>|k_relin_combine|k_group_sub_scale\(",
    "rescale": r"k_ntt_r8_lift<\d+, \d+, 1>|k_ntt_r8_finish<\d+, \d+, 1>|k_group_sub_scale2",
    "mac": r"k_mac_multi<|k_mac<|k_mac_group<",
    "add": r"k_group_add|k_add\(|k_add_plain",
}


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_stats_summary(path: str, title: str, command: str, top: int = 40) -> str:
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", f"# command: {command}", "# durations in ns",
           "name | calls | total_ns | avg_ns | percent"]
    for r in rows[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        depth, cut = 0, len(name)
        for i, ch in enumerate(name):        # drop the parameter list
            if ch == "<":
                depth += 1
            elif ch == ">":
                depth -= 1
            elif ch == "(" and depth == 0:
                cut = i
                break
        out.append(f"{name[:cut]} | {r['Calls']} | {r['TotalDurationNs']} | {float(r['AverageNs']):.1f} | "
                   f"{float(r['Percentage']):.2f}")
    return "\n".join(out) + "\n"


def _counter_sum(path: str, counter: str, pattern: str):
    rx = re.compile(pattern)
    n, kib = 0, 0.0
    for r in _rows(path):
        if r["Counter_Name"] != counter or not rx.search(r["Kernel_Name"]):
            continue
        n += 1
        kib += float(r["Counter_Value"])
    return n, kib


def source_digest(csrc: str) -> str:
    """SHA-256 over every kernel source file (sorted names and contents)."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def _copy_scale(path: str, counter: str, true_kib: float) -> tuple:
    vals = sorted(float(r["Counter_Value"]) for r in _rows(path)
                  if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"])[-3:]
    mean = sum(vals) / len(vals)
    return true_kib / mean, mean


def traffic_summary(fetch: str, write: str, copy_fetch: str, copy_write: str, copy_bytes: int, family: str,
                    bench_json: str, evals: int, csrc: str, title: str, command: str) -> str:
    """HBM bytes per launch of one kernel family: FETCH_SIZE and WRITE_SIZE
    summed over the family's dispatches, each counter scaled by what it reads
    for device copies of known size, divided by the launches of `evals`
    evaluations (launches per evaluation from the bench JSON's family table
    of the same code), against the family's algorithmic bytes per launch
    from the same table."""
    true_kib = copy_bytes / 1024.0
    fscale, fmean = _copy_scale(copy_fetch, "FETCH_SIZE", true_kib)
    wscale, wmean = _copy_scale(copy_write, "WRITE_SIZE", true_kib)
    pat = FAMILY_KERNELS[family]
    nf, f_kib = _counter_sum(fetch, "FETCH_SIZE", pat)
    nw, w_kib = _counter_sum(write, "WRITE_SIZE", pat)
    if not nf or not nw:
        raise SystemExit(f"no dispatches of family {family!r} in the counter files")
    with open(bench_json) as f:
        fam = json.load(f)["kernel_families"][family]
    launches = fam["launches_per_step"] * evals
    alg = fam["gbs"] * 1e9 * fam["avg_us"] * 1e-6       # algorithmic bytes per launch
    read_b = f_kib * 1024 * fscale / launches
    write_b = w_kib * 1024 * wscale / launches
    lines = [
        f"# {title}",
        f"# command: {command}",
        f"# calibration: FETCH_SIZE / WRITE_SIZE of device copies of {copy_bytes} bytes",
        f"family = {family}",
        f"kernels = {pat}",
        f"copy_true_kib = {true_kib:.0f}",
        f"copy_fetch_kib_mean = {fmean:.2f}",
        f"copy_write_kib_mean = {wmean:.2f}",
        f"fetch_scale = {fscale:.4f}",
        f"write_scale = {wscale:.4f}",
        f"dispatches = {nf}",
        f"launches = {launches:.0f}",
        f"measured_read_bytes_per_launch = {read_b:.1f}",
        f"measured_write_bytes_per_launch = {write_b:.1f}",
        f"measured_bytes_per_launch = {read_b + write_b:.1f}",
        f"algorithmic_bytes_per_launch = {alg:.1f}",
        f"measured_over_algorithmic = {(read_b + write_b) / alg:.4f}",
        f"source_sha256 = {source_digest(csrc)}",
    ]
    return "\n".join(lines) + "\n"


def busy_summary(path: str, title: str, command: str) -> str:
    """Per kernel (and per family): dispatches and the mean of each derived
    counter (VALUBusy, OccupancyPercent) over its dispatches."""
    per = {}
    for r in _rows(path):
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").replace("void ", "")
        cut = name.find("(")
        name = name[:cut] if cut > 0 else name
        d = per.setdefault(name, {})
        d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    counters = sorted({c for d in per.values() for c in d})
    out = [f"# {title}", f"# command: {command}",
           "# mean over dispatches; VALUBusy: percent of GPU time the vector ALUs issue; OccupancyPercent: resident "
           "waves against the maximum", "kernel | dispatches | " + " | ".join(counters)]
    for name, d in sorted(per.items(), key=lambda kv: -len(kv[1].get(counters[0], []))):
        n = len(d[counters[0]])
        if name.startswith("__amd"):
            continue
        out.append(f"{name} | {n} | " + " | ".join(f"{sum(d[c]) / len(d[c]):.1f}" for c in counters))
    fam = [f"family {f}: " + ", ".join(
        f"{c} {sum(sum(d[c]) for k, d in per.items() if re.search(p, k)) / max(1, sum(len(d[c]) for k, d in per.items() if re.search(p, k))):.1f}"
        for c in counters) for f, p in FAMILY_KERNELS.items() if any(re.search(p, k) for k in per)]
    return "\n".join(out + ["# per family (mean over its dispatches)"] + fam) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("-o", required=True)
    b = sub.add_parser("busy")
    b.add_argument("csv")
    b.add_argument("--title", required=True)
    b.add_argument("--command", required=True)
    b.add_argument("-o", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "family", "bench-json", "title", "command"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--evals", type=int, required=True, help="evaluations the counted run made")
    t.add_argument("--csrc", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc"))
    t.add_argument("-o", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        text = kernel_stats_summary(a.csv, a.title, a.command)
    elif a.cmd == "busy":
        text = busy_summary(a.csv, a.title, a.command)
    else:
        text = traffic_summary(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.family, a.bench_json,
                               a.evals, a.csrc, a.title, a.command)
    with open(a.o, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
