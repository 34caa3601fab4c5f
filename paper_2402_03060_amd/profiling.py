"""Summaries of rocprofv3 CSV output (kernel statistics and HBM counters).

    python -m paper_2402_03060_amd.profiling stats <kernel_stats.csv> --title T --command C -o out.txt
    python -m paper_2402_03060_amd.profiling traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes B --kernel SUBSTR \
        --bytes-per-item 64 --family ntt_fwd_row --source csrc/ntt.hip --title T --command C -o out.txt

`traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of one kernel into
bytes, calibrated by what the same counters read for plain device copies of
known size, and compares them with the kernel's algorithmic bytes: Grid_Size
work-items times the bytes each work-item reads (and writes) once.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def kernel_stats_summary(path: str, title: str, command: str, top: int = 40) -> str:
    rows = _rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", f"# command: {command}", "# durations in ns",
           "name | calls | total_ns | avg_ns | percent"]
    for r in rows[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "")
        name = name.split("(unsigned long")[0].split("(DevCtx")[0]
        out.append(f"{name} | {r['Calls']} | {r['TotalDurationNs']} | {float(r['AverageNs']):.1f} | "
                   f"{float(r['Percentage']):.2f}")
    return "\n".join(out) + "\n"


def _counter_sum(path: str, counter: str, substr: str):
    n, kib, items = 0, 0.0, 0
    for r in _rows(path):
        if r["Counter_Name"] != counter or substr not in r["Kernel_Name"]:
            continue
        n += 1
        kib += float(r["Counter_Value"])
        items += int(r["Grid_Size"])
    return n, kib, items


def traffic_summary(fetch: str, write: str, copy_fetch: str, copy_write: str, copy_bytes: int, kernel: str,
                    bytes_per_item: int, family: str, source: str, title: str, command: str) -> str:
    cn_f, cf_kib, _ = _counter_sum(copy_fetch, "FETCH_SIZE", "copyBuffer")
    cn_w, cw_kib, _ = _counter_sum(copy_write, "WRITE_SIZE", "copyBuffer")
    # the largest copies dominate; scale = true KiB per copy / counted KiB per copy
    true_kib = copy_bytes / 1024.0
    big_f = [float(r["Counter_Value"]) for r in _rows(copy_fetch)
             if r["Counter_Name"] == "FETCH_SIZE" and "copyBuffer" in r["Kernel_Name"]]
    big_w = [float(r["Counter_Value"]) for r in _rows(copy_write)
             if r["Counter_Name"] == "WRITE_SIZE" and "copyBuffer" in r["Kernel_Name"]]
    big_f = sorted(big_f)[-3:]
    big_w = sorted(big_w)[-3:]
    fetch_scale = true_kib / (sum(big_f) / len(big_f))
    write_scale = true_kib / (sum(big_w) / len(big_w))
    nf, f_kib, items_f = _counter_sum(fetch, "FETCH_SIZE", kernel)
    nw, w_kib, items_w = _counter_sum(write, "WRITE_SIZE", kernel)
    if not nf or not nw:
        raise SystemExit(f"no dispatches of {kernel!r} in the counter files")
    read_b = f_kib * 1024 * fetch_scale
    write_b = w_kib * 1024 * write_scale
    alg_r = items_f * bytes_per_item
    alg_w = items_w * bytes_per_item
    sha = hashlib.sha256(open(source, "rb").read()).hexdigest()
    lines = [
        f"# {title}",
        f"# command: {command}",
        f"# calibration: FETCH_SIZE / WRITE_SIZE of device copies of {copy_bytes} bytes",
        f"kernel = {kernel}",
        f"family = {family}",
        f"copy_true_kib = {true_kib:.0f}",
        f"copy_fetch_kib_mean = {sum(big_f) / len(big_f):.2f}",
        f"copy_write_kib_mean = {sum(big_w) / len(big_w):.2f}",
        f"fetch_scale = {fetch_scale:.4f}",
        f"write_scale = {write_scale:.4f}",
        f"dispatches = {nf}",
        f"measured_read_bytes_per_dispatch = {read_b / nf:.1f}",
        f"measured_write_bytes_per_dispatch = {write_b / nw:.1f}",
        f"algorithmic_read_bytes_per_dispatch = {alg_r / nf:.1f}",
        f"algorithmic_write_bytes_per_dispatch = {alg_w / nw:.1f}",
        f"read_over_algorithmic = {read_b / alg_r:.4f}",
        f"write_over_algorithmic = {write_b / alg_w:.4f}",
        f"source = {os.path.basename(source)}",
        f"source_sha256 = {sha}",
    ]
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("-o", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "kernel", "family", "source", "title", "command"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--bytes-per-item", type=int, required=True)
    t.add_argument("-o", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        text = kernel_stats_summary(a.csv, a.title, a.command)
    else:
        text = traffic_summary(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.kernel,
                               a.bytes_per_item, a.family, a.source, a.title, a.command)
    with open(a.o, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
