"""rocprofv3 output of bench.py runs -> the measured figures bench.py reports.

Two products:

* a kernel-time summary (markdown) from ``rocprofv3 --kernel-trace --stats``;
* a traffic record: the HBM bytes one launch of a kernel moves, from two
  ``rocprofv3 --pmc`` passes (FETCH_SIZE, then WRITE_SIZE, KiB per
  dispatch), each divided by the factor the same counter shows for a plain
  device copy of known size (``bench.py --copy-calibration``).

The traffic record carries the SHA-256 of the kernel's source file; bench.py
reports ``traffic: null`` when the source no longer matches.

Command line::

    python -m paper_2310_14133_amd.profiling stats STATS.csv --command CMD --out F.md
    python -m paper_2310_14133_amd.profiling traffic --kind KIND \
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \
        --copy-bytes N --command CMD... --out TRAFFIC.json
"""
import argparse
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel kind (the library's timing table) -> (kernel symbol, source file)
KIND_KERNELS = {
    "huffman_decode": ("k_huff_decode", "csrc/kernels_decode.hip"),
    "huffman_encode": ("k_huff_encode", "csrc/kernels_huff.hip"),
    "huffman_count": ("k_huff_count", "csrc/kernels_huff.hip"),
    "histogram": ("k_hist", "csrc/kernels_huff.hip"),
    "row_comp_level1": ("k_row_comp", "csrc/kernels_sweep.hip"),
    "row_decomp_level1": ("k_row_decomp", "csrc/kernels_sweep.hip"),
    "sweep_comp": ("k_sweep_comp", "csrc/kernels_sweep.hip"),
    "sweep_decomp": ("k_sweep_decomp", "csrc/kernels_sweep.hip"),
    "check_range": ("k_range", "csrc/kernels_metrics.hip"),
    "tune_alg1": ("k_alg1_level", "csrc/kernels_tune.hip"),
    "tune_trial": ("k_trial", "csrc/kernels_tune.hip"),
}
COPY_KERNEL = "copyBuffer"


def source_digest(kind):
    """SHA-256 of the source file holding the kernel of `kind`."""
    rel = KIND_KERNELS[kind][1]
    with open(os.path.join(HERE, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _short(name):
    return name.split("(")[0].replace("void ", "")


def kernel_stats(path):
    """Rows of a --stats kernel summary: (name, calls, avg_ns, total_ns)."""
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            out.append((_short(r["Name"]), int(r["Calls"]),
                        float(r["AverageNs"]), float(r["TotalDurationNs"])))
    return out


def counter_mean(path, kernel, counter):
    """Mean over dispatches of `kernel` (substring of the name) of the
    counter's per-dispatch total."""
    per = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel not in r["Kernel_Name"] or r["Counter_Name"] != counter:
                continue
            d = r["Dispatch_Id"]
            per[d] = per.get(d, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernel {kernel} in {path}")
    return sum(per.values()) / len(per), len(per)


def stats_markdown(stats_csv, command, top=16):
    rows = sorted(kernel_stats(stats_csv), key=lambda r: -r[3])
    lines = ["| kernel | calls | avg us | total ms |", "|---|---:|---:|---:|"]
    for name, calls, avg, tot in rows[:top]:
        lines.append(f"| {name} | {calls} | {avg / 1e3:.1f} | "
                     f"{tot / 1e6:.3f} |")
    return ("Command (from the repository root on the GPU host):\n\n"
            f"    {command}\n\n" + "\n".join(lines) + "\n")


def traffic_record(kind, fetch, write, copy_fetch, copy_write, copy_bytes,
                   commands):
    kern = KIND_KERNELS[kind][0]
    f_kib, nf = counter_mean(fetch, kern, "FETCH_SIZE")
    w_kib, nw = counter_mean(write, kern, "WRITE_SIZE")
    cf_kib, _ = counter_mean(copy_fetch, COPY_KERNEL, "FETCH_SIZE")
    cw_kib, _ = counter_mean(copy_write, COPY_KERNEL, "WRITE_SIZE")
    sf = cf_kib * 1024.0 / copy_bytes
    sw = cw_kib * 1024.0 / copy_bytes
    return {
        "kind": kind,
        "kernel": kern,
        "source": KIND_KERNELS[kind][1],
        "source_sha256": source_digest(kind),
        "fetch_kib_per_launch": f_kib,
        "write_kib_per_launch": w_kib,
        "dispatches": [nf, nw],
        "copy_bytes": copy_bytes,
        "copy_fetch_scale": sf,
        "copy_write_scale": sw,
        "bytes_per_launch": f_kib * 1024.0 / sf + w_kib * 1024.0 / sw,
        "commands": commands,
    }


def load_traffic(path, kind):
    """Measured bytes per launch of `kind`, or None when there is no record
    or the kernel's source changed since it was measured."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kind)
    if not rec or kind not in KIND_KERNELS:
        return None
    if rec.get("source_sha256") != source_digest(kind):
        return None
    return rec["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kind", required=True)
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        with open(a.out, "w") as f:
            f.write(stats_markdown(a.csv, a.command))
    else:
        rec = traffic_record(a.kind, a.fetch, a.write, a.copy_fetch,
                             a.copy_write, a.copy_bytes, a.command)
        data = {}
        if os.path.exists(a.out):
            with open(a.out) as f:
                data = json.load(f)
        data[a.kind] = rec
        with open(a.out, "w") as f:
            json.dump(data, f, indent=1)
            f.write("\n")
        print(json.dumps(rec))


if __name__ == "__main__":
    main()
