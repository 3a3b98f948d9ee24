"""Summaries of rocprofv3 CSV output (kernel statistics, HBM byte counters,
LDS/VALU counters) as short markdown, and the per-launch HBM traffic file
the benchmark reads.

    python -m paper_1309_1114_amd.profsum --ktrace DIR --fetch DIR --write DIR
           [--lds DIR] --workload-key KEY --out-md FILE --out-traffic FILE
           --command "..."

FETCH_SIZE and WRITE_SIZE are in KiB per dispatch.  Each is scaled by the
ratio of the known bytes of the reference copy kernel (an elementwise kernel
reading and writing 1 GiB) to what the same counter reads for it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
from collections import defaultdict

# library kernels by name (templates and plain functions alike)
KERNELS = ("k_count", "k_segsum", "k_binscan", "k_offsets", "k_scatter", "k_items",
           "k_lgcount", "k_lgscan", "k_lgscatter", "k_large", "k_splat", "k_resolve", "k_clear",
           "k_ord_init", "k_ord_project", "k_ord_rank_counts", "k_ord_pass_bounds", "k_ord_emit",
           "k_ord_items", "k_ord_composite", "k_ord_merge", "k_ord_finish",
           # learned upscaler (csrc/nn.hip)
           "k_conv_fwd", "k_conv_bwd_w", "k_flip", "k_pack", "k_head", "k_adam", "k_to_bf16",
           "k_consistency", "k_region_check", "k_sum_partials")
# the ordered render's sort and scan kernels (csrc/sort.hip), summed under
# one name each
SORT_KERNELS = {"k_rs_hist": "radix_sort", "k_rs_scatter": "radix_sort",
                "k_key_range_init": "radix_sort", "k_key_range": "radix_sort",
                "k_key32": "radix_sort", "k_fix_mark": "radix_sort", "k_fix_list": "radix_sort",
                "k_scan_partial": "scan", "k_scan_top": "scan", "k_scan_down": "scan"}
COPY_BYTES = 1 << 30


def short(name):
    for k in KERNELS:
        if f"::{k}<" in name or f"::{k}(" in name:
            return k
    for k, group in SORT_KERNELS.items():
        if f"::{k}<" in name or f"::{k}(" in name:
            return group
    if "elementwise_kernel" in name and "AUnaryFunctor" in name:
        return "copy_ref"          # dst = src * 1 over 1 GiB
    return None


def _find(d, suffix):
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def counters(d):
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(_find(d, "counter_collection.csv"))):
        k = short(r["Kernel_Name"])
        if k:
            vals[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return vals


def kernel_stats(d):
    """Calls, mean ms and share of GPU time per short name; kernels that
    share a name (the several kernels of one library sort) are summed."""
    tot = defaultdict(lambda: [0, 0.0, 0.0])
    for r in csv.DictReader(open(_find(d, "kernel_stats.csv"))):
        k = short(r["Name"])
        if k and k != "copy_ref":
            t = tot[k]
            t[0] += int(r["Calls"])
            t[1] += float(r["TotalDurationNs"])
            t[2] += float(r["Percentage"])
    return {k: dict(calls=c, avg_ms=ns / c / 1e6, pct=pct) for k, (c, ns, pct) in tot.items()}


def code_only(text):
    """C++ source without its comments and with runs of white space made one
    space, so that an edit of comments alone leaves the hash unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                         # string or character literal
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(root):
    """Hash of the code (comments aside) of the render kernels' sources: the
    traffic counters stay valid while it is unchanged."""
    h = hashlib.sha256()
    for f in ("device.h", "kernels.h", "render.hip"):
        with open(os.path.join(root, "paper_1309_1114_amd", "csrc", f), encoding="utf-8") as fh:
            h.update(code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ktrace", required=True)
    ap.add_argument("--fetch", default=None)
    ap.add_argument("--write", default=None)
    ap.add_argument("--lds", default=None)
    ap.add_argument("--workload-key", required=True)
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-traffic", default=None)
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", default="")
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    ks = kernel_stats(a.ktrace)
    have_hbm = a.fetch is not None and a.write is not None
    fe = counters(a.fetch) if have_hbm else {}
    wr = counters(a.write) if have_hbm else {}
    sf = sw = 1.0
    if have_hbm:
        ref_f = statistics.median(fe["copy_ref"]["FETCH_SIZE"]) * 1024
        ref_w = statistics.median(wr["copy_ref"]["WRITE_SIZE"]) * 1024
        sf, sw = COPY_BYTES / ref_f, COPY_BYTES / ref_w
    lines = [f"# {a.title}", "", "Command (rocprofv3 runs, one counter set each):", "",
             "```", a.command, "```", ""]
    if have_hbm:
        lines += [f"Counter scale from the 1 GiB elementwise copy: FETCH x{sf:.4f}, "
                  f"WRITE x{sw:.4f}.", ""]
    lines += ["| kernel | calls | avg ms | % of GPU time | HBM read GB/launch | "
              "HBM write GB/launch |", "|---|---|---|---|---|---|"]
    traffic = {}
    for k in sorted(ks, key=lambda k: -ks[k]["avg_ms"]):
        f = statistics.median(fe[k]["FETCH_SIZE"]) * 1024 * sf if k in fe else None
        w = statistics.median(wr[k]["WRITE_SIZE"]) * 1024 * sw if k in wr else None
        if f is not None and w is not None:
            traffic[k] = dict(read_bytes=round(f), write_bytes=round(w),
                              bytes_per_launch=round(f + w))
        lines.append(f"| {k} | {ks[k]['calls']} | {ks[k]['avg_ms']:.4f} | {ks[k]['pct']:.2f} | "
                     f"{'' if f is None else f'{f / 1e9:.3f}'} | "
                     f"{'' if w is None else f'{w / 1e9:.3f}'} |")
    if a.lds:
        lc = counters(a.lds)
        names = sorted({c for k in lc for c in lc[k]})
        lines += ["", "SQ counters per launch (median over launches):", "",
                  "| kernel | " + " | ".join(names) + " |",
                  "|---|" + "---|" * len(names)]
        for k in sorted(lc):
            if k == "copy_ref":
                continue
            lines.append(f"| {k} | " + " | ".join(
                f"{statistics.median(lc[k][c]):.4g}" if c in lc[k] else "" for c in names) + " |")
    with open(a.out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if not have_hbm:
        print("\n".join(lines))
        return
    allt = {}
    if os.path.exists(a.out_traffic):
        allt = json.load(open(a.out_traffic))
    traffic["source_hash"] = source_hash(root)
    traffic["counter_scale"] = dict(fetch=round(sf, 5), write=round(sw, 5))
    allt[a.workload_key] = traffic
    with open(a.out_traffic, "w") as fh:
        json.dump(allt, fh, indent=1, sort_keys=True)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
