"""Summaries of rocprofv3 CSV output (kernel statistics and memory counters).

    python -m paper_1910_02611_amd.profsum trace DIR/NAME_kernel_stats.csv --title T --cmd C > OUT.md
    python -m paper_1910_02611_amd.profsum traffic --fetch DIR/F_counter_collection.csv \
        --write DIR/W_counter_collection.csv --copy-bytes N --title T --cmd C --json OUT.json > OUT.md
    python -m paper_1910_02611_amd.profsum counters DIR/X_counter_collection.csv --title T --cmd C > OUT.md
    python -m paper_1910_02611_amd.profsum requests --rd DIR/R_counter_collection.csv \
        --wr DIR/W_counter_collection.csv --title T --cmd C --json OUT.json > OUT.md

The requests summary prices the L2-to-memory request counts by their size
(32, 64 and 128 bytes); FETCH_SIZE's own formula counts 128-byte reads as
64 bytes on this GPU, so a streaming read shows at half its size there.
The traffic summary turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch, each
from its own run) into bytes per launch, each scaled by what the counter
reads for the streaming copy kernel of known size (N bytes read and N bytes
written) that the same run launches.  The JSON form carries a hash of the
kernel sources, so a reader can tell whether the kernels changed since.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


def kernel_source_hash() -> str:
    """sha256 over the HIP sources and headers of the library."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def short_name(full: str) -> str:
    """rambo_dev::k_bin_windows_hold<4, 2>(...) -> k_bin_windows_hold<4, 2>"""
    s = re.sub(r"^void ", "", full)
    s = s.replace("(anonymous namespace)::", "")
    s = s.split("(")[0]
    return s.replace("rambo_dev::", "")


def trace_md(path: str, title: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["# %s" % title, "", "Command (from the repository root on the MI355X host):", "", "```", cmd, "```", "",
           "| kernel | calls | total ns | avg ns | % | min ns | max ns |", "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| %s | %s | %d | %d | %.2f | %d | %d |" % (
            short_name(r["Name"]), r["Calls"], int(float(r["TotalDurationNs"])), int(float(r["AverageNs"])),
            float(r["Percentage"]), int(float(r["MinNs"])), int(float(r["MaxNs"]))))
    return "\n".join(out) + "\n"


def per_dispatch(path: str, counter: str) -> dict[str, list[float]]:
    """kernel -> [counter value of each dispatch] (values of one dispatch summed)."""
    acc: dict[tuple[str, str], float] = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        acc[(short_name(r["Kernel_Name"]), r["Dispatch_Id"])] += float(r["Counter_Value"])
    out: dict[str, list[float]] = collections.defaultdict(list)
    for (k, _), v in acc.items():
        out[k].append(v)
    return out


def traffic(fetch_csv: str, write_csv: str, copy_bytes: int) -> dict:
    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    copy = [k for k in fetch if k.startswith("k_copy")]
    if not copy:
        raise SystemExit("no k_copy dispatch in %s: run with --calib-copy-gib" % fetch_csv)
    f_copy = max(fetch[copy[0]]) * 1024.0
    w_copy = max(write[copy[0]]) * 1024.0
    f_scale, w_scale = copy_bytes / f_copy, copy_bytes / w_copy
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, []), write.get(k, [])
        fb = (sum(fv) / len(fv)) * 1024.0 * f_scale if fv else 0.0
        wb = (sum(wv) / len(wv)) * 1024.0 * w_scale if wv else 0.0
        kernels[k] = {"dispatches": max(len(fv), len(wv)), "fetch_bytes": fb, "write_bytes": wb,
                      "bytes": fb + wb}
    return {"copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
            "kernel_source_sha256": kernel_source_hash(), "kernels": kernels}


def traffic_md(t: dict, title: str, cmd: str) -> str:
    out = ["# %s" % title, "", "Commands (from the repository root on the MI355X host):", "", "```", cmd, "```", "",
           "Calibration: a streaming copy of %d bytes (read once, written once) reads FETCH_SIZE x %.3f and "
           "WRITE_SIZE x %.3f of its true bytes; every figure below is scaled by those factors." % (
               t["copy_bytes"], 1 / t["fetch_scale"], 1 / t["write_scale"]), "",
           "Kernel source hash: `%s`" % t["kernel_source_sha256"], "",
           "| kernel | dispatches | HBM read / launch | HBM written / launch | total / launch |",
           "|---|---:|---:|---:|---:|"]
    for k, v in t["kernels"].items():
        out.append("| %s | %d | %.4g B | %.4g B | %.4g B |" % (k, v["dispatches"], v["fetch_bytes"],
                                                            v["write_bytes"], v["bytes"]))
    return "\n".join(out) + "\n"


RD_SIZES = (("TCC_EA0_RDREQ_32B_sum", 32), ("TCC_EA0_RDREQ_64B_sum", 64), ("TCC_EA0_RDREQ_128B_sum", 128))


def requests(rd_csv: str, wr_csv: str) -> dict:
    """Bytes per launch from the L2-to-memory request counts split by size:
    read = 32 n_32B + 64 n_64B + 128 n_128B (TCC_EA0_RDREQ_*_sum, one run),
    written = 32 (n - n_64B) + 64 n_64B (TCC_EA0_WRREQ_sum and _64B_sum,
    another run).  Requests of other sizes show as the difference between
    TCC_EA0_RDREQ_sum and the three sized counts (reported, not priced)."""
    rd = {c: per_dispatch(rd_csv, c) for c, _ in RD_SIZES}
    rd_all = per_dispatch(rd_csv, "TCC_EA0_RDREQ_sum")
    wr_all = per_dispatch(wr_csv, "TCC_EA0_WRREQ_sum")
    wr64 = per_dispatch(wr_csv, "TCC_EA0_WRREQ_64B_sum")
    mean = lambda v: sum(v) / len(v) if v else 0.0
    kernels = {}
    for k in sorted(set(rd_all) | set(wr_all)):
        n = {c: mean(rd[c].get(k, [])) for c, _ in RD_SIZES}
        rb = sum(n[c] * size for c, size in RD_SIZES)
        other = mean(rd_all.get(k, [])) - sum(n.values())
        if abs(other) < 1e-3:   # rounding of the per-launch means, not requests
            other = 0.0
        w_all, w64 = mean(wr_all.get(k, [])), mean(wr64.get(k, []))
        wb = 32.0 * (w_all - w64) + 64.0 * w64
        kernels[k] = {"dispatches": max(len(rd_all.get(k, [])), len(wr_all.get(k, []))),
                      "rd_32B": n[RD_SIZES[0][0]], "rd_64B": n[RD_SIZES[1][0]], "rd_128B": n[RD_SIZES[2][0]],
                      "rd_other": other, "wr": w_all, "wr_64B": w64,
                      "fetch_bytes": rb, "write_bytes": wb, "bytes": rb + wb}
    return {"method": "request counts by size", "kernel_source_sha256": kernel_source_hash(), "kernels": kernels}


def requests_md(t: dict, title: str, cmd: str, probes: str) -> str:
    out = ["# %s" % title, "", "Commands (from the repository root on the MI355X host):", "", "```", cmd, "```", "",
           "Bytes from the L2-to-memory request counters split by size (read = 32 n32 + 64 n64 + 128 n128; "
           "written = 32 (n - n64) + 64 n64), per launch, averaged over the launches of each kernel.  " + probes,
           "", "Kernel source hash: `%s`" % t["kernel_source_sha256"], "",
           "| kernel | launches | rd 32B | rd 64B | rd 128B | rd other | HBM read / launch | wr | wr 64B | "
           "HBM written / launch | total / launch |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k, v in t["kernels"].items():
        out.append("| %s | %d | %.4g | %.4g | %.4g | %.3g | %.4g B | %.4g | %.4g | %.4g B | %.4g B |" % (
            k, v["dispatches"], v["rd_32B"], v["rd_64B"], v["rd_128B"], v["rd_other"], v["fetch_bytes"], v["wr"],
            v["wr_64B"], v["write_bytes"], v["bytes"]))
    return "\n".join(out) + "\n"


def counters_md(path: str, title: str, cmd: str) -> str:
    """Per-kernel averages of every counter in a counter-collection CSV."""
    names = sorted({r["Counter_Name"] for r in csv.DictReader(open(path))})
    vals = {n: per_dispatch(path, n) for n in names}
    kernels = sorted({k for v in vals.values() for k in v})
    out = ["# %s" % title, "", "Command (from the repository root on the MI355X host):", "", "```", cmd, "```", "",
           "Values are per dispatch, averaged over the dispatches of each kernel.", "",
           "| kernel | " + " | ".join(names) + " |", "|---|" + "---:|" * len(names)]
    for k in kernels:
        cells = []
        for n in names:
            v = vals[n].get(k)
            cells.append("%.4g" % (sum(v) / len(v)) if v else "")
        out.append("| %s | %s |" % (k, " | ".join(cells)))
    return "\n".join(out) + "\n"


def load_traffic(path: str) -> dict | None:
    """The traffic summary at path, or None when missing or when the kernel
    sources changed since it was taken."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return t


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("trace")
    a.add_argument("stats_csv")
    a.add_argument("--title", required=True)
    a.add_argument("--cmd", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--title", required=True)
    b.add_argument("--cmd", required=True)
    b.add_argument("--json")
    d = sub.add_parser("requests")
    d.add_argument("--rd", required=True)
    d.add_argument("--wr", required=True)
    d.add_argument("--title", required=True)
    d.add_argument("--cmd", required=True)
    d.add_argument("--probes", default="")
    d.add_argument("--json")
    c = sub.add_parser("counters")
    c.add_argument("counter_csv")
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", required=True)
    args = ap.parse_args()
    if args.what == "trace":
        sys.stdout.write(trace_md(args.stats_csv, args.title, args.cmd))
    elif args.what == "counters":
        sys.stdout.write(counters_md(args.counter_csv, args.title, args.cmd))
    elif args.what == "requests":
        t = requests(args.rd, args.wr)
        if args.json:
            with open(args.json, "w") as f:
                json.dump(t, f, indent=1)
        sys.stdout.write(requests_md(t, args.title, args.cmd, args.probes))
    else:
        t = traffic(args.fetch, args.write, args.copy_bytes)
        if args.json:
            with open(args.json, "w") as f:
                json.dump(t, f, indent=1)
        sys.stdout.write(traffic_md(t, args.title, args.cmd))


if __name__ == "__main__":
    main()
