"""Summarise rocprofv3 CSV output of bench.py runs into short text profiles.

  python -m paper_1407_7370_amd.rocprof_summary --stats DIR/trace_kernel_stats.csv \
      [--fetch DIR/fetch_counter_collection.csv --write DIR/write_counter_collection.csv] \
      [--calib-mib N] [--traffic-json profiles/traffic_recur_laser4096.json] [--command "..."] \
      [--sq DIR/sq_counter_collection.csv] [--counters DIR/x_counter_collection.csv ...]

Kernel statistics: calls and average duration per kernel.  Counters: HBM read
and write bytes per dispatch from FETCH_SIZE / WRITE_SIZE (KiB), each scaled
by what the same counter reads for calibration kernels of known size that
bench.py --copy-calib-mib N runs: torch's fill of N MiB (writes N MiB) and
torch's neg of N MiB (reads N MiB, writes N MiB).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def short_name(n: str) -> str:
    n = n.replace("void ", "").replace("dl::(anonymous namespace)::", "")
    n = n.replace("HIP_vector_type<double, 2u>", "c128").replace("HIP_vector_type<float, 2u>", "c64")
    n = n.replace("dl::(anonymous namespace)::", "")
    return n


def kernel_class(n: str):
    """Map a kernel name to (family, precision) of the propagator."""
    if "k_recur<" in n:
        body = n[n.index("k_recur<"):]
        prec = "mixed" if "float, 2u" in n else "fp64"
        general = body.count("Paired") >= 2
        return ("recur_basis" if general else "recur_psi", prec)
    for fam in ("k_first", "k_tridiag", "k_combine", "k_apply", "k_reset"):
        if fam in n:
            prec = "mixed" if "float, 2u" in n else ("fp64" if fam == "k_combine" else "-")
            return (fam, prec)
    return (None, None)


def read_stats(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append(dict(name=r["Name"], calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                        total_ms=float(r["TotalDurationNs"]) / 1e6, pct=float(r["Percentage"])))
    return out


def read_counter(path, counter):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in d.items()}


def find(d, needle):
    for k, v in d.items():
        if needle in k:
            return v
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-mib", type=int, default=1024)
    ap.add_argument("--traffic-json")
    ap.add_argument("--sites", type=int, default=4096 * 4096)
    ap.add_argument("--command", default="")
    ap.add_argument("--sq", help="counter CSV of SQ_WAVES, SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_BUSY_CYCLES")
    ap.add_argument("--counters", action="append", default=[],
                    help="counter CSV of any other pass: mean value per dispatch of each counter, per kernel")
    ap.add_argument("--dispatches", nargs=2, metavar=("TRACE_CSV", "NAME"),
                    help="every dispatch of the kernels whose name contains NAME: grid size and duration")
    ap.add_argument("--clock-ghz", type=float, default=2.4)
    ap.add_argument("--simds", type=int, default=1024)
    args = ap.parse_args()

    lines = []
    if args.command:
        lines.append("commands:")
        for c in args.command.split(" ;; "):
            lines.append("  " + c)
        lines.append("")
    st = read_stats(args.stats)
    lines.append(f"{'kernel':78s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'%':>6s}")
    for r in sorted(st, key=lambda x: -x["total_ms"]):
        if "dl::" not in r["name"] and r["pct"] < 0.5:
            continue
        lines.append(f"{short_name(r['name'])[:78]:78s} {r['calls']:6d} {r['avg_us']:10.2f} "
                     f"{r['total_ms']:10.3f} {r['pct']:6.2f}")
    # calibration kernels of known traffic, timed in the same trace: the
    # practical streaming bandwidth of the device
    mib = args.calib_mib * (1 << 20)
    for r in st:
        if "neg_kernel" in r["name"]:
            lines.append(f"calibration torch.neg ({args.calib_mib} MiB read + write): {r['avg_us']:.1f} us = "
                         f"{2 * mib / (r['avg_us'] * 1e-6) / 1e9:.0f} GB/s")
        elif "FillFunctor" in r["name"]:
            lines.append(f"calibration torch.fill ({args.calib_mib} MiB write): {r['avg_us']:.1f} us = "
                         f"{mib / (r['avg_us'] * 1e-6) / 1e9:.0f} GB/s")
    traffic = {}
    if args.fetch and args.write:
        fetch = read_counter(args.fetch, "FETCH_SIZE")
        write = read_counter(args.write, "WRITE_SIZE")
        calib = args.calib_mib * 1024.0  # KiB
        f_neg = find(fetch, "neg_kernel")
        w_fill = find(write, "FillFunctor")
        rf = f_neg / calib if f_neg else None
        wf = w_fill / calib if w_fill else None
        lines.append("")
        lines.append(f"calibration: FETCH_SIZE(neg of {args.calib_mib} MiB) = {f_neg} KiB -> read factor "
                     f"{rf}; WRITE_SIZE(fill of {args.calib_mib} MiB) = {w_fill} KiB -> write factor {wf}")
        lines.append(f"{'kernel':78s} {'read_MB':>10s} {'write_MB':>10s} {'B/site':>8s}")
        for k in sorted(fetch):
            if "dl::" not in k:
                continue
            rd = fetch[k] * 1024 / (rf or 1.0)
            wr = write.get(k, 0.0) * 1024 / (wf or 1.0)
            lines.append(f"{short_name(k)[:78]:78s} {rd / 1e6:10.1f} {wr / 1e6:10.1f} "
                         f"{(rd + wr) / args.sites:8.2f}")
            fam, prec = kernel_class(k)
            # the dominant sweep of the benchmark grid: the largest of its kind
            if fam == "recur_basis" and rd + wr > traffic.get(prec, {}).get("bytes_per_launch", 0.0):
                traffic[prec] = {"bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                                 "kernel": short_name(k)}
    if args.sq:
        # instruction mix per kernel: VALU issue utilisation = wave-instructions /
        # (SIMDs x duration / 4 cycles per wave64 instruction)
        sq = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(args.sq)):
            sq[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        dur = {r["name"]: r["avg_us"] for r in st}
        lines.append("")
        lines.append(f"{'kernel':78s} {'waves':>7s} {'VALU_M':>8s} {'SALU_M':>8s} {'VALU_util':>9s}")
        for k in sorted(sq):
            if "dl::" not in k or k not in dur:
                continue
            a = {c: sum(v) / len(v) for c, v in sq[k].items()}
            cap = args.simds * dur[k] * 1e-6 * args.clock_ghz * 1e9 / 4.0
            lines.append(f"{short_name(k)[:78]:78s} {a.get('SQ_WAVES', 0):7.0f} {a.get('SQ_INSTS_VALU', 0) / 1e6:8.1f} "
                         f"{a.get('SQ_INSTS_SALU', 0) / 1e6:8.1f} {a.get('SQ_INSTS_VALU', 0) / cap * 100:8.1f}%")
    for path in args.counters:
        cs = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            cs[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        names = sorted({c for k in cs for c in cs[k]})
        lines.append("")
        lines.append(f"{'kernel':78s} " + " ".join(f"{c:>22s}" for c in names) + "   (mean per dispatch)")
        for k in sorted(cs):
            if "dl::" not in k:
                continue
            vals = [sum(cs[k][c]) / len(cs[k][c]) if cs[k][c] else 0.0 for c in names]
            lines.append(f"{short_name(k)[:78]:78s} " + " ".join(f"{v:22.0f}" for v in vals))
    if args.dispatches:
        path, needle = args.dispatches
        lines.append("")
        lines.append(f"dispatches of {needle}: grid (work-items), workgroup, duration")
        for r in csv.DictReader(open(path)):
            if needle not in r.get("Kernel_Name", ""):
                continue
            dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
            lines.append(f"  grid {r.get('Grid_Size_X', r.get('Grid_Size', '?')):>8s}  workgroup "
                         f"{r.get('Workgroup_Size_X', r.get('Workgroup_Size', '?')):>5s}  {dur:12.2f} us")
    text = "\n".join(lines)
    print(text)
    if args.traffic_json and traffic:
        h = hashlib.sha256()
        for name in ("kernels.hip", "sweeps.h", "device_reduce.h", "dl_internal.h"):
            with open(os.path.join(HERE, "csrc", name), "rb") as f:
                h.update(f.read())
        traffic["kernels_sha256"] = h.hexdigest()
        traffic["note"] = ("HBM bytes per launch of the dominant sweep from rocprofv3 FETCH_SIZE/WRITE_SIZE, "
                           "scaled by the calibration kernels; valid only for this digest of kernels.hip, "
                           "sweeps.h, device_reduce.h and dl_internal.h")
        with open(args.traffic_json, "w") as f:
            json.dump(traffic, f, indent=1)


if __name__ == "__main__":
    main()
