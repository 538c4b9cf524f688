"""Short text summaries of rocprofv3 CSV output (kernel traces and hardware
counters), as kept next to the benchmark results.

  python -m paper_2103_02903_amd.profiling stats --trace T.csv --match k_transport_collide --match "double>" \
      --skip 100 --take 1000 --command "..." --out profiles/NAME.txt
  python -m paper_2103_02903_amd.profiling counters --fetch F.csv --write W.csv --copy-fetch CF.csv \
      --copy-write CW.csv --match ... --skip 100 --take 1000 --workload NAME --precision 8 \
      --command "..." --out profiles/NAME_counters.json

Counter values are KiB per dispatch. They are converted to bytes with the ratio
between what the same counter reads for the library's plain copy kernel
(k_copy_u4 over a known number of bytes) and that number.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2103_02903_amd/csrc/mr_kernels.h", "paper_2103_02903_amd/csrc/mr_device.h"]
COPY_KERNEL = "k_copy_u4"


def kernel_source_hash() -> str:
    """Hash of the kernel sources: a counter summary is valid for this source only."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """Kernel name without namespace and argument list, template arguments kept."""
    n = re.sub(r"^void ", "", name)
    depth, cut = 0, len(n)
    for k, ch in enumerate(n):  # the argument list is the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = k
            break
    return n[:cut].replace("mrlbm::", "")


def _matches(name: str, patterns) -> bool:
    return all(p in name for p in patterns)


def read_trace(path: str):
    """Kernel dispatches in start order: (short name, start ns, end ns)."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            rows.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort(key=lambda t: t[1])
    return rows


def read_counters(path: str, counter: str):
    """Per dispatch, in start order: (kernel name, start ns, counter value summed over rows)."""
    acc = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            key = int(r["Dispatch_Id"])
            if key not in acc:
                acc[key] = [r["Kernel_Name"], int(r["Start_Timestamp"]), 0.0]
            acc[key][2] += float(r["Counter_Value"])
    return sorted((tuple(v) for v in acc.values()), key=lambda t: t[1])


def select(seq, patterns, skip: int, take: int, window="", index: int = 0):
    """Dispatches of the kernels matching all patterns, optionally only those
    starting between dispatches `index` and `index` + 1 of the kernel named
    `window`; then `skip` of them are dropped and at most `take` kept."""
    if window:
        marks = [x[1] for x in seq if window in x[0]]
        if len(marks) < index + 2:
            raise SystemExit("fewer than %d %s markers" % (index + 2, window))
        seq = [x for x in seq if marks[index] < x[1] < marks[index + 1]]
    hits = [x for x in seq if _matches(x[0], patterns)]
    hits = hits[skip:]
    return hits[:take] if take > 0 else hits


def stats_summary(args) -> str:
    rows = all_rows = read_trace(args.trace)
    if args.table_window:  # the table covers only the timed region
        marks = [r[1] for r in rows if args.window in r[0]]
        if len(marks) < args.window_index + 2:
            raise SystemExit("fewer than %d %s markers" % (args.window_index + 2, args.window))
        rows = [r for r in rows if marks[args.window_index] < r[1] < marks[args.window_index + 1]]
    agg = defaultdict(lambda: [0, 0, float("inf"), 0])
    for n, s, e in rows:
        a = agg[short_name(n)]
        d = e - s
        a[0] += 1
        a[1] += d
        a[2] = min(a[2], d)
        a[3] = max(a[3], d)
    total = sum(a[1] for a in agg.values()) or 1
    per = args.per_step if args.table_window and args.per_step > 0 else 0
    lines = ["# rocprofv3 kernel trace summary: %s" % args.title,
             "command: %s" % args.command,
             "",
             "%-58s %8s %12s %10s %10s %10s %6s%s" % ("kernel", "calls", "total_us", "avg_us", "min_us", "max_us", "%",
                                                    " %12s" % "us_per_step" if per else "")]
    for name, (c, t, mn, mx) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append("%-58s %8d %12.1f %10.2f %10.2f %10.2f %6.1f%s" % (
            name[:58], c, t / 1e3, t / c / 1e3, mn / 1e3, mx / 1e3, 100.0 * t / total,
            " %12.2f" % (t / 1e3 / per) if per else ""))
    if per:
        lines.append("%-58s %8s %12.1f %10s %10s %10s %6s %12.2f" % ("sum of kernel durations", "", total / 1e3, "", "",
                                                                    "", "", total / 1e3 / per))
    if args.match:
        sel = select(all_rows, args.match, args.skip, args.take, args.window, args.window_index)
        if sel:
            durs = [e - s for _, s, e in sel]
            where = ("between %s markers %d and %d" % (args.window, args.window_index + 1, args.window_index + 2)) \
                if args.window else (
                "dispatches %d..%d" % (args.skip + 1, args.skip + len(sel)))
            lines += ["",
                      "timed region: %s, kernels matching %s (%s)" % (
                          where, " & ".join(repr(p) for p in args.match), short_name(sel[0][0])),
                      "  dispatches %d, average %.3f us, min %.3f us, max %.3f us" % (
                          len(durs), sum(durs) / len(durs) / 1e3, min(durs) / 1e3, max(durs) / 1e3)]
    return "\n".join(lines) + "\n"


def counters_summary(args) -> dict:
    fetch = select(read_counters(args.fetch, "FETCH_SIZE"), args.match, args.skip, args.take, args.window,
                   args.window_index)
    write = select(read_counters(args.write, "WRITE_SIZE"), args.match, args.skip, args.take, args.window,
                   args.window_index)
    cf = select(read_counters(args.copy_fetch, "FETCH_SIZE"), [COPY_KERNEL], 1, 0)  # first launch warms up
    cw = select(read_counters(args.copy_write, "WRITE_SIZE"), [COPY_KERNEL], 1, 0)
    if not fetch or not write or not cf or not cw:
        raise SystemExit("no matching dispatches in the counter files")
    copy_kib_f = sum(v for _, _, v in cf) / len(cf)
    copy_kib_w = sum(v for _, _, v in cw) / len(cw)
    # bytes per counter KiB, from the copy kernel of known size
    sf = args.copy_bytes / copy_kib_f
    sw = args.copy_bytes / copy_kib_w
    kib_f = sum(v for _, _, v in fetch) / len(fetch)
    kib_w = sum(v for _, _, v in write) / len(write)
    return {
        "kernel": short_name(fetch[0][0]),
        "workload": args.workload,
        "precision_bytes": args.precision,
        "kernel_source_hash": kernel_source_hash(),
        "commands": args.command,
        "dispatches": {"fetch": len(fetch), "write": len(write), "skip": args.skip, "window": args.window},
        "copy_calibration": {"kernel": COPY_KERNEL, "bytes_each_way": args.copy_bytes,
                             "fetch_kib": copy_kib_f, "write_kib": copy_kib_w,
                             "bytes_per_fetch_kib": sf, "bytes_per_write_kib": sw},
        "fetch_kib_per_launch": kib_f,
        "write_kib_per_launch": kib_w,
        "hbm_read_bytes_per_launch": kib_f * sf,
        "hbm_write_bytes_per_launch": kib_w * sw,
        "hbm_bytes_per_launch": kib_f * sf + kib_w * sw,
    }


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--table-window", action="store_true", help="table only over the --window markers")
    s.add_argument("--per-step", type=int, default=0, help="steps in the window (adds a per-step column)")
    c = sub.add_parser("counters")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        c.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    c.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    c.add_argument("--workload", required=True)
    c.add_argument("--precision", type=int, required=True)
    for p in (s, c):
        p.add_argument("--match", action="append", default=[])
        p.add_argument("--skip", type=int, default=0)
        p.add_argument("--take", type=int, default=0)
        p.add_argument("--window", default="", help="kernel whose dispatches bound the selection")
        p.add_argument("--window-index", type=int, default=0,
                       help="the selection lies between dispatches INDEX and INDEX + 1 of the window kernel")
        p.add_argument("--command", action="append", default=[])
        p.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.what == "stats":
        args.command = " ; ".join(args.command)
        text = stats_summary(args)
        with open(args.out, "w") as f:
            f.write(text)
    else:
        with open(args.out, "w") as f:
            json.dump(counters_summary(args), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
