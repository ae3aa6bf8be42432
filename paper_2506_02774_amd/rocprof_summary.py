"""Summaries of rocprofv3 CSV output for the renderer's kernels.

    python -m paper_2506_02774_amd.rocprof_summary stats DIR/run_kernel_stats.csv
        per-kernel calls / average / total time (markdown table)

    python -m paper_2506_02774_amd.rocprof_summary traffic FETCH_DIR/run_counter_collection.csv \
        WRITE_DIR/run_counter_collection.csv --copy-mib 1024 --kernel 'blend_jobs<true, false, false, false>' --stage blend

        HBM traffic per dispatch from FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch), each scaled by the factor that makes the reference copy
        kernel (x * 1 over copy-mib MiB, read once and written once) read and
        write exactly its own size. Prints a markdown table for every kernel
        and one JSON line for the named kernel, tagged with the SHA-1 of the
        source file that holds it, so that a reader can tell whether the
        counters are still those of the current kernel.

    python -m paper_2506_02774_amd.rocprof_summary counters A.csv [B.csv ...] --kernels 'k1;k2'

        average per dispatch of every counter found in the given
        counter_collection CSVs, for the named kernels (markdown table).
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "")
    n = re.sub(r"^void ", "", n)
    depth, out = 0, []
    for ch in n:          # cut at the first '(' outside template brackets
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out)


def stats(path, top):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    print("| kernel | calls | avg us | min us | max us | total % |")
    print("|---|---|---|---|---|---|")
    for r in rows[:top]:
        print(f"| `{short(r['Name'])[:80]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")


def per_kernel(path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in agg.items()}


def traffic(fetch_csv, write_csv, copy_mib, copy_regex, kernel, stage, source):
    fe = per_kernel(fetch_csv, "FETCH_SIZE")
    wr = per_kernel(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if re.search(copy_regex, k)]
    if len(copy) != 1:
        raise SystemExit(f"reference copy kernel not unique: {copy}")
    nbytes = copy_mib * 2 ** 20
    f_fetch = nbytes / (fe[copy[0]][1] * 1024.0)
    f_write = nbytes / (wr[copy[0]][1] * 1024.0)
    print(f"reference copy `{copy[0][:70]}`: FETCH_SIZE {fe[copy[0]][1]:.0f} KiB, WRITE_SIZE "
          f"{wr[copy[0]][1]:.0f} KiB for {copy_mib} MiB each way -> scale factors fetch {f_fetch:.4f}, "
          f"write {f_write:.4f}\n")
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled MB/dispatch (read + write) |")
    print("|---|---|---|---|---|")
    for k in sorted(fe, key=lambda k: -(fe[k][0] * fe[k][1])):
        w = wr.get(k, (0, 0.0))[1]
        mb = (fe[k][1] * 1024 * f_fetch + w * 1024 * f_write) / 1e6
        print(f"| `{k[:70]}` | {fe[k][0]} | {fe[k][1]:.0f} | {w:.0f} | {mb:.2f} |")
    if kernel not in fe:
        raise SystemExit(f"kernel {kernel!r} not found")
    rd = fe[kernel][1] * 1024 * f_fetch
    wt = wr[kernel][1] * 1024 * f_write
    sha = hashlib.sha1(open(source, "rb").read()).hexdigest()
    print()
    print(json.dumps(dict(stage=stage, kernel=kernel, source=os.path.relpath(source, os.path.dirname(HERE)),
                          source_sha1=sha, read_bytes_per_launch=round(rd), write_bytes_per_launch=round(wt),
                          traffic_bytes_per_launch=round(rd + wt), fetch_factor=round(f_fetch, 4),
                          write_factor=round(f_write, 4), dispatches=fe[kernel][0])))


def counters(paths, kernels):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in paths:
        for r in csv.DictReader(open(p)):
            vals[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for k in kernels if k in vals for c in vals[k]})
    print("| kernel | dispatches | " + " | ".join(names) + " |")
    print("|---|---|" + "---|" * len(names))
    for k in kernels:
        if k not in vals:
            continue
        n = max(len(v) for v in vals[k].values())
        cells = [f"{sum(vals[k][c]) / len(vals[k][c]):.4g}" if vals[k].get(c) else "" for c in names]
        print(f"| `{k[:60]}` | {n} | " + " | ".join(cells) + " |")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=25)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--copy-mib", type=int, default=1024)
    b.add_argument("--copy-regex", default=r"AUnaryFunctor.*MulFunctor|AUnaryFunctor")
    b.add_argument("--kernel", default="blend_jobs<true, false, false, false>")
    b.add_argument("--stage", default="blend")
    b.add_argument("--source", default=os.path.join(HERE, "csrc", "render.hip"))
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--kernels", default="blend_jobs<true, false, false, false>")
    args = ap.parse_args()
    if args.cmd == "stats":
        stats(args.csv, args.top)
    elif args.cmd == "counters":
        counters(args.csv, [k for k in args.kernels.split(";") if k])
    else:
        traffic(args.fetch_csv, args.write_csv, args.copy_mib, args.copy_regex, args.kernel, args.stage, args.source)


if __name__ == "__main__":
    main()
