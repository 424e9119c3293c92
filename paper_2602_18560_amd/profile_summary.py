"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2602_18560_amd.profile_summary stats DIR/ks_kernel_stats.csv "COMMAND"
      -> markdown table of per-kernel calls / total / average duration

  python -m paper_2602_18560_amd.profile_summary trace DIR/ks_kernel_trace.csv KERNEL N_ITER
      -> the working dispatches of KERNEL in a --kernel-trace of gbsub runs: the
         first N_ITER of each run (a run starts at its k_prep_count; later
         dispatches belong to bodies enqueued past the settled one and exit
         at once), their average duration, and the first body's (full grid)
         against the later ones'

  python -m paper_2602_18560_amd.profile_summary traffic FETCH.csv WRITE.csv \
         COPY_FETCH.csv COPY_WRITE.csv COPY_BYTES KERNEL "COMMANDS" [OUT_BASE [N_ITER]]
      -> markdown + json: per-dispatch HBM bytes of KERNEL from the FETCH_SIZE
         and WRITE_SIZE counters, each scaled by what the counter reads for a
         plain copy kernel that moves COPY_BYTES in and out; with N_ITER, over
         the working dispatches of the runs of N_ITER loop bodies only.

Reads only the CSV files it is given.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "gbsub_kernels.hip")


def kernel_source_hash() -> str:
    """sha256 of the kernel source with comments and whitespace removed: the
    counters describe the code, so an edit of a comment keeps them valid."""
    import re
    with open(KERNEL_SOURCE, encoding="utf-8") as fh:
        src = fh.read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("gbs::", "")


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    return f"Command:\n\n    {command}\n\n" + "\n".join(out) + "\n"


def trace(path: str, kernel: str, n_iter: int) -> str:
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    runs, cur = [], None
    for r in rows:
        name = short(r["Kernel_Name"])
        if name == "k_prep_count":
            cur = []
            runs.append(cur)
        elif name == kernel and cur is not None:
            cur.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    runs = [r for r in runs if len(r) >= n_iter]
    work = [d for r in runs for d in r[:n_iter]]
    first = [r[0] for r in runs]
    later = [d for r in runs for d in r[1:n_iter]]
    extra = [d for r in runs for d in r[n_iter:]]
    mean = lambda v: sum(v) / len(v) if v else float("nan")
    return (f"{kernel} in {len(runs)} runs of {n_iter} loop bodies: {len(work)} working dispatches, "
            f"average {mean(work):.2f} us; first body (every tile) {mean(first):.2f} us; later bodies "
            f"{mean(later):.2f} us; {len(extra)} dispatches past the settled body, {mean(extra):.2f} us.\n")


def _per_dispatch(path: str):
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return acc


def _run_dispatches(path: str, kernel: str, n_iter: int):
    """Counter values of the working dispatches of `kernel`: the first n_iter
    of each run of n_iter bodies or more (runs start at k_prep_count), in
    dispatch order."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))
    runs, cur = [], None
    for r in rows:
        name = short(r["Kernel_Name"])
        if name == "k_prep_count":
            cur = []
            runs.append(cur)
        elif name == kernel and cur is not None:
            cur.append(float(r["Counter_Value"]))
    return [v for run in runs if len(run) >= n_iter for v in run[:n_iter]]


def traffic(fetch, write, cfetch, cwrite, copy_bytes, kernel, commands, n_iter=0):
    f, w = _per_dispatch(fetch), _per_dispatch(write)
    cf, cw = _per_dispatch(cfetch), _per_dispatch(cwrite)

    def copy_kib(acc):   # the largest dispatches are the copy itself (fills are smaller)
        vals = sorted(v for lst in acc.values() for v in lst)
        return vals[-1]
    kib = copy_bytes / 1024.0
    ff = kib / copy_kib(cf)
    fw = kib / copy_kib(cw)
    rows = ["| kernel | dispatches | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | "
            "HBM MB/dispatch (scaled) |", "|---|---|---|---|---|"]
    for k in sorted(f):
        fv = sum(f[k]) / len(f[k])
        wv = sum(w.get(k, [0.0])) / max(len(w.get(k, [])), 1)
        rows.append(f"| {k} | {len(f[k])} | {fv:.1f} | {wv:.1f} | {(fv * ff + wv * fw) * 1024 / 1e6:.3f} |")
    kf, kw = f[kernel], w[kernel]
    if n_iter:
        # the working dispatches of the runs that went all the way
        work = list(zip(_run_dispatches(fetch, kernel, n_iter), _run_dispatches(write, kernel, n_iter)))
    else:
        # dispatches that did work: a loop body enqueued after the loop settled
        # exits at once and reads a few KiB of descriptors only
        work = [(a, b) for a, b in zip(kf, kw) if a > 64.0]
    fa = sum(a for a, _ in work) / len(work)
    wa = sum(b for _, b in work) / len(work)
    per = (fa * ff + wa * fw) * 1024
    summary = {"kernel": kernel, "source_sha256": kernel_source_hash(),
               "fetch_factor": ff, "write_factor": fw,
               "working_dispatches": len(work), "all_dispatches": len(kf),
               "fetch_kib_per_launch": fa, "write_kib_per_launch": wa,
               "traffic_bytes_per_launch": per, "commands": commands}
    md = (f"Commands:\n\n" + "\n".join(f"    {c}" for c in commands) + "\n\n"
          f"Copy calibration: a {copy_bytes / 2**20:.0f} MiB read + {copy_bytes / 2**20:.0f} MiB write "
          f"elementwise kernel reads FETCH_SIZE {copy_kib(cf):.0f} KiB and WRITE_SIZE {copy_kib(cw):.0f} KiB, "
          f"so HBM read bytes = {ff:.3f} x FETCH_SIZE and written bytes = {fw:.3f} x WRITE_SIZE.\n\n"
          + "\n".join(rows) + "\n\n"
          f"{kernel}: {len(work)} working dispatches of {len(kf)}; "
          f"{per / 1e6:.3f} MB of HBM traffic per working dispatch.\n")
    return md, summary


def main(argv):
    if argv[0] == "stats":
        sys.stdout.write(stats(argv[1], argv[2]))
    elif argv[0] == "trace":
        sys.stdout.write(trace(argv[1], argv[2], int(argv[3])))
    elif argv[0] == "traffic":
        md, js = traffic(argv[1], argv[2], argv[3], argv[4], float(argv[5]), argv[6], argv[7].split(" ;; "),
                         int(argv[9]) if len(argv) > 9 else 0)
        base = argv[8] if len(argv) > 8 else None
        if base:
            with open(base + ".md", "w") as fh:
                fh.write(md)
            with open(base + ".json", "w") as fh:
                json.dump(js, fh, indent=1)
        sys.stdout.write(md)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
