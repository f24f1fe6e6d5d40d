"""Summaries of rocprofv3 CSV output for the committed profile records.

    python -m paper_1411_3656_amd.profiling stats   --csv <kernel_stats.csv> --command "<cmd>" --out <md>
    python -m paper_1411_3656_amd.profiling traffic --workload c2 --kernel ppf_fused_kernel \
        --fetch <csv> --write <csv> --copy-fetch <csv> --copy-write <csv> --copy-bytes 1073741824 \
        --commands "<cmd1>" "<cmd2>" ... --out-json <json> --out-md <md>

FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch. Each is scaled
by (known bytes / counter bytes) of a plain device copy of known size,
measured with the same counter, so that the result is in HBM bytes.
"""

from __future__ import annotations

import argparse
import csv
import json
import pathlib
import statistics
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def counter_kib(path, kernel_substr, counter):
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_substr!r} in {path}")
    return statistics.median(vals), len(vals)


def counter_total_kib(path, kernel_substr, counter):
    vals = [float(r["Counter_Value"]) for r in _rows(path)
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_substr!r} in {path}")
    return sum(vals)


def sq_md(a):
    """Median per dispatch of every counter in the CSVs (one pass each) for
    the kernel, with per-unit and per-CU figures."""
    vals = {}
    for path in a.csv:
        for r in _rows(path):
            if a.kernel in r["Kernel_Name"]:
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    med = {k: statistics.median(v) for k, v in vals.items()}
    out = [f"# {a.title}", "", f"Kernel matching `{a.kernel}`; counters are per dispatch (median over the "
           "profiled dispatches), summed over the chip.", "",
           "Commands (run from /tmp, repository at /root/repo), one pass each:", "", "```", *a.commands, "```", "",
           "| counter | per dispatch | per unit |" if a.units else "| counter | per dispatch |",
           "|---|---:|---:|" if a.units else "|---|---:|"]
    for k in sorted(med):
        if a.units:
            out.append(f"| {k} | {med[k]:.6g} | {med[k] / a.units:.4g} |")
        else:
            out.append(f"| {k} | {med[k]:.6g} |")
    if a.units:
        out += ["", f"Units per dispatch: {a.units:.0f} (per CU: {a.units / a.cus:.1f}, {a.cus} CUs)."]
    if a.notes:
        out += ["", *a.notes]
    return "\n".join(out) + "\n"


def kernel_stats_md(path, command):
    rows = _rows(path)
    out = ["# rocprofv3 kernel statistics", "", "Command (run from /tmp, repository at /root/repo):", "",
           "```", command, "```", "",
           "| kernel | calls | average (us) | min (us) | max (us) | share (%) |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("workload", "kernel", "fetch", "write", "copy-fetch", "copy-write", "out-json", "out-md"):
        t.add_argument(f"--{k}", required=True)
    t.add_argument("--copy-kernel", default="copyBuffer")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--commands", nargs="+", required=True)
    t.add_argument("--batches", type=int, default=0,
                   help="sum every kernel matching --kernel (a list, comma-separated) over this many batches")
    q = sub.add_parser("sq")
    q.add_argument("--kernel", required=True)
    q.add_argument("--csv", nargs="+", required=True)
    q.add_argument("--commands", nargs="+", required=True)
    q.add_argument("--title", required=True)
    q.add_argument("--units", type=float, default=0.0, help="work units (e.g. spectra) per dispatch")
    q.add_argument("--cus", type=int, default=256)
    q.add_argument("--out", required=True)
    q.add_argument("--notes", nargs="*", default=[], help="lines of interpretation appended to the summary")
    a = ap.parse_args(argv)

    if a.cmd == "stats":
        pathlib.Path(a.out).write_text(kernel_stats_md(a.csv, a.command))
        return 0
    if a.cmd == "sq":
        pathlib.Path(a.out).write_text(sq_md(a))
        return 0

    sys.path.insert(0, str(ROOT))
    import bench  # kernel-source hash recorded beside the counters

    if a.batches:
        # several kernels per batch (two-pass form): the counters of every
        # dispatch of each kernel, summed, per batch
        fetch = sum(counter_total_kib(a.fetch, k, "FETCH_SIZE") for k in a.kernel.split(",")) / a.batches
        write = sum(counter_total_kib(a.write, k, "WRITE_SIZE") for k in a.kernel.split(",")) / a.batches
        nf = nw = a.batches
    else:
        fetch, nf = counter_kib(a.fetch, a.kernel, "FETCH_SIZE")
        write, nw = counter_kib(a.write, a.kernel, "WRITE_SIZE")
    cfetch, _ = counter_kib(a.copy_fetch, a.copy_kernel, "FETCH_SIZE")
    cwrite, _ = counter_kib(a.copy_write, a.copy_kernel, "WRITE_SIZE")
    f_scale = a.copy_bytes / (cfetch * 1024)
    w_scale = a.copy_bytes / (cwrite * 1024)
    read_b = fetch * 1024 * f_scale
    write_b = write * 1024 * w_scale
    rec = {"workload": a.workload, "kernel": a.kernel, "kernel_hash": bench.kernel_hash(a.workload),
           "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write, "dispatches": [nf, nw],
           "copy_fetch_kib": cfetch, "copy_write_kib": cwrite, "copy_bytes": a.copy_bytes,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "read_bytes_per_launch": int(read_b), "write_bytes_per_launch": int(write_b),
           "bytes_per_launch": int(read_b + write_b), "commands": a.commands}
    pathlib.Path(a.out_json).write_text(json.dumps(rec, indent=1) + "\n")
    md = ["# HBM traffic per launch from rocprofv3 counters", "",
          f"Workload `{a.workload}`, kernel matching `{a.kernel}`, kernel-source hash `{rec['kernel_hash']}`.", "",
          "Commands (run from /tmp, repository at /root/repo), one counter per pass:", "", "```",
          *a.commands, "```", "",
          "| quantity | value |", "|---|---:|",
          f"| FETCH_SIZE per dispatch (KiB, median of {nf}) | {fetch:.0f} |",
          f"| WRITE_SIZE per dispatch (KiB, median of {nw}) | {write:.0f} |",
          f"| copy of {a.copy_bytes} B: FETCH_SIZE (KiB) | {cfetch:.0f} |",
          f"| copy of {a.copy_bytes} B: WRITE_SIZE (KiB) | {cwrite:.0f} |",
          f"| read scale (known / counted) | {f_scale:.4f} |",
          f"| write scale (known / counted) | {w_scale:.4f} |",
          f"| HBM read bytes per launch | {int(read_b)} |",
          f"| HBM write bytes per launch | {int(write_b)} |",
          f"| total HBM bytes per launch | {int(read_b + write_b)} |"]
    pathlib.Path(a.out_md).write_text("\n".join(md) + "\n")
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
