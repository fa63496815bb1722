"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  python -m paper_2208_13770_amd.profile_summary stats KERNEL_STATS_CSV OUT.md --cmd "..."
      per-kernel time table from `rocprofv3 --kernel-trace --stats --output-format csv`;
  python -m paper_2208_13770_amd.profile_summary traffic FETCH_CSV WRITE_CSV OUT.json \
      --kernel k_step --cmd-fetch "..." --cmd-write "..."
      HBM bytes per launch of one kernel from two `rocprofv3 --pmc` runs (FETCH_SIZE,
      then WRITE_SIZE, KiB per dispatch).  Each counter is scaled by what it reads
      for the largest device-to-device copy in the same run (a plain copy kernel of
      known size, 4 GiB read + 4 GiB written by bench.py's bandwidth probe).
"""
import argparse
import csv
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SRC = os.path.join(HERE, "csrc", "vb_kernels.hip")
COPY_BYTES = 4 << 30  # bench.py's copy probe moves 4 GiB per launch each way


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# Kernel time: {args.title}", "", f"Command: `{args.cmd}`", "",
           f"Kernel source sha256[:16]: {kernel_hash()}", "",
           "| kernel | calls | total ms | mean us | min us | max us | % |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| {} | {} | {:.3f} | {:.2f} | {:.2f} | {:.2f} | {:.1f} |".format(
            r["Name"].replace("|", "/")[:70], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            100.0 * float(r["TotalDurationNs"]) / total))
    open(args.out, "w").write("\n".join(out) + "\n")


def _per_kernel(path, counter):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def traffic(args):
    f = _per_kernel(args.fetch, "FETCH_SIZE")
    w = _per_kernel(args.write, "WRITE_SIZE")
    copy = [k for k in f if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no copy kernel in the FETCH run")
    f_copy = max(f[copy[0]]) * 1024.0
    w_copy = max(w[copy[0]]) * 1024.0
    scale_f = COPY_BYTES / f_copy
    scale_w = COPY_BYTES / w_copy
    name = [k for k in f if args.kernel in k]
    if not name:
        raise SystemExit(f"kernel {args.kernel} not found")
    fk = statistics.mean(f[name[0]]) * 1024.0 * scale_f
    wk = statistics.mean(w[name[0]]) * 1024.0 * scale_w
    out = {
        "kernel": name[0], "kernel_sha256_16": kernel_hash(),
        "launches": len(f[name[0]]),
        "fetch_bytes_per_launch": fk, "write_bytes_per_launch": wk,
        "bytes_per_launch": fk + wk,
        "copy_calibration": {"bytes": COPY_BYTES, "fetch_counter_bytes": f_copy,
                             "write_counter_bytes": w_copy, "fetch_scale": scale_f,
                             "write_scale": scale_w},
        "commands": {"fetch": args.cmd_fetch, "write": args.cmd_write},
    }
    json.dump(out, open(args.out, "w"), indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("out")
    t.add_argument("--kernel", default="k_step")
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    a = ap.parse_args()
    stats(a) if a.what == "stats" else traffic(a)


if __name__ == "__main__":
    main()
