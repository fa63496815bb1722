"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  python -m paper_2208_13770_amd.profile_summary stats KERNEL_STATS_CSV OUT.md --cmd "..."
      per-kernel time table from `rocprofv3 --kernel-trace --stats --output-format csv`;
  python -m paper_2208_13770_amd.profile_summary traffic FETCH_CSV WRITE_CSV OUT.json \
      --kernel k_step --cmd-fetch "..." --cmd-write "..."
      HBM bytes per launch of one kernel from two `rocprofv3 --pmc` runs (FETCH_SIZE,
      then WRITE_SIZE, KiB per dispatch).  Each counter is scaled by what it reads
      for the largest device-to-device copy in the same run (a plain copy kernel of
      known size, 4 GiB read + 4 GiB written by bench.py's bandwidth probe).
  python -m paper_2208_13770_amd.profile_summary sq CSV [CSV ...] OUT.md --kernel k_pairs \
      --cmd "..." [--cmd "..."]
      instruction-mix counters (SQ_*) of one kernel from `rocprofv3 --pmc` runs,
      averaged over the dispatches that did work (those issuing at least a tenth
      of the busiest dispatch's VALU instructions; a broad-phase kernel that finds
      nothing to do exits at once), with per-wave and per-lane ratios.  Runs of
      memory-pipeline counters (TA_*, TD_*, TCP_*, GRBM_GUI_ACTIVE) are averaged
      over all dispatches of the kernel and give busy and stall fractions per CU,
      latencies and the vector memory instructions in flight.
"""
N_CU = 256   # compute units; the _sum counters add one instance per CU
N_XCD = 8    # GRBM_GUI_ACTIVE adds one count per XCD
import argparse
import csv
import hashlib
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
# every source that shapes what the kernels do or how they are launched: the
# kernels, their record layouts and constants, the host code that sizes the grids
# and sequences the launches, and the build flags
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("vb_kernels.hip", "vb_device.h",
                                                          "vb_abi.hip")] + [os.path.join(HERE, "build.py")]
COPY_BYTES = 4 << 30  # bench.py's copy probe moves 4 GiB per launch each way


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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


def sq(args):
    # each counter run is filtered and averaged on its own (dispatch ids of two
    # runs need not correspond); a counter present in several runs is averaged
    name, sums, n_busy, n_all = None, {}, [], []
    for path in args.csv:
        per = {}  # dispatch id -> counter -> value
        for r in csv.DictReader(open(path)):
            if args.kernel not in r["Kernel_Name"]:
                continue
            name = r["Kernel_Name"]
            per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
        if not per:
            continue
        valu_max = max(d.get("SQ_INSTS_VALU", 0.0) for d in per.values())
        busy = [d for d in per.values() if d.get("SQ_INSTS_VALU", 0.0) >= 0.1 * valu_max]
        n_busy.append(len(busy))
        n_all.append(len(per))
        for k in {k for d in busy for k in d}:
            sums.setdefault(k, []).append(statistics.mean(d[k] for d in busy if k in d))
    if not sums:
        raise SystemExit(f"kernel {args.kernel} not found")
    keys = sorted(sums)
    mean = {k: statistics.mean(v) for k, v in sums.items()}
    busy = n_busy
    kind = "Instruction-mix" if any(k.startswith("SQ_") for k in keys) else "Memory-pipeline"
    out = [f"# {kind} counters: {args.title or name}", "",
           *[f"Command: `{c}`" for c in args.cmd], "",
           f"Kernel source sha256[:16]: {kernel_hash()}", "",
           f"Kernel: `{name}`; dispatches that did work, per run: "
           f"{', '.join(f'{b} of {t}' for b, t in zip(n_busy, n_all))} (averaged below).", "",
           "| counter | mean per working dispatch |", "|---|---:|"]
    out += [f"| {k} | {mean[k]:.4g} |" for k in keys]
    waves = mean.get("SQ_WAVES")
    ratios = []
    if waves:
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD"):
            if k in mean:
                ratios.append((f"{k} per wave", mean[k] / waves))
    if mean.get("SQ_ACTIVE_INST_VALU") and "SQ_THREAD_CYCLES_VALU" in mean:
        ratios.append(("VALU lanes active (SQ_THREAD_CYCLES_VALU / 64 SQ_ACTIVE_INST_VALU)",
                       mean["SQ_THREAD_CYCLES_VALU"] / (64.0 * mean["SQ_ACTIVE_INST_VALU"])))
    if mean.get("SQ_ACTIVE_INST_LDS") and "SQ_LDS_BANK_CONFLICT" in mean:
        ratios.append(("LDS bank-conflict cycles per active LDS instruction cycle",
                       mean["SQ_LDS_BANK_CONFLICT"] / mean["SQ_ACTIVE_INST_LDS"]))
    cycles = mean.get("GRBM_GUI_ACTIVE", 0.0) / N_XCD  # GPU cycles of one dispatch
    if cycles:
        ratios.append(("GPU cycles per dispatch (GRBM_GUI_ACTIVE / 8 XCDs)", cycles))
        if "TA_BUSY_avr" in mean:
            ratios.append(("TA busy, fraction of the cycles (TA_BUSY_avr)", mean["TA_BUSY_avr"] / cycles))
        for k, what in (("TD_TD_BUSY_sum", "TD processing or waiting for data"),
                        ("TD_TC_STALL_sum", "TD stalled by the L1 (TCP)"),
                        ("TCP_PENDING_STALL_CYCLES_sum", "L1 stalled on data pending from L2"),
                        ("TCP_TCP_TA_DATA_STALL_CYCLES_sum", "L1 stalling the TA data interface"),
                        ("TA_ADDR_STALLED_BY_TC_CYCLES_sum", "TA address path stalled by the L1"),
                        ("TA_DATA_STALLED_BY_TC_CYCLES_sum", "TA data path stalled by the L1")):
            if k in mean:
                ratios.append((f"{what}, fraction of the cycles per CU ({k} / {N_CU})",
                               mean[k] / N_CU / cycles))
    if mean.get("TCP_TCC_READ_REQ_sum") and "TCP_TCC_READ_REQ_LATENCY_sum" in mean:
        ratios.append(("L1-to-L2 read latency, cycles (TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum)",
                       mean["TCP_TCC_READ_REQ_LATENCY_sum"] / mean["TCP_TCC_READ_REQ_sum"]))
    if mean.get("TA_TOTAL_WAVEFRONTS_sum") and "TCP_TCP_LATENCY_sum" in mean:
        lat = mean["TCP_TCP_LATENCY_sum"] / mean["TA_TOTAL_WAVEFRONTS_sum"]
        ratios.append(("vector memory instruction latency in the L1, cycles "
                       "(TCP_TCP_LATENCY_sum / TA_TOTAL_WAVEFRONTS_sum)", lat))
        if cycles:
            ratios.append(("vector memory instructions in flight per CU (Little's law)",
                           mean["TA_TOTAL_WAVEFRONTS_sum"] / N_CU * lat / cycles))
    if ratios:
        out += ["", "| ratio | value |", "|---|---:|"] + [f"| {k} | {v:.3g} |" for k, v in ratios]
    open(args.out, "w").write("\n".join(out) + "\n")


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
    q = sub.add_parser("sq")
    q.add_argument("csv", nargs="+")
    q.add_argument("out")
    q.add_argument("--kernel", default="k_pairs")
    q.add_argument("--cmd", action="append", required=True)
    q.add_argument("--title", default="")
    a = ap.parse_args()
    {"stats": stats, "traffic": traffic, "sq": sq}[a.what](a)


if __name__ == "__main__":
    main()
