"""The paper's K experiment (Sec. 5.4) on the synthetic workloads.

  python -m paper_2208_13770_amd.sweep [--workload M2] [--steps 500] [--out FILE.json]

For every K in the sweep, the same steps run from the same state; the table
reports the wall time (a run without instrumentation), the time in the broad
phase and in the step kernel (HIP events on the kernels themselves, in a second
identical run), the number of broad phases and the
executed-broad-phase percentage (the quantity of Fig. executed), and Eq. impr
against the run without Verlet buffer.  Two more skin variants are run: a
uniform skin equal to the particle radius, and a broad phase at a fixed interval
with that uniform skin (the scheme Sec. 2 argues against; its results may differ
from the exact ones, which the table reports).  A last row lets the runtime
tuner choose K while the simulation runs (autotune.py).  Every row also says whether its
final state is bit-identical to the run without buffer (Sec. 4.2).  The last
part is one line in the layout of Tab. summary: the time without buffer, the
optimum K, its time and improvement, the time and improvement at K = 200, and
the overhead of K = 200 over the optimum.  Every row also gives its own overhead
over the optimum (the quantity of Fig. overhead), and with --repeats R the wall
time is the mean of R runs from the same state, with its standard deviation, so
that the optimum can be told from the noise.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import autotune, report

K_SWEEP = (0.0, 10.0, 20.0, 50.0, 100.0, 200.0, 400.0, 500.0, 1000.0, 5000.0)
K_DEFAULT = 200.0


def summary_row(name, t_without, times_by_k):
    """Tab. summary columns from the run without buffer and the times per K."""
    k_opt = min(times_by_k, key=lambda k: (times_by_k[k], k))
    t_opt = times_by_k[k_opt]
    t_def = times_by_k[K_DEFAULT]
    return {"testcase": name, "t_without": t_without, "k_opt": k_opt, "t_opt": t_opt,
            "impr_opt": report.improvement(t_without, t_opt), "t_default": t_def,
            "impr_default": report.improvement(t_without, t_def),
            "overhead": report.overhead_to_optimum(t_def, t_opt)}


def run_case(vb, torch, systems, x, v, rc, invm, steps, overrides, repeats=1, call_steps=500):
    """The same steps from the same state: `repeats` times without
    instrumentation (the wall times), then once with HIP events on every kernel
    (the split between broad phase and step kernel).  Steps go to vb_run in calls
    of at most call_steps."""
    params = [dict(s.params, **overrides) for s in systems]
    ctx = vb.vb_batch_create(params, [s.n for s in systems])
    walls = []
    try:
        for r in range(max(1, repeats)):
            vb.vb_set_state(ctx, x, v, rc, invm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            parts = [vb.vb_run(ctx, min(call_steps, steps - k), want_history=(r == 0))
                     for k in range(0, steps, call_steps)]
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            if r == 0:
                hist = np.concatenate(parts, axis=1)
        wall = walls
        xo = torch.empty_like(x)
        vo = torch.empty_like(v)
        vb.vb_get_state(ctx, xo, vo)
        vb.vb_set_state(ctx, x, v, rc, invm)
        vb.vb_set_timing(ctx, 1)
        for k in range(0, steps, call_steps):
            vb.vb_run(ctx, min(call_steps, steps - k), want_history=False)
        pt = vb.vb_phase_times(ctx)
    finally:
        vb.vb_destroy(ctx)
    return wall, hist, pt, xo, vo


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", default="M2")
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--fixed-interval", type=int, default=50)
    ap.add_argument("--repeats", type=int, default=1,
                    help="timed runs of every case from the same state (mean and spread)")
    ap.add_argument("--no-tuner", action="store_true", help="skip the tuned-K row")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch
    import paper_2208_13770_amd as vb
    import synth

    systems = synth.config_systems(args.workload, seed=0, scale=args.scale)
    n = sum(s.n for s in systems)
    x, v, rc, invm = vb.state_tensors(systems)
    # one untimed run first: library load, first allocation, caches
    run_case(vb, torch, systems, x, v, rc, invm, min(args.steps, 20), {})

    cases = [("no buffer", {"skin_mode": vb.VB_NO_BUFFER})]
    cases += [(f"K={k:g}", {"K": k}) for k in K_SWEEP]
    cases += [("uniform skin = radius", {"skin_mode": vb.VB_SKIN_UNIFORM}),
              (f"fixed interval {args.fixed_interval}, skin = radius",
               {"skin_mode": vb.VB_FIXED_INTERVAL, "fixed_interval": args.fixed_interval})]
    rows, ref = [], None
    for name, ov in cases:
        walls, hist, pt, xo, vo = run_case(vb, torch, systems, x, v, rc, invm, args.steps, ov,
                                           repeats=args.repeats)
        wall = float(np.mean(walls))
        if ref is None:
            ref = (wall, xo, vo, hist)
        exact = bool(torch.equal(xo, ref[1]) and torch.equal(vo, ref[2]))
        n_bp = int(hist["rebuilt"].sum())
        row = {"case": name, "K": ov.get("K"), "time_ms": wall * 1e3,
               "time_ms_std": float(np.std(walls, ddof=1)) * 1e3 if len(walls) > 1 else 0.0,
               "runs": len(walls),
               "broad_phase_ms": pt["ms_rebuild"], "step_kernel_ms": pt["ms_step"],
               "broad_phases": n_bp,
               "executed_pct": report.executed_fraction(n_bp, args.steps * len(systems)),
               "impr_pct": report.improvement(ref[0], wall),
               "identical_to_no_buffer": exact,
               "contacts_equal": bool(np.array_equal(hist["contacts"], ref[3]["contacts"]))}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    times = {r["K"]: r["time_ms"] / 1e3 for r in rows if r["K"] is not None}
    t_opt = min(times.values())
    for r in rows:  # Fig. overhead: each case's extra time over the optimum K, in % of its own
        r["overhead_to_opt_pct"] = report.overhead_to_optimum(r["time_ms"] / 1e3, t_opt)
    if not args.no_tuner:
        rows.append(tuned_row(vb, torch, systems, x, v, rc, invm, args.steps, ref))
    out = {"workload": args.workload, "particles": n, "systems": len(systems),
           "steps": args.steps, "repeats": args.repeats, "rows": rows,
           "summary": summary_row(args.workload, ref[0], times)}
    text = json.dumps(out, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text, flush=True)


def tuned_row(vb, torch, systems, x, v, rc, invm, steps, ref):
    """K chosen at run time, windows of about 1/20 of the run (no instrumentation)."""
    params = [dict(s.params) for s in systems]
    ctx = vb.vb_batch_create(params, [s.n for s in systems])
    rebuilds = []
    try:
        vb.vb_set_state(ctx, x, v, rc, invm)

        run_window = autotune.window_runner(
            vb, ctx, on_records=lambda h: rebuilds.append(int(h["rebuilt"].any(axis=0).sum())))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        windows, k_auto = autotune.tune(run_window, steps, K0=K_DEFAULT,
                                        window=max(10, steps // 20),
                                        exploit=max(40, steps // 4))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        xo = torch.empty_like(x)
        vo = torch.empty_like(v)
        vb.vb_get_state(ctx, xo, vo)
    finally:
        vb.vb_destroy(ctx)
    row = {"case": "auto (tuned K)", "K": None, "K_final": k_auto, "time_ms": wall * 1e3,
           "broad_phase_ms": None, "step_kernel_ms": None,
           "broad_phases": sum(rebuilds),
           "executed_pct": report.executed_fraction(sum(rebuilds), steps),
           "impr_pct": report.improvement(ref[0], wall),
           "identical_to_no_buffer": bool(torch.equal(xo, ref[1]) and torch.equal(vo, ref[2])),
           "contacts_equal": None, "windows": [[k, s_, t] for k, s_, t in windows]}
    print(json.dumps({k: v_ for k, v_ in row.items() if k != "windows"}), file=sys.stderr, flush=True)
    return row


if __name__ == "__main__":
    main()
