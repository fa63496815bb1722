"""Benchmark of the local Verlet buffer DEM step on one MI355X.

Default workload M2 (the throughput configuration): a 256x256x64 jittered
lattice of 4,194,304 particles with 64 moving boxes and 32 moving balls, sigma
0.1, K = 200, 500 time steps (Sec. 5.1: the paper's runs are >= 5000 steps on
CPU; this is the synthetic stand-in).  A "step" is one DEM time step of the
method: the conditional broad phase (skin, cap, binning, linked-cell pair
search) and the fused narrow phase + forces + integration + validity test, for
every particle of every system.

--workload M3 runs the 64 uneven systems as one batch (and, with --sequential,
also one context per system, one after the other); --workload M5 runs 16
systems of 16.8M particles (268M in all); H125, H250, H500, INCLINE and SILO are
the gravity-driven stand-ins for the paper's hopper, inclined-plane and silo
cases (planar and cylindrical walls, polydisperse radii).  Only the default
workload times the CPU oracle.

Prints ONE JSON line:
  value       whole-job throughput, Mparticle*step/s, of the method (K = 200) with
              the state resident in HBM: the mean over --repeats runs without
              instrumentation, each of the same steps from step 0 (Sec. 5.3 averages
              at least a hundred measurements);
  repeats     mean, spread and range of the wall time over those runs;
  roofline    the step kernel's algorithmic bytes per launch over its mean duration,
              taken by HIP events on the kernel in an identical further run, against
              the 8 TB/s HBM peak;
  plain       the same steps with the broad phase at every step ("without Verlet
              buffer"), and Eq. impr between the two;
  cpu_baseline the FP64 oracle on a bounded sample of the same workload on the host's
              cores (and, beside it, on one thread), with the host's CPU model and
              core count.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one particle in one step of the fused step kernel (a1, a2,
# a6), three counts, each plus 4 B per Verlet-list entry read (n_v entries per
# particle, n_v = 2 list_pairs / N):
#  - ALG: the hot-path scope's count for an FP32 state: read position and radius
#    (16 B), velocity and inverse mass (16), reference position and extended
#    radius (16) and the row length (4); write position and velocity (32).  The
#    roofline's `frac` uses it.
#  - FP64: the same with the FP64 state this library keeps (parity needs it):
#    read x and v (48 B), R_C and 1/m (8), x0 and R_NL (16), row length (4);
#    write x and v (48).
#  - KERNEL: what the step kernel's own accesses move: read x and v (48 B),
#    (R_C, 1/m) (8), x0 and R_NL (16) and the row length (4); write x and v (48)
#    and the coded position the next step's pre-test gathers (8).
STEP_BYTES = {"alg": 84, "fp64": 124, "kernel": 132}
STEP_BYTES_PER_ENTRY = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_M2_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter runs,
    only if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2208_13770_amd.profile_summary import kernel_hash
    if t.get("kernel_sha256_16") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def copy_bandwidth(torch, nbytes=4 << 30):
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del a, b
    return 2 * nbytes / dt / 1e9


def default_shape(n, friction):
    """The library's launch shape for a new context (gathers in flight, tile
    order, pair-search threads) that no tuner has seen."""
    return (8 if friction and n >= 2 ** 20 else 4, 2, 384)


def run_mode(vb, torch, systems, steps, warmup, overrides, timing, call_steps=500, repeats=1,
             shape=None):
    """One context over `systems` (a batch when more than one).  After `warmup`
    untimed steps, `repeats` timed runs of `steps` steps, each from the loaded
    initial state (step 0, whose broad phase is timed).  Returns the wall times,
    the first run's [n_sys, steps] records, phase times of the last run and the
    context info.  The steps go to vb_run in calls of at most `call_steps`."""
    params = [dict(s.params, **overrides) for s in systems]
    ctx = vb.vb_batch_create(params, [s.n for s in systems])
    walls, hist = [], None
    try:
        if shape is not None:
            vb.vb_set_launch(ctx, *shape)
        x, v, rc, invm = vb.state_tensors(systems)
        if warmup > 0:
            vb.vb_set_state(ctx, x, v, rc, invm)
            vb.vb_run(ctx, warmup, want_history=False)
        cs = max(1, call_steps)
        for r in range(max(1, repeats)):
            vb.vb_set_state(ctx, x, v, rc, invm)  # the timed steps start at step 0
            vb.vb_set_timing(ctx, timing)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            parts = [vb.vb_run(ctx, min(cs, steps - k), want_history=(r == 0))
                     for k in range(0, steps, cs)]
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            if r == 0:
                hist = np.concatenate(parts, axis=1) if parts else vb.vb_run(ctx, 0)
        del x, v, rc, invm
        pt = vb.vb_phase_times(ctx)
        info = vb.vb_get_info(ctx)
        info["launch"] = vb.vb_get_launch(ctx)
    finally:
        vb.vb_destroy(ctx)
        torch.cuda.synchronize()
    return walls, hist, pt, info


def tune_shape(vb, torch, systems, steps):
    """An untimed run of `steps` steps that chooses the launch shape by
    measurement (vb_tune); contexts of the same kind created afterwards start
    from it.  Returns the chosen shape."""
    ctx = vb.vb_batch_create([dict(s.params) for s in systems], [s.n for s in systems])
    try:
        x, v, rc, invm = vb.state_tensors(systems)
        vb.vb_set_state(ctx, x, v, rc, invm)
        vb.vb_tune(ctx, steps, want_history=False)
        return vb.vb_get_launch(ctx)
    finally:
        vb.vb_destroy(ctx)
        torch.cuda.synchronize()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(system, steps, threads=1):
    """The FP64 oracle on the first `steps` steps of the workload, on `threads`
    host threads (its results do not depend on the count)."""
    import oracle
    pos, vel = system.pos_r.astype(np.float64), system.vel_m.astype(np.float64)
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.run(system.params, pos[:, :3], vel[:, :3], pos[:, 3], vel[:, 3], steps)
    dt = time.perf_counter() - t0
    oracle.set_threads(1)
    return system.n * steps / dt / 1e6, dt


WORKLOADS = {
    "M2": "M2: 256x256x64 jittered lattice = {n} particles, 64 boxes + 32 balls moving, "
          "sigma 0.1, K=200, cap L_C/2, L_C=1.7a, eps=2e-6",
    "M3": "M3: 64 systems of (s_x/4)x(s_y/4)x16, s in {{256,384,512,768,1024}}, {n} particles "
          "in all, sigma U[0.02,0.15], K=200, one batch",
    "M5": "M5: 16 systems of 512x512x64 = {n} particles in all, 256 boxes + 128 balls, "
          "sigma U[0.05,0.2], K=200, one batch",
    "M1": "M1: 32x32x16 jittered lattice = {n} particles, 8 boxes + 4 balls, sigma 0.05, K=200",
    "H125": "hopper stand-in: wedge hopper (walls at 30 deg, outlet 8a) of {n} polydisperse "
            "particles under gravity, K=200",
    "H250": "hopper stand-in: wedge hopper (walls at 30 deg, outlet 8a) of {n} polydisperse "
            "particles under gravity, K=200",
    "H500": "hopper stand-in: wedge hopper (walls at 30 deg, outlet 8a) of {n} polydisperse "
            "particles under gravity, K=200",
    "INCLINE": "inclined-plane stand-in: slab of {n} polydisperse particles, gravity tilted "
               "25 deg, K=200",
    "SILO": "silo stand-in: vertical cylinder wall (open below 4a) holding {n} polydisperse "
            "particles under gravity, discharging onto the floor, K=200",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="M2", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=120,
                    help="steps of the single-thread oracle on the same workload (M2 only)")
    ap.add_argument("--cpu-steps-all", type=int, default=200,
                    help="steps of the oracle on every host core (the CPU baseline, M2 only)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--sequential", action="store_true",
                    help="also run every system of the batch in its own context, in turn")
    ap.add_argument("--scale", type=float, default=1.0, help="lattice scale (1 = full size)")
    ap.add_argument("--friction", type=float, default=0.0, metavar="MU",
                    help="tangential friction with Coulomb coefficient MU (kt = kn/2, "
                         "gamma_t = gamma_n/2) on every system; 0: none")
    ap.add_argument("--call-steps", type=int, default=500,
                    help="steps per vb_run call (a call whose rows or cell bins overflow runs "
                         "again from its own start)")
    ap.add_argument("--tune", type=int, default=0, metavar="STEPS",
                    help="first choose the launch shape by measurement over STEPS untimed steps "
                         "(vb_tune); the timed runs use it, and the same runs with the fixed "
                         "default shape are timed beside them")
    ap.add_argument("--launch", default=None, metavar="U,X,T",
                    help="fixed launch shape for every run: gathers in flight per step-kernel "
                         "thread U (1, 2, 4, 8), tile order X (0 launch order, 1 contiguous per "
                         "XCD, 2 runs of 32 tiles per XCD), pair-search threads T (256, 384, 512); default: the library's")
    ap.add_argument("--repeats", type=int, default=100,
                    help="timed runs of the same steps without instrumentation, each from step 0 "
                         "(value is their mean; the plain baseline runs a tenth as many)")
    args = ap.parse_args()
    shape = tuple(int(t) for t in args.launch.split(",")) if args.launch else None
    if shape is not None and (len(shape) != 3 or args.tune > 0):
        ap.error("--launch takes U,X,T and excludes --tune")
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the method's "
              "hot path is measured on one GPU's share; multi-GPU sharding is a design "
              "note, not a measured path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2208_13770_amd as vb
    import synth
    from paper_2208_13770_amd import report

    t0 = time.perf_counter()
    systems = synth.config_systems(args.workload, seed=0, scale=args.scale,
                                   workers=min(16, os.cpu_count() or 1))
    if args.friction > 0.0:
        for s in systems:
            s.params.update(kt=0.5 * s.params["kn"], gamma_t=0.5 * s.params["gamma_n"],
                            mu=args.friction)
    n = sum(s.n for s in systems)
    log(f"{args.workload} input: {len(systems)} system(s), {n} particles generated in "
        f"{time.perf_counter() - t0:.1f}s")
    torch.cuda.init()
    copy_gbs = copy_bandwidth(torch)
    log(f"device copy bandwidth {copy_gbs:.0f} GB/s")

    # the throughput comes from runs without instrumentation (mean over the
    # repeats, each from step 0 of the loaded state); the kernel durations from
    # an identical run with HIP events on every kernel (the events cost a few
    # per cent of wall time)
    cs = args.call_steps
    tuned = tune_shape(vb, torch, systems, args.tune) if args.tune > 0 else None
    if tuned:
        log(f"tuned launch shape: {tuned}")
    walls, hist, _, info = run_mode(vb, torch, systems, args.steps, args.warmup, {}, False, cs,
                                    repeats=args.repeats, shape=shape)
    wall = float(np.mean(walls))
    value = n * args.steps / wall / 1e6
    walls_ev, hist_ev, pt, _ = run_mode(vb, torch, systems, args.steps, 0, {}, True, cs,
                                        shape=shape)
    wall_ev = walls_ev[0]
    assert np.array_equal(hist_ev["contacts"], hist["contacts"])
    rebuilt = hist["rebuilt"].astype(bool)            # [n_sys, steps]
    n_rebuild = int(rebuilt.sum())                     # broad phases over all systems
    any_rebuild = int(rebuilt.any(axis=0).sum())       # steps at which some system rebuilt
    pairs = hist["list_pairs"].sum(axis=0)             # per step, all systems
    step_ms = pt["ms_step"] / max(pt["steps"], 1)
    counts = {}
    for key, fixed in STEP_BYTES.items():
        b = float(np.mean(fixed * n + 2 * STEP_BYTES_PER_ENTRY * pairs))
        a = b / (step_ms * 1e-3) / 1e9
        counts[key] = {"bytes_per_particle": f"{fixed} + {STEP_BYTES_PER_ENTRY} n_v",
                       "bytes_per_launch": b, "achieved": a, "frac": a / HBM_PEAK_GBS}
    n_v = float(np.mean(2.0 * pairs / max(n, 1)))
    log(f"method K=200: {wall * 1e3:.1f} ms mean of {len(walls)} runs of {args.steps} steps, "
        f"{n_rebuild} broad phases ({any_rebuild} steps with one), step kernel "
        f"{step_ms * 1e3:.1f} us, broad-phase launches {pt['ms_rebuild']:.1f} ms total")

    plain = None
    if not args.no_plain:
        walls_p, hist_p, _, _ = run_mode(vb, torch, systems, args.steps, args.warmup,
                                         {"skin_mode": vb.VB_NO_BUFFER}, False, cs,
                                         repeats=max(1, args.repeats // 10), shape=shape)
        wall_p = float(np.mean(walls_p))
        _, _, pt_p, _ = run_mode(vb, torch, systems, args.steps, 0,
                                 {"skin_mode": vb.VB_NO_BUFFER}, True, cs, shape=shape)
        plain = {
            "time_s": wall_p,
            "runs": len(walls_p),
            "value": n * args.steps / wall_p / 1e6,
            "broad_phase_ms_total": pt_p["ms_rebuild"],
            "step_kernel_ms_total": pt_p["ms_step"],
            "improvement_pct": report.improvement(wall_p, wall),
            "speedup": wall_p / wall,
            "contacts_equal": bool(np.array_equal(hist_p["contacts"], hist["contacts"])),
        }
        log(f"plain (broad phase every step): {wall_p * 1e3:.1f} ms; Eq. impr "
            f"{plain['improvement_pct']:.1f} %")

    launch = {"shape": info["launch"], "tuned": tuned is not None}
    if tuned:  # the same runs with the fixed default shape
        walls_f, hist_f, _, info_f = run_mode(vb, torch, systems, args.steps, args.warmup, {}, False,
                                              cs, repeats=args.repeats,
                                              shape=default_shape(n, args.friction > 0.0))
        assert np.array_equal(hist_f, hist)
        launch.update(fixed_shape=info_f["launch"], fixed_ms_mean=float(np.mean(walls_f)) * 1e3,
                      tuned_ms_mean=wall * 1e3, tune_steps=args.tune,
                      speedup=float(np.mean(walls_f)) / wall)
        log(f"fixed shape {info_f['launch']}: {np.mean(walls_f) * 1e3:.1f} ms; tuned "
            f"{wall * 1e3:.1f} ms")

    sequential = None
    if args.sequential and len(systems) > 1:
        t_seq = 0.0
        for s in systems:
            w, _, _, _ = run_mode(vb, torch, [s], args.steps, 0, {}, False, cs)
            t_seq += w[0]
        sequential = {"time_s": t_seq, "value": n * args.steps / t_seq / 1e6,
                      "batch_speedup": t_seq / wall}
        log(f"one context per system, in turn: {t_seq * 1e3:.1f} ms "
            f"(batch {t_seq / wall:.2f}x faster)")

    cpu = None
    if args.workload == "M2" and args.friction == 0 and not args.no_cpu and args.cpu_steps > 0:
        # on the host's cores (os.cpu_count() is this host's share, capped at 16), and
        # on one thread; the same FP64 oracle as the tests use, untuned
        threads = min(16, os.cpu_count() or 1)
        v_all, dt_all = cpu_baseline(systems[0], args.cpu_steps_all, threads)
        v_one, dt_one = cpu_baseline(systems[0], args.cpu_steps, 1)
        cpu = {"value": v_all, "unit": "Mparticle*step/s", "cores": threads, "kind": "oracle",
               "sample": f"M2 workload ({n} particles), first {args.cpu_steps_all} steps, K=200, "
                         f"FP64 oracle on {threads} threads, {dt_all:.1f} s",
               "single_thread": {"value": v_one, "cores": 1,
                                 "sample": f"first {args.cpu_steps} steps, {dt_one:.1f} s"},
               "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}
        log(f"cpu oracle: {v_all:.3f} Mparticle*step/s on {threads} threads ({dt_all:.1f} s), "
            f"{v_one:.3f} on one ({dt_one:.1f} s)")

    traffic = (measured_traffic()
               if args.workload == "M2" and args.scale == 1.0 and args.friction == 0 else None)
    out = {
        "metric": "Mpixel·iter/s (% HBM peak) + time-to-1e-4 residual, plain vs batched+learned",
        "metric_note": "restated for the paper's DEM method: Mparticle*step/s (% HBM peak) of "
                       "the local Verlet buffer step; time-to-budget plain vs method",
        "value": value,
        "unit": "Mparticle*step/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].format(n=n) + (
                       f", tangential friction mu={args.friction:g}" if args.friction > 0 else ""),
                   "particles": n, "systems": len(systems), "steps": args.steps,
                   "steps_per_call": cs, "K": systems[0].params["K"]},
        "roofline": {"bound": "hbm", "achieved": counts["alg"]["achieved"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": counts["alg"]["frac"], "traffic": traffic,
                     "kernel": "k_step",
                     "bytes_note": "algorithmic bytes per launch over the kernel's mean launch "
                                   "duration; frac uses the scope table's count (84 + 4 n_v B "
                                   "per particle, FP32 state); byte_counts also gives the FP64 "
                                   "state's count and what the kernel's records move; traffic is "
                                   "the measured HBM bytes per launch (rocprofv3 counters), "
                                   "traffic_gbs the rate at which the kernel moves them, to "
                                   "set against copy_bandwidth_gbs",
                     "bytes_per_launch": counts["alg"]["bytes_per_launch"], "n_v": n_v,
                     "byte_counts": counts, "mean_launch_us": step_ms * 1e3,
                     "traffic_gbs": traffic / (step_ms * 1e-3) / 1e9 if traffic else None,
                     "copy_bandwidth_gbs": copy_gbs, "events_run_ms": wall_ev * 1e3},
        "repeats": {"n": len(walls), "ms_mean": float(np.mean(walls)) * 1e3,
                    "ms_std": float(np.std(walls, ddof=1)) * 1e3 if len(walls) > 1 else 0.0,
                    "ms_min": min(walls) * 1e3, "ms_max": max(walls) * 1e3},
        "launch": launch,
        "broad_phases": n_rebuild,
        "executed_broad_phase_pct": report.executed_fraction(n_rebuild, args.steps * len(systems)),
        "broad_phase_ms_total": pt["ms_rebuild"],
        "row_width": info["row_width"],
        "mean_list_pairs": float(pairs.mean()),
        "plain": plain,
        "sequential": sequential,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
